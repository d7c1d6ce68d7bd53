// Batched z-transforms of the preconditioner (§4.2 eq. (38)) on gfx950.
//
// One workgroup transforms one r-row of length N (a power of two).  The
// orthonormal sine (Dirichlet) / cosine (Neumann) transform of a real row is
// obtained from one complex FFT of length N of the even/odd reordered row
// (Makhoul's reordering):
//     v[n] = y[2n],  v[N-1-n] = y[2n+1],   y = x (cosine) or y_k = (-1)^k x_k (sine)
//     Y_m = Re(exp(-i pi m / 2N) V_m),     V = FFT_N(v)
// Y is the unnormalised DCT-II of y; the sine transform of x is Y read
// backwards (X_l = Y_{N-l}).  The inverse runs the same steps backwards:
//     V_m = exp(+i pi m / 2N) (Y_m - i Y_{N-m}),  v = Re IFFT_N(V).
// The complex FFT is a Stockham autosort radix-4 (plus one radix-2 pass for
// odd log2 N) ping-ponging between two LDS buffers; twiddles come from a
// table exp(-2 pi i k / N) computed once in FP64.
#pragma once

#include "common.h"

namespace axipcg {

template <typename T> struct cx { T x, y; };

template <typename T> struct vec2_of;
template <> struct vec2_of<float> { using type = float2; };
template <> struct vec2_of<double> { using type = double2; };

template <typename T>
__device__ inline cx<T> cmul(cx<T> a, cx<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

template <typename T>
__device__ inline cx<T> ld_tw(const typename vec2_of<T>::type *tw, int k)
{
    const auto t = tw[k];
    return {t.x, t.y};
}

// Forward complex FFT of length N (a power of two) held in `a`; `b` is scratch.
// Returns the buffer holding the result.  All threads of the block take part;
// the block must be synchronised on entry.
template <typename T>
__device__ cx<T> *fft_stockham_part(cx<T> *a, cx<T> *b, int N, const typename vec2_of<T>::type *__restrict__ tw,
                                    int tid, int nthr);

template <typename T>
__device__ cx<T> *fft_stockham(cx<T> *a, cx<T> *b, int N,
                               const typename vec2_of<T>::type *__restrict__ tw)
{
    return fft_stockham_part<T>(a, b, N, tw, threadIdx.x, blockDim.x);
}

// The same FFT run by `nthr` threads of the block (local index `tid`); the
// block's other threads may run other FFTs of the same length alongside, as
// every pass ends with a block-wide barrier.
template <typename T>
__device__ cx<T> *fft_stockham_part(cx<T> *a, cx<T> *b, int N, const typename vec2_of<T>::type *__restrict__ tw,
                                    int tid, int nthr)
{
    cx<T> *src = a, *dst = b;
    int Ns = 1;
    while ((Ns << 2) <= N) {
        const int Q = N >> 2;
        const int stride = N / (Ns << 2);
        for (int j = tid; j < Q; j += nthr) {
            const int jm = j & (Ns - 1);
            cx<T> v0 = src[j], v1 = src[j + Q], v2 = src[j + 2 * Q], v3 = src[j + 3 * Q];
            if (Ns > 1) {
                v1 = cmul(v1, ld_tw<T>(tw, jm * stride));
                v2 = cmul(v2, ld_tw<T>(tw, 2 * jm * stride));
                v3 = cmul(v3, ld_tw<T>(tw, 3 * jm * stride));
            }
            const cx<T> t0 = {v0.x + v2.x, v0.y + v2.y};
            const cx<T> t1 = {v0.x - v2.x, v0.y - v2.y};
            const cx<T> t2 = {v1.x + v3.x, v1.y + v3.y};
            const cx<T> t3 = {v1.y - v3.y, v3.x - v1.x};  // -i (v1 - v3)
            const int o = ((j - jm) << 2) + jm;
            dst[o] = {t0.x + t2.x, t0.y + t2.y};
            dst[o + Ns] = {t1.x + t3.x, t1.y + t3.y};
            dst[o + 2 * Ns] = {t0.x - t2.x, t0.y - t2.y};
            dst[o + 3 * Ns] = {t1.x - t3.x, t1.y - t3.y};
        }
        __syncthreads();
        cx<T> *t = src; src = dst; dst = t;
        Ns <<= 2;
    }
    if (Ns < N) {  // one radix-2 pass (odd log2 N)
        const int Q = N >> 1;
        const int stride = N / (Ns << 1);
        for (int j = tid; j < Q; j += nthr) {
            const int jm = j & (Ns - 1);
            cx<T> v0 = src[j], v1 = src[j + Q];
            if (Ns > 1) v1 = cmul(v1, ld_tw<T>(tw, jm * stride));
            const int o = ((j - jm) << 1) + jm;
            dst[o] = {v0.x + v1.x, v0.y + v1.y};
            dst[o + Ns] = {v0.x - v1.x, v0.y - v1.y};
        }
        __syncthreads();
        cx<T> *t = src; src = dst; dst = t;
    }
    return src;
}

// Threads per row for a transform of length N.
// Threads of a block-wide transform: N / 4 in [64, 256], and N / 8 above
// N = 2048 (each thread handles eight elements).
inline int fft_threads(int N)
{
    if (N > 2048) return N / 8;
    int t = N / 4;
    if (t < 64) t = 64;
    if (t > 256) t = 256;
    return t;
}

}  // namespace axipcg
