// One-wavefront complex FFT of length M = 64 R2 (R2 = 2, 4, 8, 16) for the
// z-transforms of the preconditioner (§4.2 eq. (38)).
//
// The index is split as n = n0 + 8 n1 + 64 n2 (n0, n1 < 8, n2 < R2) and the
// frequency as k = k2 + R2 k1 + 8 R2 k0, so that
//     w_M^{nk} = w_R2^{n2 k2} w_M^{(n0 + 8 n1) k2} w_8^{n1 k1} w_64^{n0 k1} w_8^{n0 k0}.
// Lane l = n0 + 8 n1 starts with z[l + 64 n2] in registers; the three DFT
// steps (over n2, n1, n0) run in registers, and the two regroupings between
// them go through the wave's own LDS slice.  No workgroup barrier is needed:
// only the wave touches its slice and a wave's LDS operations complete in
// issue order, so a compiler fence between a write and the read of another
// lane's slot is enough.
//
// LDS slots (complex units): after the first step value (l, k2) sits at
// l + 72 k2, after the second (n0, k1, k2) at n0 + 9 k1 + 72 k2; both
// paddings make the writes and the reads of a half-wave hit distinct banks.
#pragma once

#include "fft.h"

namespace axipcg {
namespace wfft {

__device__ inline void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// cos(2 pi t / 16); folds to a literal when t is a compile-time constant
__device__ inline double cos16(int t)
{
    switch (t & 15) {
    case 0: return 1.0;
    case 1: case 15: return 0.92387953251128675613;
    case 2: case 14: return 0.70710678118654752440;
    case 3: case 13: return 0.38268343236508977173;
    case 4: case 12: return 0.0;
    case 5: case 11: return -0.38268343236508977173;
    case 6: case 10: return -0.70710678118654752440;
    case 7: case 9: return -0.92387953251128675613;
    default: return -1.0;
    }
}

// d * exp(-2 pi i j / R), R <= 16; exact for the multiples of a quarter turn
template <typename T, int R>
__device__ inline cx<T> rot(cx<T> d, int j)
{
    const int t = (j * (16 / R)) & 15;   // angle in sixteenths of a turn
    if (t == 0) return d;
    if (t == 4) return {d.y, -d.x};
    if (t == 8) return {-d.x, -d.y};
    if (t == 12) return {-d.y, d.x};
    const T c = (T)cos16(t), s = -(T)cos16(t + 12);
    return {d.x * c - d.y * s, d.x * s + d.y * c};
}

// In-register DFT of length R (power of two <= 16), natural order in and out
// (decimation in frequency: halves, twiddle, two half-length DFTs).
template <typename T, int R>
struct Dft {
    __device__ static inline void run(cx<T> *v)
    {
        constexpr int H = R / 2;
        cx<T> b[H], c[H];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            b[j] = {v[j].x + v[j + H].x, v[j].y + v[j + H].y};
            c[j] = rot<T, R>({v[j].x - v[j + H].x, v[j].y - v[j + H].y}, j);
        }
        Dft<T, H>::run(b);
        Dft<T, H>::run(c);
#pragma unroll
        for (int k = 0; k < H; ++k) {
            v[2 * k] = b[k];
            v[2 * k + 1] = c[k];
        }
    }
};
template <typename T>
struct Dft<T, 1> {
    __device__ static inline void run(cx<T> *) {}
};

template <int R2>
struct Geo {
    static constexpr int M = 64 * R2;            // complex FFT length
    static constexpr int N = 2 * M;              // real transform length
    static constexpr int LB = 72 * R2;           // complex slots of a wave's LDS slice
    static constexpr int U = R2 >= 8 ? R2 / 8 : 1;   // units of steps 2 and 3 per lane
    static constexpr int UNITS = 8 * R2;
};

// Padded LDS slot of the complex value with natural index c (c < M): one
// gap of four slots per 32, so that rows of 64 lanes split into two
// conflict-free halves.
__device__ inline int vslot(int c) { return c + 4 * (c >> 5); }
// float slot of the real value with index s (< 2M) when the slice holds
// the sequence as complex pairs
__device__ inline int fslot(int s) { return 2 * vslot(s >> 1) + (s & 1); }

// Per-lane twiddles of the two twiddled steps, read once from the length-N
// table tw[e] = exp(-2 pi i e / N):  step 1 w_M^{l k2} = tw[2 l k2],
// step 2 w_64^{n0 k1} = tw[2 R2 n0 k1].
template <typename T, int R2>
struct Twiddles {
    cx<T> s1[R2];
    cx<T> s2[Geo<R2>::U][8];
    __device__ inline void load(const typename vec2_of<T>::type *__restrict__ tw, int lane)
    {
#pragma unroll
        for (int k2 = 1; k2 < R2; ++k2) s1[k2] = ld_tw<T>(tw, 2 * lane * k2);
#pragma unroll
        for (int j = 0; j < Geo<R2>::U; ++j) {
            const int u = lane + 64 * j;
            const int n0 = u & 7;
#pragma unroll
            for (int k1 = 1; k1 < 8; ++k1) s2[j][k1] = ld_tw<T>(tw, 2 * R2 * n0 * k1);
        }
    }
};

// Unit u of steps 2 and 3 exists when u < 8 R2 (all lanes for R2 >= 8).
template <int R2>
__device__ inline bool unit_active(int u) { return u < Geo<R2>::UNITS; }

// The FFT.  In: a[n2] = z[lane + 64 n2].  Out: for unit u = lane + 64 j
// (k1 = u & 7, k2 = u >> 3, when active) X[k2 + R2 k1 + 8 R2 k0] in
// out[j][k0].  buf: the wave's slice of Geo<R2>::LB complex slots, free on
// entry and on exit.
template <typename T, int R2>
__device__ inline void fft(cx<T> (&a)[R2], cx<T> (&out)[Geo<R2>::U][8], cx<T> *buf, const Twiddles<T, R2> &tw,
                           int lane)
{
    constexpr int U = Geo<R2>::U;
    Dft<T, R2>::run(a);
#pragma unroll
    for (int k2 = 1; k2 < R2; ++k2) a[k2] = cmul(a[k2], tw.s1[k2]);
    wave_fence();
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) buf[lane + 72 * k2] = a[k2];
    wave_fence();
    cx<T> b[U][8];
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const int u = lane + 64 * j;
        if (unit_active<R2>(u)) {
            const int n0 = u & 7, k2 = u >> 3;
#pragma unroll
            for (int n1 = 0; n1 < 8; ++n1) b[j][n1] = buf[n0 + 8 * n1 + 72 * k2];
        }
    }
    wave_fence();
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const int u = lane + 64 * j;
        if (unit_active<R2>(u)) {
            const int n0 = u & 7, k2 = u >> 3;
            Dft<T, 8>::run(b[j]);
#pragma unroll
            for (int k1 = 1; k1 < 8; ++k1) b[j][k1] = cmul(b[j][k1], tw.s2[j][k1]);
#pragma unroll
            for (int k1 = 0; k1 < 8; ++k1) buf[n0 + 9 * k1 + 72 * k2] = b[j][k1];
        }
    }
    wave_fence();
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const int u = lane + 64 * j;
        if (unit_active<R2>(u)) {
            const int k1 = u & 7, k2 = u >> 3;
#pragma unroll
            for (int n0 = 0; n0 < 8; ++n0) out[j][n0] = buf[n0 + 9 * k1 + 72 * k2];
        }
    }
    wave_fence();
#pragma unroll
    for (int j = 0; j < U; ++j)
        if (unit_active<R2>(lane + 64 * j)) Dft<T, 8>::run(out[j]);
}

// Natural frequency index of out[j][k0].
template <int R2>
__device__ inline int out_index(int lane, int j, int k0)
{
    const int u = lane + 64 * j;
    return (u >> 3) + R2 * (u & 7) + 8 * R2 * k0;
}

}  // namespace wfft
}  // namespace axipcg
