// Preconditioner B^{-1} of §4.2 (eqs. (36)-(39)) on gfx950: batched z-transforms
// in LDS and a partitioned r-tridiagonal solver with an in-wavefront reduced
// system.
#include "fft.h"
#include "kernels.h"
#include "wfft.h"
#include "wxform.h"

namespace axipcg {

namespace {



// Copy the length-N twiddle table into LDS (when it fits) so that the FFT
// passes read it without a trip to L2.
template <typename T>
__device__ inline const typename vec2_of<T>::type *stage_twiddles(const typename vec2_of<T>::type *tw,
                                                                  typename vec2_of<T>::type *lds, int N)
{
    // eight loads in flight per round (N <= 2048, >= 64 threads: at most four rounds)
    for (int base = 0; base < N; base += 8 * (int)blockDim.x) {
        typename vec2_of<T>::type v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = base + (int)threadIdx.x + j * (int)blockDim.x;
            if (k < N) v[j] = tw[k];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = base + (int)threadIdx.x + j * (int)blockDim.x;
            if (k < N) lds[k] = v[j];
        }
    }
    return lds;
}

// ---------------------------------------------------------------------------
// Forward transform: one workgroup per ROWS consecutive r-rows.  With two
// rows the second row's loads are issued before the first row's FFT, so the
// memory traffic of one row overlaps the LDS work of the other.
// ---------------------------------------------------------------------------
template <typename T, int BC, bool FUSED, bool TWLDS, int ROWS>
__device__ __forceinline__ void zfwd_body(const double *__restrict__ rin, double *__restrict__ x,
                                          double *__restrict__ r, const double *__restrict__ p,
                                          const double *__restrict__ q, PcgState *st,
                                          double *__restrict__ partials, int n_pq, T *__restrict__ spec,
                                          const typename vec2_of<T>::type *__restrict__ tw,
                                          const typename vec2_of<T>::type *__restrict__ pt, int nr, int N,
                                          int vb)
{
    using V2 = typename vec2_of<T>::type;
    extern __shared__ char smem_raw[];
    cx<T> *a = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *b = a + N;
    V2 *twl = reinterpret_cast<V2 *>(b + N);
    __shared__ double red[RED_SLOTS];

    if (st && st->done) return;
    const int i0 = xcd_swizzle(vb, nr / ROWS) * ROWS;
    constexpr int KPT = 8;   // elements per thread (fft_threads gives N <= 8 blockDim.x)
    double xv[KPT], rv0[KPT], pv[KPT], qv[KPT];
    auto load = [&](int i) {
        const size_t row = (size_t)i * N;
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
            const int k = threadIdx.x + j * blockDim.x;
            if (k < N) {
                if (FUSED) {
                    xv[j] = x[row + k];
                    rv0[j] = r[row + k];
                    pv[j] = p[row + k];
                    qv[j] = q[row + k];
                } else {
                    rv0[j] = rin[row + k];
                }
            }
        }
    };
    // issue the first row's loads before the p.q reduction so the latencies overlap
    load(i0);
    const V2 *twp = TWLDS ? stage_twiddles<T>(tw, twl, N) : tw;
    double alpha = 0.0;
    if (FUSED) {
        const double pq = block_total(partials + SLOT_PQ * MAX_PARTIALS, n_pq, red);
        const int k_it = st->iters;
        if (!(pq > 0.0) || !(pq < 1e308)) {
            if (vb == 0 && threadIdx.x == 0) st->done = ST_BREAK;
            return;
        }
        alpha = st->rho[k_it & 1] / pq;
        if (vb == 0 && threadIdx.x == 0) st->cur = k_it;
    }

    double rr = 0.0;
    const T nrm = (T)sqrt(2.0 / N);
    const T half = (T)0.70710678118654752440;
#pragma unroll
    for (int s = 0; s < ROWS; ++s) {
        const size_t row = (size_t)(i0 + s) * N;
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
            const int k = threadIdx.x + j * blockDim.x;
            if (k >= N) continue;
            double rv;
            if (FUSED) {
                const size_t c = row + k;
                x[c] = xv[j] + alpha * pv[j];
                rv = rv0[j] - alpha * qv[j];
                r[c] = rv;
                rr += rv * rv;
            } else {
                rv = rv0[j];
            }
            T v = (T)rv;
            int n;
            if ((k & 1) == 0) {
                n = k >> 1;
            } else {
                n = N - 1 - (k >> 1);
                if (BC == DIR) v = -v;
            }
            a[n] = {v, (T)0};
        }
        if (s + 1 < ROWS) load(i0 + s + 1);
        __syncthreads();
        const cx<T> *Vr = fft_stockham<T>(a, b, N, twp);
        for (int j = threadIdx.x; j < N; j += blockDim.x) {
            const int m = (BC == DIR) ? N - 1 - j : j;
            const cx<T> w = ld_tw<T>(pt, m);
            const T Y = Vr[m].x * w.x - Vr[m].y * w.y;
            const bool edge = (BC == DIR) ? (j == N - 1) : (j == 0);
            spec[row + j] = nrm * (edge ? half : (T)1) * Y;
        }
        if (s + 1 < ROWS) __syncthreads();   // the next row refills a and b
    }
    if (FUSED) {
        const double s = block_sum(rr, red);
        if (threadIdx.x == 0) partials[SLOT_RR * MAX_PARTIALS + vb] = s;
    }
}

// (512 threads for N = 4096, 256 or fewer below)
template <typename T, int BC, bool FUSED, bool TWLDS, int ROWS>
__global__ void __launch_bounds__(512)
k_zfwd(const double *__restrict__ rin, double *__restrict__ x, double *__restrict__ r,
       const double *__restrict__ p, const double *__restrict__ q, PcgState *st,
       double *__restrict__ partials, int n_pq,
       T *__restrict__ spec, const typename vec2_of<T>::type *__restrict__ tw,
       const typename vec2_of<T>::type *__restrict__ pt, int nr, int N)
{
    zfwd_body<T, BC, FUSED, TWLDS, ROWS>(rin, x, r, p, q, st, partials, n_pq, spec, tw, pt, nr, N, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Inverse transform: one workgroup per ROWS consecutive r-rows, FP64 output;
// the next row's spectral values are loaded during the current row's FFT.
// ---------------------------------------------------------------------------

template <typename T, int BC, int MODE, bool TWLDS, int ROWS>
__device__ __forceinline__ void zinv_body(const T *__restrict__ spec, double *__restrict__ zout,
                                          const double *__restrict__ r, const PcgState *st,
                                          double *__restrict__ partials, bool pr,
                                          const typename vec2_of<T>::type *__restrict__ tw,
                                          const typename vec2_of<T>::type *__restrict__ pt, int nr, int N, int vb,
                                          double *__restrict__ dinc = nullptr, double tau = 0.0, double rho2 = 0.0)
{
    constexpr bool PCGM = (MODE == 1 || MODE == 2);
    constexpr bool CHEB = (MODE == 3 || MODE == 4);
    using V2 = typename vec2_of<T>::type;
    if (MODE != 0 && st->done) return;
    extern __shared__ char smem_raw[];
    cx<T> *a = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *b = a + N;
    V2 *twl = reinterpret_cast<V2 *>(b + N);
    __shared__ double red[RED_SLOTS];
    const V2 *twp = TWLDS ? stage_twiddles<T>(tw, twl, N) : tw;

    const int i0 = xcd_swizzle(vb, nr / ROWS) * ROWS;
    const T isc = (T)sqrt(0.5 * N);      // 1 / sqrt(2/N)
    const T sq2 = (T)1.41421356237309504880;
    constexpr int KPT = 8;   // fft_threads gives N <= 8 blockDim.x
    T ymv[KPT], ynv[KPT];
    auto Yval = [&](size_t row, int m) -> T {
        // unnormalised DCT-II coefficient Y_m of y
        const int j = (BC == DIR) ? N - 1 - m : m;
        const bool edge = (BC == DIR) ? (j == N - 1) : (j == 0);
        return spec[row + j] * isc * (edge ? sq2 : (T)1);
    };
    auto load = [&](int i) {
        const size_t row = (size_t)i * N;
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
            const int m = threadIdx.x + j * blockDim.x;
            if (m < N) {
                ymv[j] = Yval(row, m);
                ynv[j] = (m == 0) ? (T)0 : Yval(row, N - m);
            }
        }
    };
    load(i0);
    const T invN = (T)1 / (T)N;
    double rz = 0.0, rzo = 0.0;
    double c1 = 0.0, c2 = 0.0;
    if (CHEB) {
        const double alpha = cheb_alpha(st->iters + 1, rho2);
        c1 = alpha - 1.0;
        c2 = alpha * tau;
    }
#pragma unroll
    for (int s = 0; s < ROWS; ++s) {
        const size_t row = (size_t)(i0 + s) * N;
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
            const int m = threadIdx.x + j * blockDim.x;
            if (m < N) {
                const cx<T> w = ld_tw<T>(pt, m);      // exp(-i pi m / 2N)
                // V = conj(w) (ym - i yn); store conj(V) = w (ym + i yn)
                a[m] = {w.x * ymv[j] - w.y * ynv[j], w.x * ynv[j] + w.y * ymv[j]};
            }
        }
        // r (and the old z) of this row, and the next row's spectral values,
        // are in flight during the FFT
        double rv[KPT], zo[KPT];
        if (PCGM) {
#pragma unroll
            for (int j = 0; j < KPT; ++j) {
                const int k = threadIdx.x + j * blockDim.x;
                if (k < N) {
                    rv[j] = r[row + k];
                    if (pr) zo[j] = zout[row + k];
                }
            }
        }
        if (s + 1 < ROWS) load(i0 + s + 1);
        __syncthreads();
        const cx<T> *res = fft_stockham<T>(a, b, N, twp);
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
            const int k = threadIdx.x + j * blockDim.x;
            if (k >= N) continue;
            const int n = (k & 1) ? N - 1 - (k >> 1) : (k >> 1);
            T v = res[n].x * invN;
            if (BC == DIR && (k & 1)) v = -v;
            const double zv = (double)v;
            if (PCGM) {
                if (pr) rzo += rv[j] * zo[j];
                rz += rv[j] * zv;
            }
            if (CHEB) {
                if (MODE == 4) dinc[row + k] = c2 * zv;
                else dinc[row + k] = c1 * dinc[row + k] + c2 * zv;
            } else {
                zout[row + k] = zv;
            }
        }
        if (s + 1 < ROWS) __syncthreads();   // the next row refills a and b
    }
    if (PCGM) {
        const double s = block_sum(rz, red);
        if (threadIdx.x == 0) partials[SLOT_RZ * MAX_PARTIALS + vb] = s;
        if (pr) {
            const double so = block_sum(rzo, red);
            if (threadIdx.x == 0) partials[SLOT_RZOLD * MAX_PARTIALS + vb] = so;
        }
    }
}

template <typename T, int BC, int MODE, bool TWLDS, int ROWS>
__global__ void __launch_bounds__(512)
k_zinv(const T *__restrict__ spec, double *__restrict__ zout, const double *__restrict__ r,
       const PcgState *st, double *__restrict__ partials, bool pr,
       const typename vec2_of<T>::type *__restrict__ tw,
       const typename vec2_of<T>::type *__restrict__ pt, int nr, int N, double *__restrict__ dinc, double tau,
       double rho2)
{
    zinv_body<T, BC, MODE, TWLDS, ROWS>(spec, zout, r, st, partials, pr, tw, pt, nr, N, blockIdx.x, dinc, tau, rho2);
}

template <typename T, int BC, bool FUSED, int R2>
__global__ void __launch_bounds__(256)
k_zfwd_w(const double *__restrict__ rin, double *__restrict__ x, double *__restrict__ r,
         const double *__restrict__ p, const double *__restrict__ q, PcgState *st,
         double *__restrict__ partials, int n_pq, T *__restrict__ spec,
         const typename vec2_of<T>::type *__restrict__ tw, const typename vec2_of<T>::type *__restrict__ pt,
         int nr)
{
    constexpr int WR = wave_rows<T, R2>();
    const int row = blockIdx.x * WR + (threadIdx.x >> 6);
    RowStore<T> out{spec + (size_t)(row < nr ? row : 0) * wfft::Geo<R2>::N};
    zfwd_w_body<T, BC, FUSED, R2>(rin, x, r, p, q, st, partials, n_pq, tw, pt, nr, row, blockIdx.x, out);
}

template <typename T, int BC, int MODE, int R2>
__global__ void __launch_bounds__(256)
k_zinv_w(const T *__restrict__ spec, double *__restrict__ zout, const double *__restrict__ r,
         const PcgState *st, double *__restrict__ partials, bool pr,
         const typename vec2_of<T>::type *__restrict__ tw, const typename vec2_of<T>::type *__restrict__ pt,
         int nr, double *__restrict__ dinc, double tau, double rho2)
{
    constexpr int WR = wave_rows<T, R2>();
    const int row = blockIdx.x * WR + (threadIdx.x >> 6);
    RowLoad<T> in{spec + (size_t)(row < nr ? row : nr - 1) * wfft::Geo<R2>::N};
    zinv_w_body<T, BC, MODE, R2>(in, zout, r, st, partials, pr, tw, pt, nr, dinc, tau, rho2, row, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Partitioned r-tridiagonal solve (one system per z-mode l):
//     -cb[i-1] y[i-1] + (db[i] + r_i lam_l) y[i] - cb[i] y[i+1] = f[i].
// A workgroup loads the [nr][M] tile of M consecutive modes into LDS; wave w
// solves mode l0 + w.  Lane s owns rows [lo_s, hi_s): its interior rows
// lo_s..hi_s-2 are eliminated locally against three right-hand sides (data and
// the two couplings to the neighbouring interface rows), which reduces the
// line to a tridiagonal system in the interface rows hi_s - 1, one per lane;
// that system is solved across the wavefront by parallel cyclic reduction
// with cross-lane shuffles, after which each lane back-substitutes.  This is
// the divide-and-conquer idea of §3 (split a tridiagonal system into
// independent subsystems by first computing values at the partition
// boundaries) mapped onto the lanes of one wavefront.
//
// In PCG mode the kernel first runs the stop test on ||r||^2 (partials of the
// preceding kernel), recorded by workgroup 0; every workgroup reaches the
// same decision.
// ---------------------------------------------------------------------------
// UNI: every active lane owns exactly LMAX rows (nr = S * LMAX), so the
// per-row loops carry no guards.
template <typename T, int LMAX, bool UNI>
__device__ __forceinline__ void tridiag_body(T *__restrict__ spec, const T *__restrict__ cb_g,
                                             const T *__restrict__ db_g, const T *__restrict__ rw_g,
                                             const T *__restrict__ lam, PcgState *st,
                                             const double *__restrict__ partials, const TriGate &g, int nr,
                                             int nz, int M, int S, int pitch, int Lp, int vb)
{
    __shared__ double red[8];
    extern __shared__ char smem_raw[];
    T *tile = reinterpret_cast<T *>(smem_raw);
    // r-line coefficients: each lane reads its own contiguous rows from global
    // memory (L2-resident, a few KB); staged in LDS they would be read at a
    // stride of a segment, one bank for the whole wave
    const T *__restrict__ cb = cb_g;
    const T *__restrict__ db = db_g;
    const T *__restrict__ rw = rw_g;
    const int ngroups = nz / M;
    const int l0 = xcd_swizzle(vb, ngroups) * M;
    // padded LDS row index (one gap per Lp rows); for UNI, Lp = LMAX, a power of
    // two, so the division is a shift
    auto prow = [&](int row) { return UNI ? row + row / LMAX : row + row / Lp; };

    if (M * sizeof(T) == 16) {
        // one 16-byte load per row
        for (int row = threadIdx.x; row < nr; row += blockDim.x) {
            const uint4 v = *reinterpret_cast<const uint4 *>(spec + (size_t)row * nz + l0);
            const T *tv = reinterpret_cast<const T *>(&v);
            for (int m = 0; m < M; ++m) tile[m * pitch + prow(row)] = tv[m];
        }
    } else {
        for (int e = threadIdx.x; e < nr * M; e += blockDim.x) {
            const int row = e / M, m = e - row * M;
            tile[m * pitch + prow(row)] = spec[(size_t)row * nz + l0 + m];
        }
    }
    if (g.mode != 0 && tridiag_gate(st, partials, g, red, vb) != ST_RUN) return;
    __syncthreads();

    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (w < M) {
        T *col = tile + w * pitch;
        const T lm = lam[l0 + w];
        const bool active = lane < S;
        const int lo = active ? (UNI ? lane * LMAX : (int)(((long)lane * nr) / S)) : 0;
        const int hi = active ? (UNI ? lo + LMAX : (int)(((long)(lane + 1) * nr) / S)) : 0;
        const int n = active ? hi - lo - 1 : 0;   // interior rows (>= 1 when active)
        auto in_seg = [&](int t) { return UNI ? (active && t < LMAX - 1) : (t < n); };

        // prefetch the lane's data (LDS), diagonal and couplings (global)
        T fv[LMAX], dv[LMAX], cv[LMAX];
        constexpr int VW = 16 / (int)sizeof(T);
        if constexpr (UNI && LMAX % VW == 0) {
            // all LMAX rows, the interface row included, as 16-byte vectors
            typedef T V __attribute__((ext_vector_type(VW)));
            if (active) {
#pragma unroll
                for (int j = 0; j < LMAX / VW; ++j) {
                    const V c4 = *reinterpret_cast<const V *>(cb + lo + j * VW);
                    const V d4 = *reinterpret_cast<const V *>(db + lo + j * VW);
                    const V r4 = *reinterpret_cast<const V *>(rw + lo + j * VW);
#pragma unroll
                    for (int e = 0; e < VW; ++e) {
                        cv[j * VW + e] = c4[e];
                        dv[j * VW + e] = d4[e] + r4[e] * lm;
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < LMAX; ++t)
                if (in_seg(t)) fv[t] = col[prow(lo + t)];
        } else {
#pragma unroll
            for (int t = 0; t < LMAX; ++t) {
                if (in_seg(t)) {
                    const int i = lo + t;
                    fv[t] = col[prow(i)];
                    dv[t] = db[i] + rw[i] * lm;
                    cv[t] = cb[i];
                }
            }
        }
        const T cbm = (active && lo > 0) ? cb[lo - 1] : (T)0;
        T cp[LMAX], gp[LMAX], vp[LMAX];
        T cprev = 0, gprev = 0, vprev = 0, inv = 1;
#pragma unroll
        for (int t = 0; t < LMAX; ++t) {
            if (in_seg(t)) {
                const T sub = (t > 0) ? -cv[t - 1] : (T)0;
                inv = fast_rcp<T>(dv[t] - sub * cprev);
                cprev = -cv[t] * inv;
                gprev = (fv[t] - sub * gprev) * inv;
                const T vr = (t == 0) ? cbm : (T)0;
                vprev = (vr - sub * vprev) * inv;
                cp[t] = cprev;
                gp[t] = gprev;
                vp[t] = vprev;
            }
        }
        const int R = hi - 1;                        // interface row of this lane
        const T cbR1 = active ? cb[R - 1] : (T)0;    // coupling interface <- last interior
        const T wl = cbR1 * inv;                     // w' of the last interior row
        T gl = active ? gprev : (T)0, vl = active ? vprev : (T)0;
        // back-substitute to obtain the first interior values of g, v, w
        T gq = gl, v = vl, ww = wl;
#pragma unroll
        for (int t = LMAX - 2; t >= 0; --t) {
            if (UNI ? (t < LMAX - 2 + 0 && active) : (t < n - 1)) {
                gq = gp[t] - cp[t] * gq;
                v = vp[t] - cp[t] * v;
                ww = -cp[t] * ww;
            }
        }
        if (!active) { gq = 0; v = 0; ww = 0; }
        // neighbour (lane + 1) first values
        const T gfn = __shfl_down(gq, 1, 64);
        const T vfn = __shfl_down(v, 1, 64);
        const T wfn = __shfl_down(ww, 1, 64);
        const bool has_right = active && (lane + 1 < S);
        const T cbR = has_right ? cb[R] : (T)0;
        T ra = 0, rb = 1, rc = 0, re = 0;
        if (active) {
            ra = -cbR1 * vl;
            rb = db[R] + rw[R] * lm - cbR1 * wl - (has_right ? cbR * vfn : (T)0);
            rc = has_right ? -cbR * wfn : (T)0;
            re = col[prow(R)] + cbR1 * gl + (has_right ? cbR * gfn : (T)0);
        }
        // parallel cyclic reduction over the S interface unknowns
        for (int k = 1; k < S; k <<= 1) {
            const T am = __shfl_up(ra, k, 64), bm = __shfl_up(rb, k, 64);
            const T cm = __shfl_up(rc, k, 64), em = __shfl_up(re, k, 64);
            const T ap = __shfl_down(ra, k, 64), bp = __shfl_down(rb, k, 64);
            const T cq = __shfl_down(rc, k, 64), ep = __shfl_down(re, k, 64);
            const bool hm = lane >= k, hp = lane + k < S;
            const T al = hm ? -ra * fast_rcp<T>(bm) : (T)0;
            const T ga = hp ? -rc * fast_rcp<T>(bp) : (T)0;
            const T na = hm ? al * am : (T)0;
            const T nc = hp ? ga * cq : (T)0;
            const T nb = rb + (hm ? al * cm : (T)0) + (hp ? ga * ap : (T)0);
            const T ne = re + (hm ? al * em : (T)0) + (hp ? ga * ep : (T)0);
            if (active) { ra = na; rb = nb; rc = nc; re = ne; }
        }
        const T xs = active ? re / rb : (T)0;
        T xm = __shfl_up(xs, 1, 64);
        if (lane == 0) xm = 0;
        // interior values: forward-eliminated rhs y' = g' + v' x_{s-1} (+ w' x_s
        // on the last interior row), then the backward sweep
        if (active) {
            T y = 0;
#pragma unroll
            for (int t = LMAX - 1; t >= 0; --t) {
                if (in_seg(t)) {
                    const T yp = gp[t] + vp[t] * xm;
                    if (t == n - 1) y = yp + wl * xs;
                    else y = yp - cp[t] * y;
                    col[prow(lo + t)] = y;
                }
            }
            col[prow(R)] = xs;
        }
    }
    __syncthreads();
    if (M * sizeof(T) == 16) {
        for (int row = threadIdx.x; row < nr; row += blockDim.x) {
            uint4 v;
            T *tv = reinterpret_cast<T *>(&v);
            for (int m = 0; m < M; ++m) tv[m] = tile[m * pitch + prow(row)];
            *reinterpret_cast<uint4 *>(spec + (size_t)row * nz + l0) = v;
        }
    } else {
        for (int e = threadIdx.x; e < nr * M; e += blockDim.x) {
            const int row = e / M, m = e - row * M;
            spec[(size_t)row * nz + l0 + m] = tile[m * pitch + prow(row)];
        }
    }
}

template <typename T, int LMAX, bool UNI>
__global__ void __launch_bounds__(256)
k_tridiag(T *__restrict__ spec, const T *__restrict__ cb_g, const T *__restrict__ db_g,
          const T *__restrict__ rw_g, const T *__restrict__ lam, PcgState *st,
          const double *__restrict__ partials, TriGate g, int nr, int nz, int M, int S, int pitch, int Lp)
{
    tridiag_body<T, LMAX, UNI>(spec, cb_g, db_g, rw_g, lam, st, partials, g, nr, nz, M, S, pitch, Lp, blockIdx.x);
}

// ---- batched launches ----------------------------------------------------
template <typename T> __device__ inline const T *pd_cb(const ProbDesc &P);
template <> __device__ inline const float *pd_cb<float>(const ProbDesc &P) { return P.cb32; }
template <> __device__ inline const double *pd_cb<double>(const ProbDesc &P) { return P.cb64; }
template <typename T> __device__ inline const T *pd_db(const ProbDesc &P);
template <> __device__ inline const float *pd_db<float>(const ProbDesc &P) { return P.db32; }
template <> __device__ inline const double *pd_db<double>(const ProbDesc &P) { return P.db64; }
template <typename T> __device__ inline const T *pd_rw(const ProbDesc &P);
template <> __device__ inline const float *pd_rw<float>(const ProbDesc &P) { return P.rw32; }
template <> __device__ inline const double *pd_rw<double>(const ProbDesc &P) { return P.rw64; }
template <typename T> __device__ inline const T *pd_lam(const ProbDesc &P);
template <> __device__ inline const float *pd_lam<float>(const ProbDesc &P) { return P.lam32; }
template <> __device__ inline const double *pd_lam<double>(const ProbDesc &P) { return P.lam64; }
template <typename T> __device__ inline const typename vec2_of<T>::type *pd_tw(const ProbDesc &P);
template <> __device__ inline const float2 *pd_tw<float>(const ProbDesc &P) { return P.tw32; }
template <> __device__ inline const double2 *pd_tw<double>(const ProbDesc &P) { return P.tw64; }
template <typename T> __device__ inline const typename vec2_of<T>::type *pd_pt(const ProbDesc &P);
template <> __device__ inline const float2 *pd_pt<float>(const ProbDesc &P) { return P.pt32; }
template <> __device__ inline const double2 *pd_pt<double>(const ProbDesc &P) { return P.pt64; }

// The batched transforms run one launch per transform plan; `d` holds the
// problems of that plan, with tr_start counted within the launch.
template <typename T, bool FUSED, bool TWLDS>
__global__ void __launch_bounds__(256) k_b_zfwd(const ProbDesc *__restrict__ d, int n, int parity)
{
    const int p = find_problem(d, n, blockIdx.x, RANGE_TR);
    const ProbDesc &P = d[p];
    const double *pnew = parity ? P.p0 : P.p1;   // written by this iteration's SpMV
    const int vb = blockIdx.x - P.tr_start;
    // the start-up transform runs before the r-solve launch resets the state,
    // so only the in-loop (fused) transform may read the stop flag
    PcgState *st = FUSED ? P.state : nullptr;
    if (P.bc_z == DIR)
        zfwd_body<T, DIR, FUSED, TWLDS, 1>(P.r, P.x, P.r, pnew, P.q, st, P.partials, P.nr, (T *)P.spec,
                                        pd_tw<T>(P), pd_pt<T>(P), P.nr, P.nz, vb);
    else
        zfwd_body<T, AXIPCG_Z_NEUMANN, FUSED, TWLDS, 1>(P.r, P.x, P.r, pnew, P.q, st, P.partials, P.nr,
                                                     (T *)P.spec, pd_tw<T>(P), pd_pt<T>(P), P.nr, P.nz, vb);
}

template <typename T, int MODE, bool TWLDS>
__global__ void __launch_bounds__(256) k_b_zinv(const ProbDesc *__restrict__ d, int n, bool pr)
{
    const int p = find_problem(d, n, blockIdx.x, RANGE_TR);
    const ProbDesc &P = d[p];
    const int vb = blockIdx.x - P.tr_start;
    if (P.bc_z == DIR)
        zinv_body<T, DIR, MODE, TWLDS, 1>((const T *)P.spec, P.z, P.r, P.state, P.partials, pr, pd_tw<T>(P),
                                       pd_pt<T>(P), P.nr, P.nz, vb);
    else
        zinv_body<T, AXIPCG_Z_NEUMANN, MODE, TWLDS, 1>((const T *)P.spec, P.z, P.r, P.state, P.partials, pr,
                                                    pd_tw<T>(P), pd_pt<T>(P), P.nr, P.nz, vb);
}

template <typename T, bool FUSED, int R2>
__global__ void __launch_bounds__(256) k_b_zfwd_w(const ProbDesc *__restrict__ d, int n, int parity)
{
    const int p = find_problem(d, n, blockIdx.x, RANGE_TR);
    const ProbDesc &P = d[p];
    const double *pnew = parity ? P.p0 : P.p1;
    const int vb = blockIdx.x - P.tr_start;
    PcgState *st = FUSED ? P.state : nullptr;   // as in k_b_zfwd
    constexpr int WR = wave_rows<T, R2>();
    const int row = vb * WR + (threadIdx.x >> 6);
    RowStore<T> out{(T *)P.spec + (size_t)(row < P.nr ? row : 0) * wfft::Geo<R2>::N};
    if (P.bc_z == DIR)
        zfwd_w_body<T, DIR, FUSED, R2>(P.r, P.x, P.r, pnew, P.q, st, P.partials, P.nr, pd_tw<T>(P), pd_pt<T>(P),
                                       P.nr, row, vb, out);
    else
        zfwd_w_body<T, AXIPCG_Z_NEUMANN, FUSED, R2>(P.r, P.x, P.r, pnew, P.q, st, P.partials, P.nr, pd_tw<T>(P),
                                                    pd_pt<T>(P), P.nr, row, vb, out);
}

template <typename T, int MODE, int R2>
__global__ void __launch_bounds__(256) k_b_zinv_w(const ProbDesc *__restrict__ d, int n, bool pr)
{
    const int p = find_problem(d, n, blockIdx.x, RANGE_TR);
    const ProbDesc &P = d[p];
    const int vb = blockIdx.x - P.tr_start;
    constexpr int WR = wave_rows<T, R2>();
    const int row = vb * WR + (threadIdx.x >> 6);
    RowLoad<T> in{(const T *)P.spec + (size_t)(row < P.nr ? row : P.nr - 1) * wfft::Geo<R2>::N};
    if (P.bc_z == DIR)
        zinv_w_body<T, DIR, MODE, R2>(in, P.z, P.r, P.state, P.partials, pr, pd_tw<T>(P), pd_pt<T>(P), P.nr, nullptr,
                                      0.0, 0.0, row, vb);
    else
        zinv_w_body<T, AXIPCG_Z_NEUMANN, MODE, R2>(in, P.z, P.r, P.state, P.partials, pr, pd_tw<T>(P), pd_pt<T>(P),
                                                   P.nr, nullptr, 0.0, 0.0, row, vb);
}

template <typename T>
__global__ void __launch_bounds__(256) k_b_tridiag(const ProbDesc *__restrict__ d, int n, TriGate g, int M)
{
    const int p = find_problem(d, n, blockIdx.x, RANGE_TRI);
    const ProbDesc &P = d[p];
    const int vb = blockIdx.x - P.tri_start;
    g.state = P.state;
    g.n_rr = g.mode == 2 ? P.nr : P.n_tr;   // start: the init partials, one per row
    const bool uni = (P.nr % P.tri_S) == 0;
#define AXI_BTRI(LM, U)                                                                                       \
    tridiag_body<T, LM, U>((T *)P.spec, pd_cb<T>(P), pd_db<T>(P), pd_rw<T>(P), pd_lam<T>(P), P.state,           \
                           P.partials, g, P.nr, P.nz, M, P.tri_S, P.tri_pitch, P.tri_Lp, vb)
    if (uni && P.tri_L == 2) AXI_BTRI(2, true);
    else if (uni && P.tri_L == 4) AXI_BTRI(4, true);
    else if (uni && P.tri_L == 8) AXI_BTRI(8, true);
    else if (uni && P.tri_L == 16) AXI_BTRI(16, true);
    else if (P.tri_L <= 4) AXI_BTRI(4, false);
    else if (P.tri_L <= 8) AXI_BTRI(8, false);
    else AXI_BTRI(16, false);
#undef AXI_BTRI
}

template <typename T>
struct Tables {
    const typename vec2_of<T>::type *tw, *pt;
    const T *cb, *db, *rw, *lam;
};
template <typename T> Tables<T> tables(const Operator &op);
template <> Tables<float> tables<float>(const Operator &op)
{
    return {op.tw32, op.pt32, op.cb32, op.db32, op.rw32, op.lam32};
}
template <> Tables<double> tables<double>(const Operator &op)
{
    return {op.tw64, op.pt64, op.cb64, op.db64, op.rw64, op.lam64};
}

// LDS of a transform workgroup: two data buffers, plus the twiddle table when
// the total stays within 64 KiB.
template <typename T>
bool twiddles_in_lds(int N) { return 3 * (size_t)N * sizeof(cx<T>) <= 65536; }
template <typename T>
size_t transform_lds(int N) { return (twiddles_in_lds<T>(N) ? 3 : 2) * (size_t)N * sizeof(cx<T>); }

// Rows per transform workgroup: two (pipelined) for the FP64 transforms when
// that still leaves at least 256 workgroups, else one.  (Measured at 1024^2:
// two rows take the FP64 forward transform from 28 to 25 us but slow the FP32
// ones, whose FFT is too short to hide a second row's loads behind while the
// grid loses half its workgroups.)
inline int transform_rows(int nr, int prec)
{
    return (prec == AXIPCG_PREC_FP64 && nr % 2 == 0 && nr >= 512) ? 2 : 1;
}

// Dynamic LDS above the default 64 KiB (FP64 rows of 4096) needs the
// kernel's attribute, set once per kernel.
inline void allow_transform_lds(const void *fn, size_t bytes, bool &done)
{
    if (done || bytes <= 65536) return;
    AXI_CHECK_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    done = true;
}

template <typename T, int BC, bool TWL, int ROWS>
void zfwd_ttr(const Operator &op, const ZfwdArgs &a, hipStream_t s)
{
    const int N = op.nz;
    const auto tb = tables<T>(op);
    const size_t shm = transform_lds<T>(N);
    const int thr = fft_threads(N);
    const dim3 grid(op.nr / ROWS);
    static bool lds_set[2] = {false, false};
    allow_transform_lds(reinterpret_cast<const void *>(&k_zfwd<T, BC, true, TWL, ROWS>), shm, lds_set[0]);
    allow_transform_lds(reinterpret_cast<const void *>(&k_zfwd<T, BC, false, TWL, ROWS>), shm, lds_set[1]);
    if (a.fused)
        hipLaunchKernelGGL((k_zfwd<T, BC, true, TWL, ROWS>), grid, dim3(thr), shm, s, nullptr, a.x, a.r, a.p, a.q,
                           a.state, op.partials, a.n_pq, (T *)op.spec, tb.tw, tb.pt, op.nr, N);
    else
        hipLaunchKernelGGL((k_zfwd<T, BC, false, TWL, ROWS>), grid, dim3(thr), shm, s, a.rin, nullptr, nullptr,
                           nullptr, nullptr, a.state, op.partials, 0, (T *)op.spec, tb.tw, tb.pt, op.nr, N);
    AXI_CHECK_HIP(hipGetLastError());
}

// Rows per workgroup of the one-wave transforms for length N, 0 when N has
// no one-wave plan (then the block-wide Stockham kernels run).
template <typename T>
int wave_plan_rows(int N)
{
    switch (N) {
    case 256: return wave_rows<T, 2>();
    case 512: return wave_rows<T, 4>();
    case 1024: return wave_rows<T, 8>();
    case 2048: return sizeof(T) == 4 ? wave_rows<T, 16>() : 0;   // FP64 at 2048 would spill
    default: return 0;
    }
}

template <typename T, int BC, int R2>
void zfwd_wave(const Operator &op, const ZfwdArgs &a, hipStream_t s)
{
    constexpr int WR = wave_rows<T, R2>();
    const auto tb = tables<T>(op);
    const dim3 grid((op.nr + WR - 1) / WR), block(64 * WR);
    const size_t shm = (size_t)WR * wfft::Geo<R2>::LB * sizeof(cx<T>);
    if (a.fused)
        hipLaunchKernelGGL((k_zfwd_w<T, BC, true, R2>), grid, block, shm, s, nullptr, a.x, a.r, a.p, a.q, a.state,
                           op.partials, a.n_pq, (T *)op.spec, tb.tw, tb.pt, op.nr);
    else
        hipLaunchKernelGGL((k_zfwd_w<T, BC, false, R2>), grid, block, shm, s, a.rin, nullptr, nullptr, nullptr,
                           nullptr, a.state, op.partials, 0, (T *)op.spec, tb.tw, tb.pt, op.nr);
    AXI_CHECK_HIP(hipGetLastError());
}

template <typename T, int BC>
void zfwd_t(const Operator &op, const ZfwdArgs &a, hipStream_t s)
{
    switch (op.nz) {
    case 256: return zfwd_wave<T, BC, 2>(op, a, s);
    case 512: return zfwd_wave<T, BC, 4>(op, a, s);
    case 1024: return zfwd_wave<T, BC, 8>(op, a, s);
    case 2048:
        if constexpr (sizeof(T) == 4) return zfwd_wave<T, BC, 16>(op, a, s);
        break;
    default: break;
    }
    const bool twl = twiddles_in_lds<T>(op.nz);
    if (transform_rows(op.nr, sizeof(T) == 8 ? AXIPCG_PREC_FP64 : AXIPCG_PREC_FP32) == 2) {
        if (twl) zfwd_ttr<T, BC, true, 2>(op, a, s);
        else zfwd_ttr<T, BC, false, 2>(op, a, s);
    } else {
        if (twl) zfwd_ttr<T, BC, true, 1>(op, a, s);
        else zfwd_ttr<T, BC, false, 1>(op, a, s);
    }
}

template <typename T, int BC, bool TWL, int ROWS>
void zinv_ttr(const Operator &op, const ZinvArgs &a, hipStream_t s)
{
    const int N = op.nz;
    const auto tb = tables<T>(op);
    const size_t shm = transform_lds<T>(N);
    const int thr = fft_threads(N);
    const dim3 grid(op.nr / ROWS);
    static bool lds_set[5] = {false, false, false, false, false};
    allow_transform_lds(reinterpret_cast<const void *>(&k_zinv<T, BC, 0, TWL, ROWS>), shm, lds_set[0]);
    allow_transform_lds(reinterpret_cast<const void *>(&k_zinv<T, BC, 1, TWL, ROWS>), shm, lds_set[1]);
    allow_transform_lds(reinterpret_cast<const void *>(&k_zinv<T, BC, 2, TWL, ROWS>), shm, lds_set[2]);
    allow_transform_lds(reinterpret_cast<const void *>(&k_zinv<T, BC, 3, TWL, ROWS>), shm, lds_set[3]);
    allow_transform_lds(reinterpret_cast<const void *>(&k_zinv<T, BC, 4, TWL, ROWS>), shm, lds_set[4]);
    switch (a.mode) {
    case 0:
        hipLaunchKernelGGL((k_zinv<T, BC, 0, TWL, ROWS>), grid, dim3(thr), shm, s, (const T *)op.spec, a.zout,
                           nullptr, nullptr, op.partials, false, tb.tw, tb.pt, op.nr, N, nullptr, 0.0, 0.0);
        break;
    case 1:
        hipLaunchKernelGGL((k_zinv<T, BC, 1, TWL, ROWS>), grid, dim3(thr), shm, s, (const T *)op.spec, a.zout,
                           a.r, a.state, op.partials, a.pr, tb.tw, tb.pt, op.nr, N, nullptr, 0.0, 0.0);
        break;
    case 2:
        hipLaunchKernelGGL((k_zinv<T, BC, 2, TWL, ROWS>), grid, dim3(thr), shm, s, (const T *)op.spec, a.zout,
                           a.r, a.state, op.partials, false, tb.tw, tb.pt, op.nr, N, nullptr, 0.0, 0.0);
        break;
    case 3:
        hipLaunchKernelGGL((k_zinv<T, BC, 3, TWL, ROWS>), grid, dim3(thr), shm, s, (const T *)op.spec, nullptr,
                           nullptr, a.state, op.partials, false, tb.tw, tb.pt, op.nr, N, a.d, a.tau, a.rho2);
        break;
    default:
        hipLaunchKernelGGL((k_zinv<T, BC, 4, TWL, ROWS>), grid, dim3(thr), shm, s, (const T *)op.spec, nullptr,
                           nullptr, a.state, op.partials, false, tb.tw, tb.pt, op.nr, N, a.d, a.tau, a.rho2);
        break;
    }
    AXI_CHECK_HIP(hipGetLastError());
}

template <typename T, int BC, int R2>
void zinv_wave(const Operator &op, const ZinvArgs &a, hipStream_t s)
{
    constexpr int WR = wave_rows<T, R2>();
    const auto tb = tables<T>(op);
    const dim3 grid((op.nr + WR - 1) / WR), block(64 * WR);
    const size_t shm = (size_t)WR * wfft::Geo<R2>::LB * sizeof(cx<T>);
    const T *spec = (const T *)op.spec;
    switch (a.mode) {
    case 0:
        hipLaunchKernelGGL((k_zinv_w<T, BC, 0, R2>), grid, block, shm, s, spec, a.zout, nullptr, nullptr,
                           op.partials, false, tb.tw, tb.pt, op.nr, nullptr, 0.0, 0.0);
        break;
    case 1:
        hipLaunchKernelGGL((k_zinv_w<T, BC, 1, R2>), grid, block, shm, s, spec, a.zout, a.r, a.state, op.partials,
                           a.pr, tb.tw, tb.pt, op.nr, nullptr, 0.0, 0.0);
        break;
    case 2:
        hipLaunchKernelGGL((k_zinv_w<T, BC, 2, R2>), grid, block, shm, s, spec, a.zout, a.r, a.state, op.partials,
                           false, tb.tw, tb.pt, op.nr, nullptr, 0.0, 0.0);
        break;
    case 3:
        hipLaunchKernelGGL((k_zinv_w<T, BC, 3, R2>), grid, block, shm, s, spec, nullptr, nullptr, a.state,
                           op.partials, false, tb.tw, tb.pt, op.nr, a.d, a.tau, a.rho2);
        break;
    default:
        hipLaunchKernelGGL((k_zinv_w<T, BC, 4, R2>), grid, block, shm, s, spec, nullptr, nullptr, a.state,
                           op.partials, false, tb.tw, tb.pt, op.nr, a.d, a.tau, a.rho2);
        break;
    }
    AXI_CHECK_HIP(hipGetLastError());
}

template <typename T, int BC>
void zinv_t(const Operator &op, const ZinvArgs &a, hipStream_t s)
{
    switch (op.nz) {
    case 256: return zinv_wave<T, BC, 2>(op, a, s);
    case 512: return zinv_wave<T, BC, 4>(op, a, s);
    case 1024: return zinv_wave<T, BC, 8>(op, a, s);
    case 2048:
        if constexpr (sizeof(T) == 4) return zinv_wave<T, BC, 16>(op, a, s);
        break;
    default: break;
    }
    const bool twl = twiddles_in_lds<T>(op.nz);
    if (transform_rows(op.nr, sizeof(T) == 8 ? AXIPCG_PREC_FP64 : AXIPCG_PREC_FP32) == 2) {
        if (twl) zinv_ttr<T, BC, true, 2>(op, a, s);
        else zinv_ttr<T, BC, false, 2>(op, a, s);
    } else {
        if (twl) zinv_ttr<T, BC, true, 1>(op, a, s);
        else zinv_ttr<T, BC, false, 1>(op, a, s);
    }
}

struct TriGeom {
    int M, S, L, Lp, pitch;
    size_t shm;
};

template <typename T>
TriGeom tri_geom(int nr, int nz)
{
    TriGeom g;
    g.S = nr / 2 < 64 ? nr / 2 : 64;
    g.L = (nr + g.S - 1) / g.S;
    g.Lp = nr / g.S;
    g.pitch = nr + nr / g.Lp + 1;
    g.M = 16 / (int)sizeof(T);   // one 16-byte vector of modes per row
    auto lds = [&](int M) { return (size_t)M * g.pitch * sizeof(T); };
    while (g.M > 1 && (lds(g.M) > 65536 || nz % g.M != 0)) g.M >>= 1;
    g.shm = lds(g.M);
    return g;
}

template <typename T>
void tridiag_t(const Operator &op, const TriGate &gate, hipStream_t s)
{
    const TriGeom g = tri_geom<T>(op.nr, op.nz);
    const auto tb = tables<T>(op);
    const dim3 grid(op.nz / g.M), block(64 * g.M);
    T *spec = (T *)op.spec;
#define AXI_TRI(LM, U)                                                                                   \
    hipLaunchKernelGGL((k_tridiag<T, LM, U>), grid, block, g.shm, s, spec, tb.cb, tb.db, tb.rw, tb.lam,  \
                       gate.state, op.partials, gate, op.nr, op.nz, g.M, g.S, g.pitch, g.Lp)
    const bool uni = (op.nr % g.S) == 0;
    if (uni && g.L == 2) AXI_TRI(2, true);
    else if (uni && g.L == 4) AXI_TRI(4, true);
    else if (uni && g.L == 8) AXI_TRI(8, true);
    else if (uni && g.L == 16) AXI_TRI(16, true);
    else if (uni && g.L == 32) AXI_TRI(32, true);
    else if (g.L <= 4) AXI_TRI(4, false);
    else if (g.L <= 8) AXI_TRI(8, false);
    else if (g.L <= 16) AXI_TRI(16, false);
    else if (g.L <= 32) AXI_TRI(32, false);
    else if (g.L <= 64) AXI_TRI(64, false);
    else throw Error{AXIPCG_EINVAL, "nr too large for the r-solver"};
#undef AXI_TRI
    AXI_CHECK_HIP(hipGetLastError());
}

}  // namespace

// Strip height of the solves' launches: the handle's, except that 8-row
// strips at FP32 rows of 2048 (whose PCG-form kernels would spill registers
// in 8-wave workgroups) run as 4-row strips.
int strip_solve_rows(const Operator &op, int prec)
{
    return (op.strip_rows == 8 && prec == AXIPCG_PREC_FP32 && op.nz == 2048) ? 4 : op.strip_rows;
}

int transform_blocks(const Operator &op, int prec)
{
    if (strip_usable(op, prec, strip_solve_rows(op, prec))) return op.nr / strip_solve_rows(op, prec);
    const int wr = (prec == AXIPCG_PREC_FP32) ? wave_plan_rows<float>(op.nz) : wave_plan_rows<double>(op.nz);
    if (wr > 0) return (op.nr + wr - 1) / wr;
    return op.nr / transform_rows(op.nr, prec);
}

// ---- batched launchers -------------------------------------------------------
void batch_tri_geom(int nr, int prec, int M, int *S, int *L, int *Lp, int *pitch, size_t *shm)
{
    *S = nr / 2 < 64 ? nr / 2 : 64;
    *L = (nr + *S - 1) / *S;
    *Lp = nr / *S;
    *pitch = nr + nr / *Lp + 1;
    const size_t el = (prec == AXIPCG_PREC_FP32) ? sizeof(float) : sizeof(double);
    *shm = (size_t)M * *pitch * el;
}

int batch_transform_plan(int nz, int prec, int *rows_per_wg)
{
    const int wr = (prec == AXIPCG_PREC_FP32) ? wave_plan_rows<float>(nz) : wave_plan_rows<double>(nz);
    *rows_per_wg = wr > 0 ? wr : 1;
    return wr > 0 ? nz / 128 : 0;
}

template <typename T, int R2>
void b_zfwd_wave(const ProbDesc *d, const BatchPlan &pl, bool fused, int parity, hipStream_t s)
{
    constexpr int WR = wave_rows<T, R2>();
    const size_t shm = (size_t)WR * wfft::Geo<R2>::LB * sizeof(cx<T>);
    if (fused)
        hipLaunchKernelGGL((k_b_zfwd_w<T, true, R2>), dim3(pl.blocks), dim3(64 * WR), shm, s, d + pl.off, pl.n,
                           parity);
    else
        hipLaunchKernelGGL((k_b_zfwd_w<T, false, R2>), dim3(pl.blocks), dim3(64 * WR), shm, s, d + pl.off, pl.n,
                           parity);
}

template <typename T, int R2>
void b_zinv_wave(const ProbDesc *d, const BatchPlan &pl, int mode, bool pr, hipStream_t s)
{
    constexpr int WR = wave_rows<T, R2>();
    const size_t shm = (size_t)WR * wfft::Geo<R2>::LB * sizeof(cx<T>);
    if (mode == 1)
        hipLaunchKernelGGL((k_b_zinv_w<T, 1, R2>), dim3(pl.blocks), dim3(64 * WR), shm, s, d + pl.off, pl.n, pr);
    else
        hipLaunchKernelGGL((k_b_zinv_w<T, 2, R2>), dim3(pl.blocks), dim3(64 * WR), shm, s, d + pl.off, pl.n, pr);
}

template <typename T>
void b_zfwd_t(const ProbDesc *d, const BatchPlan &pl, bool fused, int parity, hipStream_t s)
{
    switch (pl.r2) {
    case 2: b_zfwd_wave<T, 2>(d, pl, fused, parity, s); break;
    case 4: b_zfwd_wave<T, 4>(d, pl, fused, parity, s); break;
    case 8: b_zfwd_wave<T, 8>(d, pl, fused, parity, s); break;
    case 16:
        if constexpr (sizeof(T) == 4) b_zfwd_wave<T, 16>(d, pl, fused, parity, s);
        else AXI_REQUIRE(false, "no one-wave FP64 plan for N = 2048");
        break;
    default: {
        const size_t shm = transform_lds<T>(pl.nz_max);
        const dim3 grid(pl.blocks), block(256);
        const ProbDesc *dp = d + pl.off;
        if (twiddles_in_lds<T>(pl.nz_max)) {
            if (fused) hipLaunchKernelGGL((k_b_zfwd<T, true, true>), grid, block, shm, s, dp, pl.n, parity);
            else hipLaunchKernelGGL((k_b_zfwd<T, false, true>), grid, block, shm, s, dp, pl.n, parity);
        } else {
            if (fused) hipLaunchKernelGGL((k_b_zfwd<T, true, false>), grid, block, shm, s, dp, pl.n, parity);
            else hipLaunchKernelGGL((k_b_zfwd<T, false, false>), grid, block, shm, s, dp, pl.n, parity);
        }
    }
    }
    AXI_CHECK_HIP(hipGetLastError());
}

template <typename T>
void b_zinv_t(const ProbDesc *d, const BatchPlan &pl, int mode, bool pr, hipStream_t s)
{
    switch (pl.r2) {
    case 2: b_zinv_wave<T, 2>(d, pl, mode, pr, s); break;
    case 4: b_zinv_wave<T, 4>(d, pl, mode, pr, s); break;
    case 8: b_zinv_wave<T, 8>(d, pl, mode, pr, s); break;
    case 16:
        if constexpr (sizeof(T) == 4) b_zinv_wave<T, 16>(d, pl, mode, pr, s);
        else AXI_REQUIRE(false, "no one-wave FP64 plan for N = 2048");
        break;
    default: {
        const size_t shm = transform_lds<T>(pl.nz_max);
        const bool twl = twiddles_in_lds<T>(pl.nz_max);
        const dim3 grid(pl.blocks), block(256);
        const ProbDesc *dp = d + pl.off;
#define AXI_BZI(MD, TW) hipLaunchKernelGGL((k_b_zinv<T, MD, TW>), grid, block, shm, s, dp, pl.n, pr)
        if (mode == 1) { if (twl) AXI_BZI(1, true); else AXI_BZI(1, false); }
        else { if (twl) AXI_BZI(2, true); else AXI_BZI(2, false); }
#undef AXI_BZI
    }
    }
    AXI_CHECK_HIP(hipGetLastError());
}

void launch_b_zfwd(const ProbDesc *d, const BatchPlan &pl, int prec, bool fused, int parity, hipStream_t s)
{
    if (prec == AXIPCG_PREC_FP32) b_zfwd_t<float>(d, pl, fused, parity, s);
    else b_zfwd_t<double>(d, pl, fused, parity, s);
}

void launch_b_zinv(const ProbDesc *d, const BatchPlan &pl, int prec, int mode, bool pr, hipStream_t s)
{
    if (prec == AXIPCG_PREC_FP32) b_zinv_t<float>(d, pl, mode, pr, s);
    else b_zinv_t<double>(d, pl, mode, pr, s);
}

void launch_b_tridiag(const ProbDesc *d, int n, int blocks, int prec, const TriGate &g, int M, size_t shm,
                      hipStream_t s)
{
    if (prec == AXIPCG_PREC_FP32)
        hipLaunchKernelGGL(k_b_tridiag<float>, dim3(blocks), dim3(64 * M), shm, s, d, n, g, M);
    else
        hipLaunchKernelGGL(k_b_tridiag<double>, dim3(blocks), dim3(64 * M), shm, s, d, n, g, M);
    AXI_CHECK_HIP(hipGetLastError());
}

void launch_zfwd(const Operator &op, int prec, const ZfwdArgs &a, hipStream_t s)
{
    if (strip_usable(op, prec, strip_solve_rows(op, prec))) return strip_fwd(op, prec, strip_solve_rows(op, prec), a, s);
    if (prec == AXIPCG_PREC_FP32) {
        if (op.bc_z == DIR) zfwd_t<float, DIR>(op, a, s);
        else zfwd_t<float, AXIPCG_Z_NEUMANN>(op, a, s);
    } else {
        if (op.bc_z == DIR) zfwd_t<double, DIR>(op, a, s);
        else zfwd_t<double, AXIPCG_Z_NEUMANN>(op, a, s);
    }
}

void launch_zinv(const Operator &op, int prec, const ZinvArgs &a, hipStream_t s)
{
    if (strip_usable(op, prec, strip_solve_rows(op, prec))) return strip_inv(op, prec, strip_solve_rows(op, prec), a, s);
    if (prec == AXIPCG_PREC_FP32) {
        if (op.bc_z == DIR) zinv_t<float, DIR>(op, a, s);
        else zinv_t<float, AXIPCG_Z_NEUMANN>(op, a, s);
    } else {
        if (op.bc_z == DIR) zinv_t<double, DIR>(op, a, s);
        else zinv_t<double, AXIPCG_Z_NEUMANN>(op, a, s);
    }
}

void launch_tridiag(const Operator &op, int prec, const TriGate &g, hipStream_t s)
{
    if (strip_usable(op, prec, strip_solve_rows(op, prec)))
        return strip_reduced(op, prec, strip_solve_rows(op, prec), g, s);
    if (prec == AXIPCG_PREC_FP32) tridiag_t<float>(op, g, s);
    else tridiag_t<double>(op, g, s);
}

// Standalone applies of FP32 rows of length 2048 use strips of 8 rows when
// strips are on (their transform kernels fit the registers of 8-wave
// workgroups without the PCG vectors, and the reduced system halves); the
// solves keep strip_solve_rows.
void precond_apply_impl(const Operator &op, const double *r, double *z, int prec, hipStream_t s)
{
    int rows = strip_solve_rows(op, prec);
    if (rows == 4 && prec == AXIPCG_PREC_FP32 && op.nz == 2048 && strip_usable(op, prec, 8)) rows = 8;
    if (rows > 0 && strip_usable(op, prec, rows)) {
        ZfwdArgs fa;
        fa.rin = r;
        strip_fwd(op, prec, rows, fa, s);
        strip_reduced(op, prec, rows, TriGate{}, s);
        ZinvArgs ia;
        ia.zout = z;
        strip_inv(op, prec, rows, ia, s);
        return;
    }
    ZfwdArgs fa;
    fa.rin = r;
    launch_zfwd(op, prec, fa, s);
    launch_tridiag(op, prec, TriGate{}, s);
    ZinvArgs ia;
    ia.zout = z;
    launch_zinv(op, prec, ia, s);
}

}  // namespace axipcg
