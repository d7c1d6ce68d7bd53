// Device bodies of the preconditioner's launches (§4.2 eqs. (36)-(39)):
// the block-wide forward and inverse z-transforms of whole rows (any
// transform length with a Stockham plan), the partitioned r-tridiagonal
// solve of M modes per workgroup, and the per-precision tables of a batch
// member.  Each body takes its work item (vb) as an argument, so a launch
// may map one item per workgroup or deal items to resident workgroups.
#pragma once

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
// rows, both real, one complex FFT transforms them together (the first as
// real, the second as imaginary part), and the two spectra are separated
// by the conjugate symmetry of a real row's FFT; the second row's loads are
// issued while the first row is reordered into LDS.
// ---------------------------------------------------------------------------
template <typename T, int BC, bool FUSED, bool TWLDS, int ROWS, bool WG_STOP = false>
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

    if constexpr (WG_STOP) {
        if (st && wg_flag(&st->done)) return;
    } else {
        if (st && st->done) return;
    }
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
    // two rows: one complex FFT of (row 0) + i (row 1), both rows real
    constexpr bool PAIR = (ROWS == 2);
    static_assert(ROWS == 1 || ROWS == 2, "one or two rows per workgroup");
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
            if constexpr (PAIR) {
                if (s == 0) a[n].x = v;
                else a[n].y = v;
            } else {
                a[n] = {v, (T)0};
            }
        }
        if (s + 1 < ROWS) load(i0 + s + 1);
        if (PAIR && s == 0) continue;   // the second row fills the imaginary parts
        __syncthreads();
        const cx<T> *Vr = fft_stockham<T>(a, b, N, twp);
        if constexpr (PAIR) {
            // Z = V0 + i V1 with V0, V1 the spectra of the two real rows:
            // V0_m = (Z_m + conj Z_{N-m}) / 2, V1_m = (Z_m - conj Z_{N-m}) / 2i
            const size_t row0 = (size_t)i0 * N;
            for (int j = threadIdx.x; j < N; j += blockDim.x) {
                const int m = (BC == DIR) ? N - 1 - j : j;
                const cx<T> zm = Vr[m], zc = Vr[(N - m) & (N - 1)];
                const cx<T> w = ld_tw<T>(pt, m);
                const T v0x = (T)0.5 * (zm.x + zc.x), v0y = (T)0.5 * (zm.y - zc.y);
                const T v1x = (T)0.5 * (zm.y + zc.y), v1y = (T)0.5 * (zc.x - zm.x);
                const bool edge = (BC == DIR) ? (j == N - 1) : (j == 0);
                const T sc = nrm * (edge ? half : (T)1);
                spec[row0 + j] = sc * (v0x * w.x - v0y * w.y);
                spec[row0 + N + j] = sc * (v1x * w.x - v1y * w.y);
            }
        } else {
            for (int j = threadIdx.x; j < N; j += blockDim.x) {
                const int m = (BC == DIR) ? N - 1 - j : j;
                const cx<T> w = ld_tw<T>(pt, m);
                const T Y = Vr[m].x * w.x - Vr[m].y * w.y;
                const bool edge = (BC == DIR) ? (j == N - 1) : (j == 0);
                spec[row + j] = nrm * (edge ? half : (T)1) * Y;
            }
        }
    }
    if (FUSED) {
        const double s = block_sum(rr, red);
        if (threadIdx.x == 0) partials[SLOT_RR * MAX_PARTIALS + vb] = s;
    }
}

// ---------------------------------------------------------------------------
// Inverse transform: one workgroup per ROWS consecutive r-rows, FP64 output;
// two rows go through one complex FFT as in the forward transform.
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
    // two rows: one FFT of conj(V0) + i conj(V1), whose real and imaginary
    // parts are N times the two real rows
    constexpr bool PAIR = (ROWS == 2);
    static_assert(ROWS == 1 || ROWS == 2, "one or two rows per workgroup");
    if (!PAIR) load(i0);
    const T invN = (T)1 / (T)N;
    double rz = 0.0, rzo = 0.0;
    double c1 = 0.0, c2 = 0.0;
    if (CHEB) {
        const double alpha = cheb_alpha(st->iters + 1, rho2);
        c1 = alpha - 1.0;
        c2 = alpha * tau;
    }
    // r (and the old z) of the rows are in flight during the FFT
    double rv[ROWS][KPT], zo[ROWS][KPT];
    auto load_r = [&](int si) {
        const size_t row = (size_t)(i0 + si) * N;
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
            const int k = threadIdx.x + j * blockDim.x;
            if (k < N) {
                rv[si][j] = r[row + k];
                if (pr) zo[si][j] = zout[row + k];
            }
        }
    };
    // z of row si from the FFT's output: real (t = 0) or imaginary (t = 1) parts
    auto store = [&](const cx<T> *res, int si, int t) {
        const size_t rowt = (size_t)(i0 + si) * N;
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
            const int k = threadIdx.x + j * blockDim.x;
            if (k >= N) continue;
            const int n = (k & 1) ? N - 1 - (k >> 1) : (k >> 1);
            T v = (t == 0 ? res[n].x : res[n].y) * invN;
            if (BC == DIR && (k & 1)) v = -v;
            const double zv = (double)v;
            if (PCGM) {
                if (pr) rzo += rv[si][j] * zo[si][j];
                rz += rv[si][j] * zv;
            }
            if (CHEB) {
                if (MODE == 4) dinc[rowt + k] = c2 * zv;
                else dinc[rowt + k] = c1 * dinc[rowt + k] + c2 * zv;
            } else {
                zout[rowt + k] = zv;
            }
        }
    };
    if constexpr (PAIR) {
        // both rows' Y_m staged in b (the FFT's scratch until it starts), so
        // that each spectral value is read from memory once; Y_{N-m} then
        // comes from LDS
        const size_t row0 = (size_t)i0 * N;
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
            const int m = threadIdx.x + j * blockDim.x;
            if (m < N) b[m] = {Yval(row0, m), Yval(row0 + N, m)};
        }
        if (PCGM) {
            load_r(0);
            load_r(1);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
            const int m = threadIdx.x + j * blockDim.x;
            if (m < N) {
                const cx<T> y = b[m];
                const cx<T> yn = (m == 0) ? cx<T>{(T)0, (T)0} : b[N - m];
                const cx<T> w = ld_tw<T>(pt, m);      // exp(-i pi m / 2N)
                // conj(V) = w (ym + i yn) for each row
                const cx<T> q0 = {w.x * y.x - w.y * yn.x, w.x * yn.x + w.y * y.x};
                const cx<T> q1 = {w.x * y.y - w.y * yn.y, w.x * yn.y + w.y * y.y};
                a[m] = {q0.x - q1.y, q0.y + q1.x};
            }
        }
        __syncthreads();
        const cx<T> *res = fft_stockham<T>(a, b, N, twp);
        store(res, 0, 0);
        store(res, 1, 1);
    } else {
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
            const int m = threadIdx.x + j * blockDim.x;
            if (m < N) {
                const cx<T> w = ld_tw<T>(pt, m);      // exp(-i pi m / 2N)
                // V = conj(w) (ym - i yn); store conj(V) = w (ym + i yn)
                a[m] = {w.x * ymv[j] - w.y * ynv[j], w.x * ynv[j] + w.y * ymv[j]};
            }
        }
        if (PCGM) load_r(0);
        __syncthreads();
        const cx<T> *res = fft_stockham<T>(a, b, N, twp);
        store(res, 0, 0);
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
    __shared__ double red[RED_SLOTS];
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

    GatePre pre;
    if (g.mode == 1) gate_issue(st, partials, g, pre);
    constexpr int VW = 16 / (int)sizeof(T);   // modes per 16-byte piece
    if (M % VW == 0) {
        // the row's M modes as 16-byte pieces (one or two per row)
        const int nv = M / VW;
        for (int e = threadIdx.x; e < nr * nv; e += blockDim.x) {
            const int row = e / nv, h = e - row * nv;
            const uint4 v = *reinterpret_cast<const uint4 *>(spec + (size_t)row * nz + l0 + h * VW);
            const T *tv = reinterpret_cast<const T *>(&v);
            for (int m = 0; m < VW; ++m) tile[(h * VW + m) * pitch + prow(row)] = tv[m];
        }
    } else {
        for (int e = threadIdx.x; e < nr * M; e += blockDim.x) {
            const int row = e / M, m = e - row * M;
            tile[m * pitch + prow(row)] = spec[(size_t)row * nz + l0 + m];
        }
    }
    if (g.mode != 0 && tridiag_gate(st, partials, g, red, vb, g.mode == 1 ? &pre : nullptr) != ST_RUN) return;
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
    if (M % VW == 0) {
        const int nv = M / VW;
        for (int e = threadIdx.x; e < nr * nv; e += blockDim.x) {
            const int row = e / nv, h = e - row * nv;
            uint4 v;
            T *tv = reinterpret_cast<T *>(&v);
            for (int m = 0; m < VW; ++m) tv[m] = tile[(h * VW + m) * pitch + prow(row)];
            *reinterpret_cast<uint4 *>(spec + (size_t)row * nz + l0 + h * VW) = v;
        }
    } else {
        for (int e = threadIdx.x; e < nr * M; e += blockDim.x) {
            const int row = e / M, m = e - row * M;
            spec[(size_t)row * nz + l0 + m] = tile[m * pitch + prow(row)];
        }
    }
}

// ---- batch members' tables by precision -------------------------------
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

// ---- work items of the batched launches ------------------------------------
// One item of a batched phase, `g` its index over the batch's items of that
// phase: a launch passes its workgroup index; the single-launch batch deals
// the items to its resident workgroups.  The transforms' `d` holds the
// problems of one transform plan, with tr_start counted within the plan.
// WG_STOP: the fused forward reads the stop flag once per workgroup, for
// workgroups that go on to other items (no wave may leave an item that the
// others go on with).  GATE: the plain transform of the Chebyshev step, which
// returns once the member has stopped.  The inverse transforms' modes 3 and 4
// form the Chebyshev increment in the member's p0 buffer with its tau, rho2.
template <typename T, bool FUSED, bool TWLDS, bool WG_STOP, bool GATE = false>
__device__ __forceinline__ void b_zfwd_item(const ProbDesc *__restrict__ d, int n, int g, int parity)
{
    const int p = find_problem(d, n, g, RANGE_TR);
    const ProbDesc &P = d[p];
    const double *pnew = parity ? P.p0 : P.p1;   // written by this iteration's SpMV
    const int vb = g - P.tr_start;
    // the start-up transform runs before the r-solve launch resets the state,
    // so only the in-loop transforms may read the stop flag
    PcgState *st = (FUSED || GATE) ? P.state : nullptr;
    if (P.bc_z == DIR)
        zfwd_body<T, DIR, FUSED, TWLDS, 1, WG_STOP>(P.r, P.x, P.r, pnew, P.q, st, P.partials, P.n_sp, (T *)P.spec,
                                        pd_tw<T>(P), pd_pt<T>(P), P.nr, P.nz, vb);
    else
        zfwd_body<T, AXIPCG_Z_NEUMANN, FUSED, TWLDS, 1, WG_STOP>(P.r, P.x, P.r, pnew, P.q, st, P.partials, P.n_sp,
                                                     (T *)P.spec, pd_tw<T>(P), pd_pt<T>(P), P.nr, P.nz, vb);
}

template <typename T, int MODE, bool TWLDS>
__device__ __forceinline__ void b_zinv_item(const ProbDesc *__restrict__ d, int n, int g, bool pr)
{
    const int p = find_problem(d, n, g, RANGE_TR);
    const ProbDesc &P = d[p];
    const int vb = g - P.tr_start;
    if (P.bc_z == DIR)
        zinv_body<T, DIR, MODE, TWLDS, 1>((const T *)P.spec, P.z, P.r, P.state, P.partials, pr, pd_tw<T>(P),
                                       pd_pt<T>(P), P.nr, P.nz, vb, P.p0, P.tau, P.rho2);
    else
        zinv_body<T, AXIPCG_Z_NEUMANN, MODE, TWLDS, 1>((const T *)P.spec, P.z, P.r, P.state, P.partials, pr,
                                                    pd_tw<T>(P), pd_pt<T>(P), P.nr, P.nz, vb, P.p0, P.tau, P.rho2);
}

template <typename T, bool FUSED, int R2, bool WG_STOP, bool GATE = false>
__device__ __forceinline__ void b_zfwd_w_item(const ProbDesc *__restrict__ d, int n, int g, int parity)
{
    const int p = find_problem(d, n, g, RANGE_TR);
    const ProbDesc &P = d[p];
    const double *pnew = parity ? P.p0 : P.p1;
    const int vb = g - P.tr_start;
    PcgState *st = (FUSED || GATE) ? P.state : nullptr;   // as in b_zfwd_item
    constexpr int WR = wave_rows<T, R2>();
    const int row = vb * WR + (threadIdx.x >> 6);
    RowStore<T> out{(T *)P.spec + (size_t)(row < P.nr ? row : 0) * wfft::Geo<R2>::N};
    if (P.bc_z == DIR)
        zfwd_w_body<T, DIR, FUSED, R2, WG_STOP>(P.r, P.x, P.r, pnew, P.q, st, P.partials, P.n_sp, pd_tw<T>(P), pd_pt<T>(P),
                                       P.nr, row, vb, out);
    else
        zfwd_w_body<T, AXIPCG_Z_NEUMANN, FUSED, R2, WG_STOP>(P.r, P.x, P.r, pnew, P.q, st, P.partials, P.n_sp, pd_tw<T>(P),
                                                    pd_pt<T>(P), P.nr, row, vb, out);
}

template <typename T, int MODE, int R2>
__device__ __forceinline__ void b_zinv_w_item(const ProbDesc *__restrict__ d, int n, int g, bool pr)
{
    const int p = find_problem(d, n, g, RANGE_TR);
    const ProbDesc &P = d[p];
    const int vb = g - P.tr_start;
    constexpr int WR = wave_rows<T, R2>();
    const int row = vb * WR + (threadIdx.x >> 6);
    RowLoad<T> in{(const T *)P.spec + (size_t)(row < P.nr ? row : P.nr - 1) * wfft::Geo<R2>::N};
    if (P.bc_z == DIR)
        zinv_w_body<T, DIR, MODE, R2>(in, P.z, P.r, P.state, P.partials, pr, pd_tw<T>(P), pd_pt<T>(P), P.nr, P.p0,
                                      P.tau, P.rho2, row, vb);
    else
        zinv_w_body<T, AXIPCG_Z_NEUMANN, MODE, R2>(in, P.z, P.r, P.state, P.partials, pr, pd_tw<T>(P), pd_pt<T>(P),
                                                   P.nr, P.p0, P.tau, P.rho2, row, vb);
}

template <typename T>
__device__ __forceinline__ void b_tridiag_item(const ProbDesc *__restrict__ d, int n, TriGate g, int M, int item)
{
    const int p = find_problem(d, n, item, RANGE_TRI);
    const ProbDesc &P = d[p];
    const int vb = item - P.tri_start;
    g.state = P.state;
    g.n_rr = (g.mode == 2 || g.rr_rows) ? P.nr : P.n_tr;   // one partial per row: the start's, Chebyshev's
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

}  // namespace
}  // namespace axipcg
