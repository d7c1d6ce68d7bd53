// Device phases of the strip-partitioned preconditioner (§4.2 eqs.
// (36)-(39) with the partition idea of §3), shared by its three-launch form
// (strip.hip) and its single-launch form (pfused.hip).  Notation and the
// algebra of the reduced equations: strip.hip.
#pragma once

#include "wxform.h"

namespace axipcg {
namespace {

template <typename T>
struct Lines {
    const T *cb, *db, *rw, *lam;
};

// ---------------------------------------------------------------------------
// Phase 1 (K1): transform of the strip's rows into the LDS tile (row t = the
// LDS slice of wave t), then per mode the forward sweep over the interior
// rows.  f' replaces f in the tile (and, with `fprime`, is written to global
// memory for a separate K3); E1 and G0 go to the reduced arrays.  Returns
// false when the workgroup has nothing to do (stopped or broken down).
// ---------------------------------------------------------------------------
template <typename T, int BC, bool FUSED, int R2, int R>
__device__ __forceinline__ bool
strip_phase1(const double *__restrict__ rin, double *__restrict__ x, double *__restrict__ r,
             const double *__restrict__ p, const double *__restrict__ q, PcgState *st,
             double *__restrict__ partials, int n_pq, T *__restrict__ fprime, T *__restrict__ red_e,
             T *__restrict__ red_g, const typename vec2_of<T>::type *__restrict__ tw,
             const typename vec2_of<T>::type *__restrict__ pt, const Lines<T> &ln, int nr, int s, T *tile)
{
    using Gm = wfft::Geo<R2>;
    constexpr int N = Gm::N, PITCH = 2 * Gm::LB, n = R - 1, NT = 64 * R;
    const int wv = threadIdx.x >> 6;
    const int i0 = s * R;
    // the r-line coefficients of the strip and this thread's modes'
    // eigenvalues: issued before the transform in the plain form, after it
    // in the PCG form (there the early reads made the launch 1.3 us slower
    // at 1024^2, 13.8 -> 15.1 us)
    T cbv[R], dbv[R], rwv[R];
    constexpr int NL = (N + NT - 1) / NT;
    T lamv[NL];
    auto load_lines = [&]() {
#pragma unroll
        for (int t = 0; t < R; ++t) {
            cbv[t] = ln.cb[i0 + t];
            dbv[t] = ln.db[i0 + t];
            rwv[t] = ln.rw[i0 + t];
        }
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int l = threadIdx.x + u * NT;
            lamv[u] = l < N ? ln.lam[l] : (T)0;
        }
    };
    if constexpr (!FUSED) load_lines();
    if (!zfwd_w_body<T, BC, FUSED, R2>(rin, x, r, p, q, st, partials, n_pq, tw, pt, nr, i0 + wv, s,
                                        RowStore<T>{tile + wv * PITCH}))
        return false;
    if constexpr (FUSED) load_lines();
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NL; ++u) {
        const int l = threadIdx.x + u * NT;
        if (l >= N) break;
        const T lam = lamv[u];
        T f[R];
#pragma unroll
        for (int t = 0; t < R; ++t) f[t] = tile[t * PITCH + l];
        T cp[R], fp[R];
        T cprev = 0, gprev = 0;
#pragma unroll
        for (int t = 0; t < n; ++t) {
            const T L = t > 0 ? cbv[t - 1] : (T)0;
            const T inv = fast_rcp<T>(dbv[t] + rwv[t] * lam - L * cprev);
            cprev = cbv[t] * inv;
            gprev = (f[t] + L * gprev) * inv;
            cp[t] = cprev;
            fp[t] = gprev;
        }
        if (fprime) {
#pragma unroll
            for (int t = 0; t < n; ++t) fprime[(size_t)(i0 + t) * N + l] = fp[t];
        } else {
#pragma unroll
            for (int t = 0; t < n; ++t) tile[t * PITCH + l] = fp[t];
        }
        T g0 = fp[n - 1];
#pragma unroll
        for (int t = n - 2; t >= 0; --t) g0 = fp[t] + cp[t] * g0;
        red_e[(size_t)s * N + l] = f[n] + cbv[n - 1] * fp[n - 1];
        red_g[(size_t)s * N + l] = g0;
    }
    return true;
}

// ---------------------------------------------------------------------------
// K2
// ---------------------------------------------------------------------------
// The r-line arrays staged in LDS, row i at i + i / 32 (the rows a lane
// reads are 4 R apart, so without the gap they would share banks).
template <typename T>
struct LdsLines {
    const T *cb, *db, *rw;
    __device__ static int at(int i) { return i + (i >> 5); }
    __device__ T c(int i) const { return cb[at(i)]; }
    __device__ T d(int i) const { return db[at(i)]; }
    __device__ T w(int i) const { return rw[at(i)]; }
};

// Coefficient-only quantities of strip s for mode lam: v'_{n-1}, c'_{n-1},
// v_0 and w_0 (see the header comment).
template <typename T, int R>
__device__ inline void strip_coefs(const LdsLines<T> &ln, int s, T lam, T &vL, T &wL, T &v0, T &w0)
{
    constexpr int n = R - 1;
    const int i0 = s * R;
    T cp[R], vp[R];
    T cprev = 0, vprev = 0;
    const T cbm = s > 0 ? ln.c(i0 - 1) : (T)0;
#pragma unroll
    for (int t = 0; t < n; ++t) {
        const T L = t > 0 ? ln.c(i0 + t - 1) : (T)0;
        const T inv = fast_rcp<T>(ln.d(i0 + t) + ln.w(i0 + t) * lam - L * cprev);
        cprev = ln.c(i0 + t) * inv;
        vprev = (t == 0 ? cbm : L * vprev) * inv;
        cp[t] = cprev;
        vp[t] = vprev;
    }
    vL = vp[n - 1];
    wL = cp[n - 1];
    T v = vL, w = wL;
#pragma unroll
    for (int t = n - 2; t >= 0; --t) {
        v = vp[t] + cp[t] * v;
        w = cp[t] * w;
    }
    v0 = v;
    w0 = w;
}

// One tridiagonal system a_k x_{k-1} + b_k x_k + c_k x_{k+1} = e_k of G
// unknowns per wavefront: lane `lane` < S = min(64, G) owns k in [lo, hi)
// (m = hi - lo rows in registers, index 0 .. m-1).  Its interior rows are
// eliminated in terms of the previous lane's last unknown and its own last
// unknown; the S last unknowns then form a tridiagonal system solved by
// parallel cyclic reduction over the lanes; each lane back-substitutes.
// On return x[0 .. m-1] hold the lane's unknowns.
template <typename T, int LMAX>
__device__ inline void wave_tri(const T (&a)[LMAX], const T (&b)[LMAX], const T (&c)[LMAX], const T (&e)[LMAX],
                                T (&x)[LMAX], int m, int S, int lane)
{
    const bool active = lane < S;
    T gp[LMAX], vp[LMAX], cq[LMAX];
    T gl = 0, vl = 0, wl = 0;
#pragma unroll
    for (int t = 0; t < LMAX; ++t) {
        if (t < m - 1) {
            const T den = t == 0 ? b[0] : b[t] + a[t] * cq[t - 1];
            const T inv = fast_rcp<T>(den);
            gp[t] = (t == 0 ? e[0] : e[t] - a[t] * gp[t - 1]) * inv;
            vp[t] = -(t == 0 ? a[0] : a[t] * vp[t - 1]) * inv;
            cq[t] = -c[t] * inv;
            gl = gp[t];
            vl = vp[t];
            wl = cq[t];
        }
    }
    // the first row in terms of (X_prev, X_own): y_0 = g0 + v0 X_prev + w0 X_own
    T g0 = 0, v0 = 0, w0 = 1;
    if (m >= 2) {
        g0 = gl;
        v0 = vl;
        w0 = wl;
#pragma unroll
        for (int t = LMAX - 1; t >= 0; --t) {
            if (t < m - 2) {
                g0 = gp[t] + cq[t] * g0;
                v0 = vp[t] + cq[t] * v0;
                w0 = cq[t] * w0;
            }
        }
    }
    if (!active) { g0 = 0; v0 = 0; w0 = 0; }
    const T G0n = __shfl_down(g0, 1, 64), V0n = __shfl_down(v0, 1, 64), W0n = __shfl_down(w0, 1, 64);
    const bool has_next = active && lane + 1 < S;
    T ra = 0, rb = 1, rc = 0, re = 0;
    if (active) {
        T am = 0, bm = 0, cm = 0, em = 0;   // the lane's last row
#pragma unroll
        for (int t = 0; t < LMAX; ++t)
            if (t == m - 1) { am = a[t]; bm = b[t]; cm = c[t]; em = e[t]; }
        const T gn = has_next ? G0n : (T)0, vn = has_next ? V0n : (T)0, wn = has_next ? W0n : (T)0;
        if (m >= 2) {
            ra = am * vl;
            rb = bm + am * wl + cm * vn;
            re = em - am * gl - cm * gn;
        } else {
            ra = am;
            rb = bm + cm * vn;
            re = em - cm * gn;
        }
        rc = cm * wn;
    }
    for (int k = 1; k < S; k <<= 1) {
        const T am = __shfl_up(ra, k, 64), bm = __shfl_up(rb, k, 64);
        const T cm = __shfl_up(rc, k, 64), em = __shfl_up(re, k, 64);
        const T ap = __shfl_down(ra, k, 64), bp = __shfl_down(rb, k, 64);
        const T cp = __shfl_down(rc, k, 64), ep = __shfl_down(re, k, 64);
        const bool hm = lane >= k, hp = lane + k < S;
        const T al = hm ? -ra * fast_rcp<T>(bm) : (T)0;
        const T ga = hp ? -rc * fast_rcp<T>(bp) : (T)0;
        const T na = hm ? al * am : (T)0;
        const T nc = hp ? ga * cp : (T)0;
        const T nb = rb + (hm ? al * cm : (T)0) + (hp ? ga * ap : (T)0);
        const T ne = re + (hm ? al * em : (T)0) + (hp ? ga * ep : (T)0);
        if (active) { ra = na; rb = nb; rc = nc; re = ne; }
    }
    const T X = active ? re / rb : (T)0;
    T Xp = __shfl_up(X, 1, 64);
    if (lane == 0) Xp = 0;
    T y = X;
#pragma unroll
    for (int t = LMAX - 1; t >= 0; --t) {
        if (t == m - 1) x[t] = X;
        if (t < m - 1) {
            y = gp[t] + vp[t] * Xp + cq[t] * y;
            x[t] = y;
        }
    }
}

// LDS of the reduced-system phase: the r-line arrays (padded, LdsLines) and
// the reduced data of `mt` modes, [mt][G] each for E1 and G0.
template <typename T>
__host__ __device__ inline size_t strip_red_lds(int nr, int G, int mt)
{
    return (3 * (size_t)(nr + nr / 32 + 1) + 2 * (size_t)mt * G) * sizeof(T);
}

// Phase 2 (K2) part 1: stage the r-line arrays and the reduced data of modes
// [l0, l0 + mt) into LDS (`base`); vector loads when the mt values of a
// strip's row are 16-byte pieces.
template <typename T, bool VEC>
__device__ __forceinline__ void strip_stage2(const T *__restrict__ red_e, const T *__restrict__ red_g,
                                             const Lines<T> &ln, int nr, int N, int G, int l0, int mt, T *base)
{
    const int npad = nr + nr / 32 + 1;
    T *lc = base, *ld = lc + npad, *lw = ld + npad, *te = lw + npad, *tg = te + mt * G;
    for (int i = threadIdx.x; i < nr; i += blockDim.x) {
        const int a = LdsLines<T>::at(i);
        lc[a] = ln.cb[i];
        ld[a] = ln.db[i];
        lw[a] = ln.rw[i];
    }
    if constexpr (VEC) {
        constexpr int VW = 16 / (int)sizeof(T);
        typedef T V __attribute__((ext_vector_type(VW)));
        const int nv = mt / VW;
        for (int e = threadIdx.x; e < G * nv; e += blockDim.x) {
            const int s = e / nv, u = (e - s * nv) * VW;
            const V ve = *reinterpret_cast<const V *>(red_e + (size_t)s * N + l0 + u);
            const V vg = *reinterpret_cast<const V *>(red_g + (size_t)s * N + l0 + u);
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                te[(u + k) * G + s] = ve[k];
                tg[(u + k) * G + s] = vg[k];
            }
        }
    } else {
        for (int e = threadIdx.x; e < G * mt; e += blockDim.x) {
            const int s = e / mt, mm = e - s * mt;
            te[mm * G + s] = red_e[(size_t)s * N + l0 + mm];
            tg[mm * G + s] = red_g[(size_t)s * N + l0 + mm];
        }
    }
}

// Phase 2 (K2) part 2, after the stage is visible to the workgroup: the
// reduced systems of modes [l0, l0 + mt), wave w taking modes l0 + w,
// l0 + w + waves, ...; the solutions X_s go to red_x.
template <typename T, int R, int LMAX, bool VEC>
__device__ __forceinline__ void strip_solve2(T *__restrict__ red_x, const Lines<T> &ln, int nr, int N, int G, int l0,
                                             int mt, T *base)
{
    const int npad = nr + nr / 32 + 1;
    T *lc = base, *ld = lc + npad, *lw = ld + npad, *te = lw + npad, *tg = te + mt * G;
    const LdsLines<T> ll{lc, ld, lw};
    const int waves = blockDim.x >> 6, lane = threadIdx.x & 63;
    const int S = G < 64 ? G : 64;
    const int lo = lane < S ? (int)(((long)lane * G) / S) : G;
    const int hi = lane < S ? (int)(((long)(lane + 1) * G) / S) : G;
    const int m = hi - lo;
    for (int w = threadIdx.x >> 6; w < mt; w += waves) {
        const T lam = ln.lam[l0 + w];
        // this lane's strips: vL, wL, and the next strip's v0, w0, G0
        T vL[LMAX], wL[LMAX], v0[LMAX], w0[LMAX];
#pragma unroll
        for (int k = 0; k < LMAX; ++k)
            if (k < m) strip_coefs<T, R>(ll, lo + k, lam, vL[k], wL[k], v0[k], w0[k]);
        const T v0n_l = __shfl_down(m > 0 ? v0[0] : (T)0, 1, 64);
        const T w0n_l = __shfl_down(m > 0 ? w0[0] : (T)0, 1, 64);
        T a[LMAX], b[LMAX], c[LMAX], e[LMAX], xs[LMAX];
#pragma unroll
        for (int k = 0; k < LMAX; ++k) {
            a[k] = 0; b[k] = 1; c[k] = 0; e[k] = 0;
            if (k < m) {
                const int s = lo + k, j = s * R + R - 1;
                const bool last = s + 1 >= G;
                T vn = 0, wn = 0, gn = 0;
                if (!last) {
                    vn = (k + 1 < m) ? v0[k + 1] : v0n_l;
                    wn = (k + 1 < m) ? w0[k + 1] : w0n_l;
                    gn = tg[w * G + s + 1];
                }
                const T cjm = ll.c(j - 1), cj = last ? (T)0 : ll.c(j);
                a[k] = -cjm * vL[k];
                b[k] = ll.d(j) + ll.w(j) * lam - cjm * wL[k] - cj * vn;
                c[k] = -cj * wn;
                e[k] = te[w * G + s] + cj * gn;
            }
        }
        wave_tri<T, LMAX>(a, b, c, e, xs, m, S, lane);
        // te row w is this wave's alone: its solution replaces it (every lane
        // has read its e values above)
#pragma unroll
        for (int k = 0; k < LMAX; ++k)
            if (k < m) te[w * G + lo + k] = xs[k];
    }
    __syncthreads();
    if constexpr (VEC) {
        constexpr int VW = 16 / (int)sizeof(T);
        typedef T V __attribute__((ext_vector_type(VW)));
        const int nv = mt / VW;
        for (int e2 = threadIdx.x; e2 < G * nv; e2 += blockDim.x) {
            const int s = e2 / nv, u = (e2 - s * nv) * VW;
            V vx;
#pragma unroll
            for (int k = 0; k < VW; ++k) vx[k] = te[(u + k) * G + s];
            *reinterpret_cast<V *>(red_x + (size_t)s * N + l0 + u) = vx;
        }
    } else {
        for (int e2 = threadIdx.x; e2 < G * mt; e2 += blockDim.x) {
            const int s = e2 / mt, mm = e2 - s * mt;
            red_x[(size_t)s * N + l0 + mm] = te[mm * G + s];
        }
    }
}

// ---------------------------------------------------------------------------
// Phase 3 (K3): the strip's interior rows from f', X_{s-1} and X_s in the
// LDS tile (f' loaded from global memory when `fprime` is given, else
// already in the tile), then each wave's inverse transform of its row.
// ---------------------------------------------------------------------------
template <typename T, int BC, int MODE, int R2, int R>
__device__ __forceinline__ void
strip_phase3(const T *__restrict__ fprime, const T *__restrict__ red_x, double *__restrict__ zout,
             const double *__restrict__ r, const PcgState *st, double *__restrict__ partials, bool pr,
             const typename vec2_of<T>::type *__restrict__ tw, const typename vec2_of<T>::type *__restrict__ pt,
             const Lines<T> &ln, int nr, double *__restrict__ dinc, double tau, double rho2, int s, T *tile)
{
    using Gm = wfft::Geo<R2>;
    constexpr int N = Gm::N, PITCH = 2 * Gm::LB, n = R - 1, NT = 64 * R;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i0 = s * R;
    // PCG modes: this wave's r row is loaded first, so that its latency
    // overlaps the back substitution (where it fits in registers)
    constexpr bool PRE = (MODE == 1 || MODE == 2) && R2 <= 8;
    double2 rpre[PRE ? R2 : 1];
    if constexpr (PRE) {
#pragma unroll
        for (int t = 0; t < R2; ++t)
            rpre[t] = *reinterpret_cast<const double2 *>(r + (size_t)(i0 + wv) * N + 2 * lane + 128 * t);
    }
    // this thread's modes' eigenvalues and reduced solutions X_s, X_{s-1}
    // (the previous launch's output), issued with the row loads instead of
    // after the workgroup barrier below
    constexpr int NL = (N + NT - 1) / NT;
    T lamv[NL], xsv[NL], xpv[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
        const int l = threadIdx.x + u * NT;
        lamv[u] = l < N ? ln.lam[l] : (T)0;
        xsv[u] = l < N ? red_x[(size_t)s * N + l] : (T)0;
        xpv[u] = (l < N && s > 0) ? red_x[(size_t)(s - 1) * N + l] : (T)0;
    }
    if (fprime) {
        // f' of the interior rows into the tile, 16 bytes per access
        constexpr int VW = 16 / (int)sizeof(T);
        typedef T V __attribute__((ext_vector_type(VW)));
        for (int e = threadIdx.x; e < n * (N / VW); e += NT) {
            const int t = e / (N / VW), k = (e - t * (N / VW)) * VW;
            const V v = *reinterpret_cast<const V *>(fprime + (size_t)(i0 + t) * N + k);
#pragma unroll
            for (int u = 0; u < VW; ++u) tile[t * PITCH + k + u] = v[u];
        }
    }
    T cbv[R], dbv[R], rwv[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
        cbv[t] = ln.cb[i0 + t];
        dbv[t] = ln.db[i0 + t];
        rwv[t] = ln.rw[i0 + t];
    }
    const T cbm = s > 0 ? ln.cb[i0 - 1] : (T)0;
    // a stopped solve (every workgroup alike) returns here, its loads already
    // issued rather than waiting on the flag before them
    if (MODE != 0 && st->done) return;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NL; ++u) {
        const int l = threadIdx.x + u * NT;
        if (l >= N) break;
        const T lam = lamv[u], Xs = xsv[u], Xp = xpv[u];
        T cp[R], vp[R];
        T cprev = 0, vprev = 0;
#pragma unroll
        for (int t = 0; t < n; ++t) {
            const T L = t > 0 ? cbv[t - 1] : (T)0;
            const T inv = fast_rcp<T>(dbv[t] + rwv[t] * lam - L * cprev);
            cprev = cbv[t] * inv;
            vprev = (t == 0 ? cbm : L * vprev) * inv;
            cp[t] = cprev;
            vp[t] = vprev;
        }
        T y = Xs;
        tile[n * PITCH + l] = Xs;
#pragma unroll
        for (int t = n - 1; t >= 0; --t) {
            y = tile[t * PITCH + l] + vp[t] * Xp + cp[t] * y;
            tile[t * PITCH + l] = y;
        }
    }
    __syncthreads();
    zinv_w_body<T, BC, MODE, R2>(RowLoad<T>{tile + wv * PITCH}, zout, r, st, partials, pr, tw, pt, nr, dinc, tau,
                                 rho2, i0 + wv, s, PRE ? rpre : nullptr);
}

}  // namespace
}  // namespace axipcg
