// Strip-partitioned preconditioner z = B^{-1} r (§4.2 eqs. (36)-(39)) with
// the partition idea of §3: the grid is cut into strips of R consecutive
// r-rows, one workgroup each, the interior of every strip is eliminated in
// terms of the strips' boundary rows (the "preparatory" solutions of
// eqs. (18)-(22)), and only one reduced equation per strip and z-mode crosses
// workgroups.  Three launches:
//
//  K1 (forward + local elimination): each wave z-transforms one row of the
//     strip into the workgroup's LDS tile; then, per mode, the strip's
//     interior rows are swept forward (Thomas) and the forward-eliminated
//     data f' is written back row by row, together with two values per
//     (strip, mode) that the reduced equations need (E1, G0 below).
//  K2 (reduced systems): per mode, the tridiagonal system in the strips'
//     last rows X_s (G = nr / R unknowns), solved by one wavefront (segments
//     per lane, parallel cyclic reduction across lanes).  In PCG mode it
//     first runs the stop test.
//  K3 (back substitution + inverse): each strip rebuilds its interior rows
//     from f', X_{s-1} and X_s in the LDS tile, and each wave inverse-
//     transforms one row to z.
//
// Every global access is along z (whole rows), so no kernel gathers or
// scatters the strided [nr][modes] tiles a per-mode r-solve needs; the
// spectral data crosses HBM once each way as f' (4 + 4 bytes per point in
// FP32), and the reduced data is 3 values per strip and mode.
//
// Notation for strip s (rows i0 = s R + t, t < R; n = R - 1 interior rows,
// interface row j = i0 + n), mode l with lam = kbar mu_l + qbar:
//   row equation  -cb[i-1] y[i-1] + (db[i] + rw[i] lam) y[i] - cb[i] y[i+1] = f[i];
//   interior sweep  den_t = D_t - L_t c'_{t-1},  c'_t = cb[i0+t] / den_t,
//                   f'_t = (f_t + L_t f'_{t-1}) / den_t,
//                   v'_t = (t = 0 ? cb[i0-1] : L_t v'_{t-1}) / den_t,
//     with L_t = cb[i0+t-1] (t >= 1), so that
//                   y_t = f'_t + v'_t X_{s-1} + c'_t y_{t+1},  y_n = X_s;
//   back to the first interior row: y_0 = G0 + v_0 X_{s-1} + w_0 X_s and
//   y_{n-1} = f'_{n-1} + v'_{n-1} X_{s-1} + c'_{n-1} X_s;
//   reduced equation of strip s (the interface row with both neighbours
//   eliminated):
//     a_s = -cb[j-1] v'_{n-1},  b_s = D_j - cb[j-1] c'_{n-1} - cb[j] v_0(s+1),
//     c_s = -cb[j] w_0(s+1),    e_s = E1_s + cb[j] G0_{s+1},
//     E1_s = f_j + cb[j-1] f'_{n-1}.
// The coefficient-only quantities (c', v', v_0, w_0) are recomputed where
// needed from the O(nr) r-line arrays instead of being stored.
#include "wxform.h"

namespace axipcg {
namespace {

template <typename T>
struct Lines {
    const T *cb, *db, *rw, *lam;
};

// ---------------------------------------------------------------------------
// K1
// ---------------------------------------------------------------------------
template <typename T, int BC, bool FUSED, int R2, int R>
__global__ void __launch_bounds__(64 * R)
k_strip_fwd(const double *__restrict__ rin, double *__restrict__ x, double *__restrict__ r,
            const double *__restrict__ p, const double *__restrict__ q, PcgState *st, double *__restrict__ partials,
            int n_pq, T *__restrict__ fprime, T *__restrict__ red_e, T *__restrict__ red_g,
            const typename vec2_of<T>::type *__restrict__ tw, const typename vec2_of<T>::type *__restrict__ pt,
            Lines<T> ln, int nr)
{
    using Gm = wfft::Geo<R2>;
    constexpr int N = Gm::N, PITCH = 2 * Gm::LB, n = R - 1, NT = 64 * R;
    extern __shared__ char smem_raw[];
    T *tile = reinterpret_cast<T *>(smem_raw);   // row t = the LDS slice of wave t
    const int wv = threadIdx.x >> 6;
    const int s = blockIdx.x, i0 = s * R;
    if (!zfwd_w_body<T, BC, FUSED, R2>(rin, x, r, p, q, st, partials, n_pq, tw, pt, nr, i0 + wv, s,
                                        RowStore<T>{tile + wv * PITCH}))
        return;
    T cbv[R], dbv[R], rwv[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
        cbv[t] = ln.cb[i0 + t];
        dbv[t] = ln.db[i0 + t];
        rwv[t] = ln.rw[i0 + t];
    }
    __syncthreads();
    for (int l = threadIdx.x; l < N; l += NT) {
        const T lam = ln.lam[l];
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
#pragma unroll
        for (int t = 0; t < n; ++t) fprime[(size_t)(i0 + t) * N + l] = fp[t];
        T g0 = fp[n - 1];
#pragma unroll
        for (int t = n - 2; t >= 0; --t) g0 = fp[t] + cp[t] * g0;
        red_e[(size_t)s * N + l] = f[n] + cbv[n - 1] * fp[n - 1];
        red_g[(size_t)s * N + l] = g0;
    }
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

// MT modes per workgroup (one wave each).  The r-line arrays are staged in
// LDS once for the workgroup (every mode reads them), and the reduced data of
// the tile [G][MT] is staged as [MT][G].
template <typename T, int MT>
__host__ __device__ constexpr size_t strip_red_lds(int nr, int G)
{
    return (3 * (size_t)(nr + nr / 32 + 1) + 2 * (size_t)MT * G) * sizeof(T);
}

template <typename T, int R, int LMAX, int MT>
__global__ void __launch_bounds__(64 * MT)
k_strip_reduced(const T *__restrict__ red_e, const T *__restrict__ red_g, T *__restrict__ red_x, Lines<T> ln,
                PcgState *st, const double *__restrict__ partials, TriGate g, int nr, int N, int G)
{
    __shared__ double red[RED_SLOTS];
    extern __shared__ char smem_raw[];
    const int npad = nr + nr / 32 + 1;
    T *lc = reinterpret_cast<T *>(smem_raw);
    T *ld = lc + npad;
    T *lw = ld + npad;
    T *te = lw + npad;       // [MT][G], then the solution
    T *tg = te + MT * G;     // [MT][G]
    const int l0 = xcd_swizzle(blockIdx.x, N / MT) * MT;
    for (int i = threadIdx.x; i < nr; i += blockDim.x) {
        const int a = LdsLines<T>::at(i);
        lc[a] = ln.cb[i];
        ld[a] = ln.db[i];
        lw[a] = ln.rw[i];
    }
    // MT consecutive modes of strip s are MT * sizeof(T) contiguous bytes:
    // 16-byte pieces (MT * sizeof(T) is 32 in both precisions)
    constexpr int VW = 16 / (int)sizeof(T), NV = MT / VW;
    typedef T V __attribute__((ext_vector_type(VW)));
    for (int e = threadIdx.x; e < G * NV; e += blockDim.x) {
        const int s = e / NV, u = (e - s * NV) * VW;
        const V ve = *reinterpret_cast<const V *>(red_e + (size_t)s * N + l0 + u);
        const V vg = *reinterpret_cast<const V *>(red_g + (size_t)s * N + l0 + u);
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            te[(u + k) * G + s] = ve[k];
            tg[(u + k) * G + s] = vg[k];
        }
    }
    if (g.mode != 0 && tridiag_gate(st, partials, g, red, blockIdx.x) != ST_RUN) return;
    __syncthreads();
    const LdsLines<T> ll{lc, ld, lw};
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int S = G < 64 ? G : 64;
    const int lo = lane < S ? (int)(((long)lane * G) / S) : G;
    const int hi = lane < S ? (int)(((long)(lane + 1) * G) / S) : G;
    const int m = hi - lo;
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
    __syncthreads();   // every wave has read its te row
#pragma unroll
    for (int k = 0; k < LMAX; ++k)
        if (k < m) te[w * G + lo + k] = xs[k];
    __syncthreads();
    for (int e2 = threadIdx.x; e2 < G * NV; e2 += blockDim.x) {
        const int s = e2 / NV, u = (e2 - s * NV) * VW;
        V vx;
#pragma unroll
        for (int k = 0; k < VW; ++k) vx[k] = te[(u + k) * G + s];
        *reinterpret_cast<V *>(red_x + (size_t)s * N + l0 + u) = vx;
    }
}

// ---------------------------------------------------------------------------
// K3
// ---------------------------------------------------------------------------
template <typename T, int BC, int MODE, int R2, int R>
__global__ void __launch_bounds__(64 * R)
k_strip_inv(const T *__restrict__ fprime, const T *__restrict__ red_x, double *__restrict__ zout,
            const double *__restrict__ r, const PcgState *st, double *__restrict__ partials, bool pr,
            const typename vec2_of<T>::type *__restrict__ tw, const typename vec2_of<T>::type *__restrict__ pt,
            Lines<T> ln, int nr, double *__restrict__ dinc, double tau, double rho2)
{
    using Gm = wfft::Geo<R2>;
    constexpr int N = Gm::N, PITCH = 2 * Gm::LB, n = R - 1, NT = 64 * R;
    if (MODE != 0 && st->done) return;
    extern __shared__ char smem_raw[];
    T *tile = reinterpret_cast<T *>(smem_raw);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int s = blockIdx.x, i0 = s * R;
    // PCG modes: this wave's r row is loaded first, so that its latency
    // overlaps the back substitution (where it fits in registers)
    constexpr bool PRE = (MODE == 1 || MODE == 2) && R2 <= 8;
    double2 rpre[PRE ? R2 : 1];
    if constexpr (PRE) {
#pragma unroll
        for (int t = 0; t < R2; ++t)
            rpre[t] = *reinterpret_cast<const double2 *>(r + (size_t)(i0 + wv) * N + 2 * lane + 128 * t);
    }
    // f' of the interior rows into the tile, 16 bytes per access
    constexpr int VW = 16 / (int)sizeof(T);
    typedef T V __attribute__((ext_vector_type(VW)));
    for (int e = threadIdx.x; e < n * (N / VW); e += NT) {
        const int t = e / (N / VW), k = (e - t * (N / VW)) * VW;
        const V v = *reinterpret_cast<const V *>(fprime + (size_t)(i0 + t) * N + k);
#pragma unroll
        for (int u = 0; u < VW; ++u) tile[t * PITCH + k + u] = v[u];
    }
    T cbv[R], dbv[R], rwv[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
        cbv[t] = ln.cb[i0 + t];
        dbv[t] = ln.db[i0 + t];
        rwv[t] = ln.rw[i0 + t];
    }
    const T cbm = s > 0 ? ln.cb[i0 - 1] : (T)0;
    __syncthreads();
    for (int l = threadIdx.x; l < N; l += NT) {
        const T lam = ln.lam[l];
        const T Xs = red_x[(size_t)s * N + l];
        const T Xp = s > 0 ? red_x[(size_t)(s - 1) * N + l] : (T)0;
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

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
template <typename T>
Lines<T> lines_of(const Operator &op);
template <>
Lines<float> lines_of<float>(const Operator &op) { return {op.cb32, op.db32, op.rw32, op.lam32}; }
template <>
Lines<double> lines_of<double>(const Operator &op) { return {op.cb64, op.db64, op.rw64, op.lam64}; }

template <typename T>
const typename vec2_of<T>::type *tw_of(const Operator &op);
template <>
const float2 *tw_of<float>(const Operator &op) { return op.tw32; }
template <>
const double2 *tw_of<double>(const Operator &op) { return op.tw64; }
template <typename T>
const typename vec2_of<T>::type *pt_of(const Operator &op);
template <>
const float2 *pt_of<float>(const Operator &op) { return op.pt32; }
template <>
const double2 *pt_of<double>(const Operator &op) { return op.pt64; }

template <typename T>
struct RedBufs {
    T *e, *g, *x;
};
template <typename T>
RedBufs<T> red_bufs(const Operator &op, int R)
{
    T *b = static_cast<T *>(op.strip_red);
    const size_t gn = (size_t)(op.nr / R) * op.nz;
    return {b, b + gn, b + 2 * gn};
}

// modes per reduced-system workgroup: 32 bytes of each strip's row
template <typename T>
constexpr int red_mt() { return 32 / (int)sizeof(T); }

// Dynamic LDS above the default 64 KiB needs the kernel's attribute, set
// once per kernel.
void allow_lds(const void *fn, size_t bytes, bool &done)
{
    if (done || bytes <= 65536) return;
    AXI_CHECK_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    done = true;
}

template <typename T, int BC, int R2, int R>
void fwd_r(const Operator &op, const ZfwdArgs &a, hipStream_t s)
{
    const RedBufs<T> rb = red_bufs<T>(op, R);
    const dim3 grid(op.nr / R), block(64 * R);
    const size_t shm = (size_t)R * wfft::Geo<R2>::LB * sizeof(cx<T>);
    if (a.fused)
        hipLaunchKernelGGL((k_strip_fwd<T, BC, true, R2, R>), grid, block, shm, s, nullptr, a.x, a.r, a.p, a.q,
                           a.state, op.partials, a.n_pq, (T *)op.spec, rb.e, rb.g, tw_of<T>(op), pt_of<T>(op),
                           lines_of<T>(op), op.nr);
    else
        hipLaunchKernelGGL((k_strip_fwd<T, BC, false, R2, R>), grid, block, shm, s, a.rin, nullptr, nullptr,
                           nullptr, nullptr, a.state, op.partials, 0, (T *)op.spec, rb.e, rb.g, tw_of<T>(op),
                           pt_of<T>(op), lines_of<T>(op), op.nr);
    AXI_CHECK_HIP(hipGetLastError());
}

template <typename T, int BC, int R2, int R>
void inv_r(const Operator &op, const ZinvArgs &a, hipStream_t s)
{
    const RedBufs<T> rb = red_bufs<T>(op, R);
    const dim3 grid(op.nr / R), block(64 * R);
    const size_t shm = (size_t)R * wfft::Geo<R2>::LB * sizeof(cx<T>);
    const T *fp = (const T *)op.spec;
    const auto tw = tw_of<T>(op);
    const auto pt = pt_of<T>(op);
    const Lines<T> ln = lines_of<T>(op);
#define AXI_SINV(MD, Z, RR, ST, PR, D)                                                                           \
    hipLaunchKernelGGL((k_strip_inv<T, BC, MD, R2, R>), grid, block, shm, s, fp, rb.x, Z, RR, ST, op.partials,  \
                       PR, tw, pt, ln, op.nr, D, a.tau, a.rho2)
    switch (a.mode) {
    case 0: AXI_SINV(0, a.zout, nullptr, nullptr, false, nullptr); break;
    case 1: AXI_SINV(1, a.zout, a.r, a.state, a.pr, nullptr); break;
    case 2: AXI_SINV(2, a.zout, a.r, a.state, false, nullptr); break;
    case 3: AXI_SINV(3, nullptr, nullptr, a.state, false, a.d); break;
    default: AXI_SINV(4, nullptr, nullptr, a.state, false, a.d); break;
    }
#undef AXI_SINV
    AXI_CHECK_HIP(hipGetLastError());
}

template <typename T, int R, int LM>
void red_launch(const Operator &op, const TriGate &g, hipStream_t s)
{
    constexpr int MT = red_mt<T>();
    const RedBufs<T> rb = red_bufs<T>(op, R);
    const int G = op.nr / R;
    const size_t shm = strip_red_lds<T, MT>(op.nr, G);
    static bool lds_set = false;
    allow_lds(reinterpret_cast<const void *>(&k_strip_reduced<T, R, LM, MT>), shm, lds_set);
    hipLaunchKernelGGL((k_strip_reduced<T, R, LM, MT>), dim3(op.nz / MT), dim3(64 * MT), shm, s, rb.e, rb.g, rb.x,
                       lines_of<T>(op), g.state, op.partials, g, op.nr, op.nz, G);
    AXI_CHECK_HIP(hipGetLastError());
}

template <typename T, int R>
void red_r(const Operator &op, const TriGate &g, hipStream_t s)
{
    const int per = (op.nr / R + 63) / 64;
    if (per <= 1) red_launch<T, R, 1>(op, g, s);
    else if (per <= 2) red_launch<T, R, 2>(op, g, s);
    else if (per <= 4) red_launch<T, R, 4>(op, g, s);
    else if (per <= 8) red_launch<T, R, 8>(op, g, s);
    else red_launch<T, R, 16>(op, g, s);
}

template <typename T>
int strip_r2(int nz)
{
    switch (nz) {
    case 256: return 2;
    case 512: return 4;
    case 1024: return 8;
    case 2048: return sizeof(T) == 4 ? 16 : 0;   // FP64 at 2048 would spill
    default: return 0;
    }
}

template <typename T, int BC, int R>
void fwd_rb(const Operator &op, const ZfwdArgs &a, hipStream_t s)
{
    switch (op.nz) {
    case 256: fwd_r<T, BC, 2, R>(op, a, s); break;
    case 512: fwd_r<T, BC, 4, R>(op, a, s); break;
    case 1024: fwd_r<T, BC, 8, R>(op, a, s); break;
    default:
        if constexpr (sizeof(T) == 4) fwd_r<T, BC, 16, R>(op, a, s);
        break;
    }
}

template <typename T, int BC, int R>
void inv_rb(const Operator &op, const ZinvArgs &a, hipStream_t s)
{
    switch (op.nz) {
    case 256: inv_r<T, BC, 2, R>(op, a, s); break;
    case 512: inv_r<T, BC, 4, R>(op, a, s); break;
    case 1024: inv_r<T, BC, 8, R>(op, a, s); break;
    default:
        if constexpr (sizeof(T) == 4) inv_r<T, BC, 16, R>(op, a, s);
        break;
    }
}

template <typename T>
void fwd_t(const Operator &op, int rows, const ZfwdArgs &a, hipStream_t s)
{
    const bool dir = op.bc_z == DIR;
    if (rows == 8) {
        if (dir) fwd_rb<T, DIR, 8>(op, a, s);
        else fwd_rb<T, AXIPCG_Z_NEUMANN, 8>(op, a, s);
    } else {
        if (dir) fwd_rb<T, DIR, 4>(op, a, s);
        else fwd_rb<T, AXIPCG_Z_NEUMANN, 4>(op, a, s);
    }
}

template <typename T>
void inv_t(const Operator &op, int rows, const ZinvArgs &a, hipStream_t s)
{
    const bool dir = op.bc_z == DIR;
    if (rows == 8) {
        if (dir) inv_rb<T, DIR, 8>(op, a, s);
        else inv_rb<T, AXIPCG_Z_NEUMANN, 8>(op, a, s);
    } else {
        if (dir) inv_rb<T, DIR, 4>(op, a, s);
        else inv_rb<T, AXIPCG_Z_NEUMANN, 4>(op, a, s);
    }
}

template <typename T>
bool usable_t(const Operator &op, int R)
{
    if (R != 4 && R != 8) return false;
    if (strip_r2<T>(op.nz) == 0 || op.nr % R != 0) return false;
    const int G = op.nr / R;
    return G >= 1 && G <= 1024 && strip_red_lds<T, red_mt<T>()>(op.nr, G) <= 160 * 1024;
}

}  // namespace

// The strip path serves an operator and precision with strips of `rows`
// rows (4 or 8) when the one-wave transforms cover nz, the rows split into
// such strips and the reduced system fits one wavefront's registers (at most
// 1024 strips) and its workgroup's LDS.
bool strip_usable(const Operator &op, int prec, int rows)
{
    if (!op.strip_red) return false;
    return prec == AXIPCG_PREC_FP32 ? usable_t<float>(op, rows) : usable_t<double>(op, rows);
}

// Reduced data for strips of 4 rows (the larger of the two heights' needs).
size_t strip_red_bytes(int nr, int nz)
{
    return (nr % 4 == 0) ? 3 * (size_t)(nr / 4) * nz * sizeof(double) : 0;
}

void strip_fwd(const Operator &op, int prec, int rows, const ZfwdArgs &a, hipStream_t s)
{
    if (prec == AXIPCG_PREC_FP32) fwd_t<float>(op, rows, a, s);
    else fwd_t<double>(op, rows, a, s);
}

void strip_reduced(const Operator &op, int prec, int rows, const TriGate &g, hipStream_t s)
{
    if (prec == AXIPCG_PREC_FP32) {
        if (rows == 8) red_r<float, 8>(op, g, s);
        else red_r<float, 4>(op, g, s);
    } else {
        if (rows == 8) red_r<double, 8>(op, g, s);
        else red_r<double, 4>(op, g, s);
    }
}

void strip_inv(const Operator &op, int prec, int rows, const ZinvArgs &a, hipStream_t s)
{
    if (prec == AXIPCG_PREC_FP32) inv_t<float>(op, rows, a, s);
    else inv_t<double>(op, rows, a, s);
}

}  // namespace axipcg
