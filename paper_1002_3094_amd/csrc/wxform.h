// Shared device code of the preconditioner's kernels (§4.2 eqs. (36)-(39)):
// the one-wavefront z-transforms of a row with pluggable output / input (a
// global row, or a row of a workgroup's LDS tile), the Chebyshev parameters
// of eq. (8), and the stop test that opens the r-solve launch in PCG mode.
#pragma once

#include "kernels.h"
#include "wfft.h"

namespace axipcg {
namespace {

constexpr int DIR = AXIPCG_Z_DIRICHLET;

// Row views for the transform bodies.
template <typename T>
struct RowStore {
    T *row;
    __device__ void operator()(int j, T v) const { row[j] = v; }
};
template <typename T>
struct RowLoad {
    const T *row;
    __device__ T operator()(int j) const { return row[j]; }
};

template <typename T> __device__ inline T fast_rcp(T x);
template <> __device__ inline float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ inline double fast_rcp<double>(double x) { return 1.0 / x; }
// alpha_m of eq. (8) with Chebyshev parameters: alpha_1 = 1,
// alpha_2 = 2 / (2 - rho0^2), alpha_{k+1} = 4 / (4 - rho0^2 alpha_k).
__device__ inline double cheb_alpha(int m, double rho2)
{
    if (m <= 1) return 1.0;
    double a = 2.0 / (2.0 - rho2);
    for (int k = 2; k < m; ++k) a = 4.0 / (4.0 - rho2 * a);
    return a;
}
// ---------------------------------------------------------------------------
// One-wavefront-per-row transforms for N = 128 R2 (R2 = 2, 4, 8, 16): the
// sequence v of Makhoul's reordering, read as M = N/2 complex numbers
// z[n] = v[2n] + i v[2n+1], is transformed with one length-M FFT (wfft.h)
// and split into the length-N spectrum of v:
//     V_m = (Z_m + conj Z_{M-m}) / 2 - i w_N^m (Z_m - conj Z_{M-m}) / 2,
// V_{N-m} = conj V_m.  Each wave owns one row; the workgroup's WR waves meet
// only for the partial sums.  Lane l loads and stores the element pairs
// (2 l + 128 t, 2 l + 128 t + 1), t < R2, as 16-byte vectors.
// ---------------------------------------------------------------------------
template <typename T, int R2>
constexpr int wave_rows() { return (sizeof(T) == 8 && R2 >= 16) ? 2 : 4; }

// A flag as one value for the whole workgroup (thread 0 reads it), for bodies
// whose workgroup goes on to other work after they return: waves that read
// different values would next meet at different barriers.
__device__ inline int wg_flag(const int *p)
{
    __shared__ int f;
    if (threadIdx.x == 0) f = *(const volatile int *)p;
    __syncthreads();
    const int v = f;
    __syncthreads();
    return v;
}

// Forward transform of row `row` by the calling wave (rows >= nr: the wave
// runs for the partial sums only).  Every wave of the workgroup calls it
// (block-wide reductions).  The spectrum leaves through store(j, value) for
// each index j of the row, after the wave's last read of its LDS slice, so
// the store may write into that slice.  Returns false when the solve has
// stopped (or the step broke down): the whole workgroup then returns.
template <typename T, int BC, bool FUSED, int R2, bool WG_STOP = false, typename Store>
__device__ __forceinline__ bool
zfwd_w_body(const double *__restrict__ rin, double *__restrict__ x, double *__restrict__ r,
            const double *__restrict__ p, const double *__restrict__ q, PcgState *st,
            double *__restrict__ partials, int n_pq,
            const typename vec2_of<T>::type *__restrict__ tw, const typename vec2_of<T>::type *__restrict__ pt,
            int nr, int row, int blk, const Store &store)
{
    using G = wfft::Geo<R2>;
    constexpr int M = G::M, N = G::N, U = G::U;
    extern __shared__ char smem_raw[];
    __shared__ double red[RED_SLOTS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw) + wv * G::LB;
    T *fbuf = reinterpret_cast<T *>(buf);
    const bool valid = row < nr;
    const size_t base = (size_t)(valid ? row : nr - 1) * N + 2 * lane;

    // every global read first: the row (and the PCG vectors), the twiddles
    double2 rv[R2], xv[R2], pv[R2], qv[R2];
#pragma unroll
    for (int t = 0; t < R2; ++t) {
        if (FUSED) {
            xv[t] = *reinterpret_cast<const double2 *>(x + base + 128 * t);
            rv[t] = *reinterpret_cast<const double2 *>(r + base + 128 * t);
            pv[t] = *reinterpret_cast<const double2 *>(p + base + 128 * t);
            qv[t] = *reinterpret_cast<const double2 *>(q + base + 128 * t);
        } else {
            rv[t] = *reinterpret_cast<const double2 *>(rin + base + 128 * t);
        }
    }
    wfft::Twiddles<T, R2> twd;
    twd.load(tw, lane);
    cx<T> wN[U][8], cP[U][8];   // w_N^m and exp(-i pi m / 2N) of this lane's outputs
#pragma unroll
    for (int j = 0; j < U; ++j)
#pragma unroll
        for (int k0 = 0; k0 < 8; ++k0) {
            const int m = wfft::out_index<R2>(lane, j, k0) & (M - 1);
            wN[j][k0] = ld_tw<T>(tw, m);
            cP[j][k0] = ld_tw<T>(pt, m);
        }
    // (the stop flag before the reduction: deferring it past the reduction,
    // as the other PCG kernels do, made the 2048-point forward kernel slower)
    if constexpr (WG_STOP) {
        if (st && wg_flag(&st->done)) return false;
    } else {
        if (st && st->done) return false;
    }
    double alpha = 0.0;
    if (FUSED) {
        const int k_it = st->iters;
        // both r.z slots read now: the loads overlap the reduction
        const double rho_slot[2] = {st->rho[0], st->rho[1]};
        const double pq = block_total(partials + SLOT_PQ * MAX_PARTIALS, n_pq, red);
        if (!(pq > 0.0) || !(pq < 1e308)) {
            if (blk == 0 && threadIdx.x == 0) st->done = ST_BREAK;
            return false;
        }
        alpha = rho_slot[k_it & 1] / pq;
        if (blk == 0 && threadIdx.x == 0) st->cur = k_it;
    }

    // r update, Makhoul reordering into the slice (even k -> v[k/2], odd k -> v[N-1-(k-1)/2])
    double rr = 0.0;
#pragma unroll
    for (int t = 0; t < R2; ++t) {
        double2 rn = rv[t];
        if (FUSED) {
            double2 xn;
            xn.x = xv[t].x + alpha * pv[t].x;
            xn.y = xv[t].y + alpha * pv[t].y;
            rn.x = rv[t].x - alpha * qv[t].x;
            rn.y = rv[t].y - alpha * qv[t].y;
            if (valid) {
                *reinterpret_cast<double2 *>(x + base + 128 * t) = xn;
                *reinterpret_cast<double2 *>(r + base + 128 * t) = rn;
                rr += rn.x * rn.x + rn.y * rn.y;
            }
        }
        const int sv = lane + 64 * t;
        fbuf[wfft::fslot(sv)] = (T)rn.x;
        fbuf[wfft::fslot(N - 1 - sv)] = (BC == DIR) ? -(T)rn.y : (T)rn.y;   // sine: y_k = (-1)^k x_k
    }
    wfft::wave_fence();
    cx<T> a[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) a[n2] = buf[wfft::vslot(lane + 64 * n2)];
    cx<T> X[U][8];
    wfft::fft<T, R2>(a, X, buf, twd, lane);

    // split: the partner of Z_m is Z_{M-m}, exchanged through the slice
#pragma unroll
    for (int j = 0; j < U; ++j)
        if (wfft::unit_active<R2>(lane + 64 * j))
#pragma unroll
            for (int k0 = 0; k0 < 8; ++k0) buf[wfft::vslot(wfft::out_index<R2>(lane, j, k0))] = X[j][k0];
    wfft::wave_fence();
    const T nrm = (T)sqrt(2.0 / N);
    const T half = (T)0.70710678118654752440;
    T ya[U][8], yb[U][8];   // Y_m and Y_{N-m} (Y_M for m = 0), normalised
#pragma unroll
    for (int j = 0; j < U; ++j) {
        if (!wfft::unit_active<R2>(lane + 64 * j)) continue;
#pragma unroll
        for (int k0 = 0; k0 < 8; ++k0) {
            const int m = wfft::out_index<R2>(lane, j, k0);
            const cx<T> Zm = X[j][k0];
            T Ym, YNm;
            if (m == 0) {
                Ym = Zm.x + Zm.y;
                YNm = (Zm.x - Zm.y) * half;
            } else {
                const cx<T> Zp = buf[wfft::vslot(M - m)];
                const cx<T> sum = {Zm.x + Zp.x, Zm.y - Zp.y};        // Z_m + conj Z_{M-m}
                const cx<T> dif = {Zm.x - Zp.x, Zm.y + Zp.y};        // Z_m - conj Z_{M-m}
                const cx<T> wd = cmul(wN[j][k0], dif);
                const cx<T> V = {(T)0.5 * (sum.x + wd.y), (T)0.5 * (sum.y - wd.x)};
                const cx<T> cv = cmul(cP[j][k0], V);
                Ym = cv.x;
                YNm = -cv.y;
            }
            ya[j][k0] = nrm * ((m == 0) ? half : (T)1) * Ym;
            yb[j][k0] = nrm * YNm;
        }
    }
    wfft::wave_fence();   // every read of the slice is done: the store may reuse it
    if (valid) {
#pragma unroll
        for (int j = 0; j < U; ++j) {
            if (!wfft::unit_active<R2>(lane + 64 * j)) continue;
#pragma unroll
            for (int k0 = 0; k0 < 8; ++k0) {
                const int m = wfft::out_index<R2>(lane, j, k0);
                const int mN = (m == 0) ? M : N - m;
                store((BC == DIR) ? N - 1 - m : m, ya[j][k0]);
                store((BC == DIR) ? N - 1 - mN : mN, yb[j][k0]);
            }
        }
    }
    if (FUSED) {
        const double s = block_sum(rr, red);
        if (threadIdx.x == 0) partials[SLOT_RR * MAX_PARTIALS + blk] = s;
    }
    return true;
}

// Inverse transform of row `row` by the calling wave: the spectral value of
// index j comes from ld(j) (all of them are read before the wave's FFT uses
// its LDS slice, so ld may read from that slice); z (or, in the Chebyshev
// modes, the increment d) is written to global memory.  Every wave of the
// workgroup calls it (block-wide reductions).
// `rpre`, when given, holds this lane's r values of the row (the element
// pairs the body would load, t < R2), already loaded by the caller.
template <typename T, int BC, int MODE, int R2, typename Load>
__device__ __forceinline__ void
zinv_w_body(const Load &ld, double *__restrict__ zout, const double *__restrict__ r,
            const PcgState *st, double *__restrict__ partials, bool pr,
            const typename vec2_of<T>::type *__restrict__ tw, const typename vec2_of<T>::type *__restrict__ pt,
            int nr, double *__restrict__ dinc, double tau, double rho2, int row, int blk,
            const double2 *rpre = nullptr)
{
    constexpr bool PCGM = (MODE == 1 || MODE == 2);
    constexpr bool CHEB = (MODE == 3 || MODE == 4);
    using G = wfft::Geo<R2>;
    constexpr int M = G::M, N = G::N, U = G::U;
    extern __shared__ char smem_raw[];
    __shared__ double red[RED_SLOTS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw) + wv * G::LB;
    const T *fbuf = reinterpret_cast<const T *>(buf);
    const bool valid = row < nr;
    const int rowc = valid ? row : nr - 1;
    const size_t base = (size_t)rowc * N + 2 * lane;

    // spectral values Y_m, Y_{N-m}, Y_{M-m}, Y_{M+m} for m = lane + 64 n2
    // (unnormalised DCT-II coefficients of y; Y_N = 0)
    const T isc = (T)sqrt(0.5 * N);
    const T sq2 = (T)1.41421356237309504880;
    auto yidx = [&](int m) { return (BC == DIR) ? N - 1 - m : m; };
    T y0[R2], y1[R2], y2[R2], y3[R2];
    cx<T> cm[R2], cq[R2], wm[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
        const int m = lane + 64 * n2;
        y0[n2] = ld(yidx(m));
        y1[n2] = ld(yidx(m == 0 ? M : N - m));   // (m = 0: unused)
        y2[n2] = ld(yidx(M - m));
        y3[n2] = ld(yidx(M + m == N ? M : M + m));
        cm[n2] = ld_tw<T>(pt, m);
        cq[n2] = ld_tw<T>(pt, M - m);
        wm[n2] = ld_tw<T>(tw, m);
    }
    wfft::Twiddles<T, R2> twd;
    twd.load(tw, lane);
    double2 rv[R2], zo[R2], dv[R2];
#pragma unroll
    for (int t = 0; t < R2; ++t) {
        if (PCGM) {
            rv[t] = rpre ? rpre[t] : *reinterpret_cast<const double2 *>(r + base + 128 * t);
            if (pr) zo[t] = *reinterpret_cast<const double2 *>(zout + base + 128 * t);
        }
        if (MODE == 3) dv[t] = *reinterpret_cast<const double2 *>(dinc + base + 128 * t);
    }
    if (MODE != 0 && st->done) return;
    double c1 = 0.0, c2 = 0.0;
    if (CHEB) {
        const double alpha = cheb_alpha(st->iters + 1, rho2);
        c1 = alpha - 1.0;
        c2 = alpha * tau;
    }

    // Z'_m = E_m + i O_m with E_m = (V_m + V_{m+M}) / 2, O_m = w_N^{-m} (V_m - V_{m+M}) / 2,
    // V_m = exp(i pi m / 2N) (Y_m - i Y_{N-m}); the FFT runs on its conjugate
    cx<T> a[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
        const int m = lane + 64 * n2;
        const auto edge = [&](int mm) { return yidx(mm) == ((BC == DIR) ? N - 1 : 0); };
        const T Ym = y0[n2] * isc * (edge(m) ? sq2 : (T)1);
        const T YMm = y2[n2] * isc * (edge(M - m) ? sq2 : (T)1);
        cx<T> Vm, Vp;   // V_m, V_{m+M}
        if (m == 0) {
            Vm = {Ym, (T)0};
            Vp = {sq2 * YMm, (T)0};
        } else {
            const T YNm = y1[n2] * isc;
            const T YMp = y3[n2] * isc;
            Vm = cmul<T>({cm[n2].x, -cm[n2].y}, {Ym, -YNm});
            const cx<T> Vq = cmul<T>({cq[n2].x, -cq[n2].y}, {YMm, -YMp});   // V_{M-m}
            Vp = {Vq.x, -Vq.y};
        }
        const cx<T> E = {(T)0.5 * (Vm.x + Vp.x), (T)0.5 * (Vm.y + Vp.y)};
        const cx<T> O = cmul<T>({wm[n2].x, -wm[n2].y}, {(T)0.5 * (Vm.x - Vp.x), (T)0.5 * (Vm.y - Vp.y)});
        a[n2] = {E.x - O.y, -(E.y + O.x)};
    }
    cx<T> X[U][8];
    wfft::fft<T, R2>(a, X, buf, twd, lane);

    // z = conj(X) / M as v[2k] + i v[2k+1]; back to y through the slice
    const T invM = (T)1 / (T)M;
#pragma unroll
    for (int j = 0; j < U; ++j)
        if (wfft::unit_active<R2>(lane + 64 * j))
#pragma unroll
            for (int k0 = 0; k0 < 8; ++k0)
                buf[wfft::vslot(wfft::out_index<R2>(lane, j, k0))] = {X[j][k0].x * invM, -X[j][k0].y * invM};
    wfft::wave_fence();
    double rz = 0.0, rzo = 0.0;
#pragma unroll
    for (int t = 0; t < R2; ++t) {
        const int sv = lane + 64 * t;
        double2 zv;
        zv.x = (double)fbuf[wfft::fslot(sv)];
        const T yo = fbuf[wfft::fslot(N - 1 - sv)];
        zv.y = (double)((BC == DIR) ? -yo : yo);
        if (!valid) continue;
        double *dst = (CHEB ? dinc : zout) + base + 128 * t;
        if (PCGM) {
            if (pr) rzo += rv[t].x * zo[t].x + rv[t].y * zo[t].y;
            rz += rv[t].x * zv.x + rv[t].y * zv.y;
        }
        if (CHEB) {
            double2 d;
            d.x = (MODE == 4) ? c2 * zv.x : c1 * dv[t].x + c2 * zv.x;
            d.y = (MODE == 4) ? c2 * zv.y : c1 * dv[t].y + c2 * zv.y;
            *reinterpret_cast<double2 *>(dst) = d;
        } else {
            *reinterpret_cast<double2 *>(dst) = zv;
        }
    }
    if (PCGM) {
        const double s = block_sum(rz, red);
        if (threadIdx.x == 0) partials[SLOT_RZ * MAX_PARTIALS + blk] = s;
        if (pr) {
            const double so = block_sum(rzo, red);
            if (threadIdx.x == 0) partials[SLOT_RZOLD * MAX_PARTIALS + blk] = so;
        }
    }
}

// Gate of the r-solve launch in PCG mode: returns the stop status (ST_RUN to
// go on).  Workgroup 0 records it.
// Publish a solve's progress to the host (one thread).
__device__ inline void publish(HostMirror *m, unsigned seq, double rr, double bb, int iters, int done)
{
    m->rr = rr;
    m->bb = bb;
    __threadfence_system();
    *reinterpret_cast<volatile unsigned long long *>(&m->word) = mirror_word(seq, iters, done);
}

// The loads of a PCG step's gate (mode 1): the state fields and the first
// round of the ||r||^2 partials, issued before the launch stages its own
// data so that the two latencies overlap.
struct GatePre {
    TotalLoads rr;
    int done, cur, maxit;
    double tol2;
};

__device__ inline void gate_issue(const PcgState *st, const double *__restrict__ partials, const TriGate &g,
                                  GatePre &p)
{
    p.done = st->done;
    p.cur = st->cur;
    p.maxit = st->maxit;
    p.tol2 = st->tol2;
    total_issue(partials + SLOT_RR * MAX_PARTIALS, g.n_rr, p.rr);
}

__device__ inline int tridiag_gate(PcgState *st, const double *__restrict__ partials, const TriGate &g, double *red,
                                   int vb, const GatePre *pre = nullptr)
{
    if (g.mode == 1) {
        // every state field read at once, their latency overlapping the
        // reduction
        GatePre loc;
        if (!pre) {
            gate_issue(st, partials, g, loc);
            pre = &loc;
        }
        const int done = pre->done, k_it = pre->cur, maxit = pre->maxit;
        const double tol2 = pre->tol2;
        const double rr = total_finish(partials + SLOT_RR * MAX_PARTIALS, g.n_rr, pre->rr, red);
        if (done) return done;   // stopped earlier: leave the state alone
        int status = ST_RUN;
        if (!(rr == rr) || rr > 1e300) status = ST_BREAK;
        else if (rr <= tol2) status = ST_CONV;
        else if (k_it + 1 >= maxit) status = ST_MAXIT;
        if (vb == 0 && threadIdx.x == 0) {
            st->rr = rr;
            st->iters = k_it + 1;
            st->done = status;
            if (g.mirror && (status != ST_RUN || g.report)) publish(g.mirror, g.seq, rr, st->bb, k_it + 1, status);
        }
        return status;
    }
    const double rr = block_total(partials + SLOT_RR * MAX_PARTIALS, g.n_rr, red);
    const double bb = block_total(partials + SLOT_MISC * MAX_PARTIALS, g.n_rr, red);
    const double tol2 = g.rtol2 * bb;
    int status = ST_RUN;
    if (bb == 0.0) status = ST_BZERO;
    else if (!(rr == rr) || rr > 1e300) status = ST_BREAK;
    else if (rr <= tol2) status = ST_CONV;
    if (vb == 0 && threadIdx.x == 0) {
        st->rr = rr;
        st->bb = bb;
        st->tol2 = tol2;
        st->iters = 0;
        st->cur = 0;
        st->maxit = g.maxit;
        st->flags = g.flags;
        st->done = status;
        if (g.mirror && (status != ST_RUN || g.report)) publish(g.mirror, g.seq, rr, bb, 0, status);
    }
    return status;
}

}  // namespace
}  // namespace axipcg
