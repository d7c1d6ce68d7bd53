// Device bodies of the PCG step's SpMV (§2.2 eq. (8) with conjugate-
// gradient parameters; the operator of §2.1) that more than one launch form
// shares: the 5-point r-weighted stencil, the tiled SpMV with the p update
// and p.q partials, and the start r = b - A x.  Each body takes its work
// item (vb, of vnb) as an argument.
#pragma once

#include "kernels.h"

namespace axipcg {
namespace {

// 5-point stencil of the r-weighted scheme at (i, k) applied to the field
// returned by `val(offset)`.
template <typename F>
__device__ inline double stencil(const double *__restrict__ D, const double *__restrict__ CR,
                                 const double *__restrict__ CZ, size_t e, int i, int k, int nr, int nz, F val)
{
    double v = D[e] * val(0);
    if (i + 1 < nr) v -= CR[e] * val((long)nz);
    if (i > 0) v -= CR[e - nz] * val(-(long)nz);
    if (k + 1 < nz) v -= CZ[e] * val(1);
    if (k > 0) v -= CZ[e - 1] * val(-1);
    return v;
}

struct Pair { double a, b; };

__device__ inline Pair ld2(const double *p) { const double2 v = *reinterpret_cast<const double2 *>(p); return {v.x, v.y}; }

// (A v) at the pair (e, e+1) of row i, columns k, k+1 (k even, k + 1 < nz)
__device__ inline Pair stencil2(const double *__restrict__ v, const double *__restrict__ D,
                                const double *__restrict__ CR, const double *__restrict__ CZ, size_t e, int i, int k,
                                int nr, int nz, const Pair &c)
{
    const Pair d = ld2(D + e), cz = ld2(CZ + e);
    Pair y{d.a * c.a, d.b * c.b};
    if (i + 1 < nr) {
        const Pair cr = ld2(CR + e), vn = ld2(v + e + nz);
        y.a -= cr.a * vn.a;
        y.b -= cr.b * vn.b;
    }
    if (i > 0) {
        const Pair cr = ld2(CR + e - nz), vn = ld2(v + e - nz);
        y.a -= cr.a * vn.a;
        y.b -= cr.b * vn.b;
    }
    // z-couplings: (k, k+1) inside the pair, k-1 and k+2 outside
    y.a -= cz.a * c.b;
    y.b -= cz.a * c.a;
    if (k + 2 < nz) y.b -= cz.b * v[e + 2];
    if (k > 0) y.a -= CZ[e - 1] * v[e - 1];
    return y;
}

// The SpMV step of PCG: rho_k, beta; p_new = z + beta p_old; q = A p_new;
// p_new . q partials.  A z and A p_old are formed first (no scalar needed),
// so the loads overlap the reduction of the r.z partials; q = A z + beta A
// p_old is the same product up to rounding (no recurrence: both terms are
// recomputed from the stored vectors every iteration).
//
// It runs on tiles of RW consecutive rows by
// SPMV_CHUNK columns: a thread owns one column pair and sweeps the tile's
// rows with a three-row window of z and p_old in registers (each row is
// loaded once per tile, plus one halo row above and below), and the
// z-neighbours k - 1, k + 2 (and the coupling CZ[k - 1]) come from the
// adjacent lanes, with loads only at the wave's edges.  The stencil's
// arithmetic is that of stencil2, term for term.  Tiles are dealt to the
// XCDs in contiguous runs (xcd_swizzle), so a tile's halo rows are the
// neighbouring tiles' rows in the same L2.  The tiles t = vb, vb + vnb, ...
// of the nb * nc of the problem; one p.q partial, in slot vb.
constexpr int SPMV_CHUNK = 512;   // columns per tile: 256 threads x one pair

template <bool PR, int RW>
__device__ __forceinline__ void spmv_tiles(const double *__restrict__ z, const double *__restrict__ pold,
                                           double *__restrict__ pnew, double *__restrict__ q,
                                           const double *__restrict__ D, const double *__restrict__ CR,
                                           const double *__restrict__ CZ, int nr, int nz, PcgState *st,
                                           double *__restrict__ partials, int n_rz, int vb, int vnb)
{
    __shared__ double red[8];
    double acc = 0.0, beta = 0.0;
    bool have_beta = false;
    int k_it = 0;
    const int nb = (nr + RW - 1) / RW, nc = (nz + SPMV_CHUNK - 1) / SPMV_CHUNK;
    const int lane = threadIdx.x & 63;
    // the first round of the r.z partials, issued ahead of the first tile's
    // rows so that the two reads are in flight together (not in the
    // Polak-Ribiere form, whose second sum would cost it a wave per SIMD)
    TotalLoads rz_pre;
    if constexpr (!PR) total_issue(partials + SLOT_RZ * MAX_PARTIALS, n_rz, rz_pre);
    for (int t = vb; t < nb * nc; t += vnb) {
        const int item = xcd_swizzle(t, nb * nc);
        const int i0 = RW * (item / nc);
        const int k = (item % nc) * SPMV_CHUNK + 2 * (int)threadIdx.x;
        const bool in = k < nz;
        // window: [0] row i - 1, [1] row i, [2] row i + 1; crm = CR of row i - 1
        Pair zw[3], pw[3], crm;
        {
            const size_t e = (size_t)i0 * nz + k;
            const bool dn = in && i0 > 0;
            zw[0] = dn ? ld2(z + e - nz) : Pair{0.0, 0.0};
            pw[0] = dn ? ld2(pold + e - nz) : Pair{0.0, 0.0};
            crm = dn ? ld2(CR + e - nz) : Pair{0.0, 0.0};
            zw[1] = in ? ld2(z + e) : Pair{0.0, 0.0};
            pw[1] = in ? ld2(pold + e) : Pair{0.0, 0.0};
        }
#pragma unroll
        for (int rr = 0; rr < RW; ++rr) {
            const int i = i0 + rr;
            if (i >= nr) break;
            const bool up = i + 1 < nr;
            const size_t e = (size_t)i * nz + k;
            zw[2] = (in && up) ? ld2(z + e + nz) : Pair{0.0, 0.0};
            pw[2] = (in && up) ? ld2(pold + e + nz) : Pair{0.0, 0.0};
            const Pair cr = (in && up) ? ld2(CR + e) : Pair{0.0, 0.0};
            const Pair d = in ? ld2(D + e) : Pair{0.0, 0.0};
            const Pair cz = in ? ld2(CZ + e) : Pair{0.0, 0.0};
            // every lane takes part in the shuffles (lanes past nz hold zeros)
            double zl = __shfl_up(zw[1].b, 1), pl = __shfl_up(pw[1].b, 1), czl = __shfl_up(cz.b, 1);
            double zr = __shfl_down(zw[1].a, 1), pr = __shfl_down(pw[1].a, 1);
            if (lane == 0 && in && k > 0) {
                zl = z[e - 1];
                pl = pold[e - 1];
                czl = CZ[e - 1];
            }
            if (lane == 63 && in && k + 2 < nz) {
                zr = z[e + 2];
                pr = pold[e + 2];
            }
            auto row = [&](const Pair &c, const Pair &vu, const Pair &vd, double vl, double vr) {
                Pair y{d.a * c.a, d.b * c.b};
                if (up) {
                    y.a -= cr.a * vu.a;
                    y.b -= cr.b * vu.b;
                }
                if (i > 0) {
                    y.a -= crm.a * vd.a;
                    y.b -= crm.b * vd.b;
                }
                y.a -= cz.a * c.b;
                y.b -= cz.a * c.a;
                if (k + 2 < nz) y.b -= cz.b * vr;
                if (k > 0) y.a -= czl * vl;
                return y;
            };
            const Pair az = row(zw[1], zw[2], zw[0], zl, zr);
            const Pair ap = row(pw[1], pw[2], pw[0], pl, pr);
            if (!have_beta) {   // scalars once per workgroup, after the first row's loads
                // every state field read at once (the r.z slot needed depends
                // on iters), their latency overlapping the reduction; the
                // stop flag is acted on after it (every workgroup alike)
                const int done = st->done;
                k_it = st->iters;
                const double rho_slot[2] = {st->rho[0], st->rho[1]};
                const double rho = PR ? block_total(partials + SLOT_RZ * MAX_PARTIALS, n_rz, red)
                                      : total_finish(partials + SLOT_RZ * MAX_PARTIALS, n_rz, rz_pre, red);
                if (done) return;
                if (k_it > 0) {
                    double num = rho;
                    if (PR) num -= block_total(partials + SLOT_RZOLD * MAX_PARTIALS, n_rz, red);
                    beta = num / rho_slot[(k_it - 1) & 1];
                }
                if (vb == 0 && threadIdx.x == 0) st->rho[k_it & 1] = rho;
                have_beta = true;
            }
            if (in) {
                double2 pn, qn;
                pn.x = (k_it > 0) ? zw[1].a + beta * pw[1].a : zw[1].a;
                pn.y = (k_it > 0) ? zw[1].b + beta * pw[1].b : zw[1].b;
                qn.x = (k_it > 0) ? az.a + beta * ap.a : az.a;
                qn.y = (k_it > 0) ? az.b + beta * ap.b : az.b;
                *reinterpret_cast<double2 *>(pnew + e) = pn;
                *reinterpret_cast<double2 *>(q + e) = qn;
                acc += pn.x * qn.x;
                acc += pn.y * qn.y;
            }
            zw[0] = zw[1];
            zw[1] = zw[2];
            pw[0] = pw[1];
            pw[1] = pw[2];
            crm = cr;
        }
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[SLOT_PQ * MAX_PARTIALS + vb] = s;
}

// Chebyshev step of eq. (8) in increment form: x += d, r -= A d, ||r||^2
// partials (rows vb, vb + vnb, ...; one partial, in slot vb, for the stop
// test of the r-solve launch); item 0 records the iteration being processed.
__device__ __forceinline__ void cheb_update_body(const double *__restrict__ d, double *__restrict__ x,
                                                 double *__restrict__ r, const double *__restrict__ D,
                                                 const double *__restrict__ CR, const double *__restrict__ CZ,
                                                 int nr, int nz, PcgState *st, double *__restrict__ partials, int vb,
                                                 int vnb)
{
    __shared__ double red[8];
    if (st->done) return;
    if (vb == 0 && threadIdx.x == 0) st->cur = st->iters;
    double acc = 0.0;
    for (int b = vb; b < nr; b += vnb) {
        const int i = xcd_swizzle(b, nr);
        for (int k = 2 * (int)threadIdx.x; k < nz; k += 2 * (int)blockDim.x) {
            const size_t e = (size_t)i * nz + k;
            const Pair dc = ld2(d + e);
            const Pair ad = stencil2(d, D, CR, CZ, e, i, k, nr, nz, dc);
            const Pair xc = ld2(x + e), rc = ld2(r + e);
            double2 xn, rn;
            xn.x = xc.a + dc.a;
            xn.y = xc.b + dc.b;
            rn.x = rc.a - ad.a;
            rn.y = rc.b - ad.b;
            *reinterpret_cast<double2 *>(x + e) = xn;
            *reinterpret_cast<double2 *>(r + e) = rn;
            acc += rn.x * rn.x + rn.y * rn.y;
        }
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[SLOT_RR * MAX_PARTIALS + vb] = s;
}

// r = b - A x; ||r||^2 and ||b||^2 partials.
__device__ __forceinline__ void init_body(const double *__restrict__ b, const double *__restrict__ x,
                                          double *__restrict__ r, const double *__restrict__ D,
                                          const double *__restrict__ CR, const double *__restrict__ CZ, int nr,
                                          int nz, double *__restrict__ partials, int vb, int vnb)
{
    __shared__ double red[8];
    double s_r = 0.0, s_b = 0.0;
    for (int blk = vb; blk < nr; blk += vnb) {
        const int i = xcd_swizzle(blk, nr);
        for (int k = threadIdx.x; k < nz; k += blockDim.x) {
            const size_t e = (size_t)i * nz + k;
            const double v = stencil(D, CR, CZ, e, i, k, nr, nz, [&](long o) { return x[e + o]; });
            const double bv = b[e];
            const double d = bv - v;
            r[e] = d;
            s_r += d * d;
            s_b += bv * bv;
        }
    }
    const double tb = block_sum(s_b, red);
    const double tr = block_sum(s_r, red);
    if (threadIdx.x == 0) {
        partials[SLOT_MISC * MAX_PARTIALS + vb] = tb;
        partials[SLOT_RR * MAX_PARTIALS + vb] = tr;
    }
}


// ---- work items of the batched launches ------------------------------------
// One item of a batched phase, `g` its index over the whole batch's items (a
// launch passes its workgroup index; the single-launch batch deals the items
// to its resident workgroups): an SpMV tile, or a row.
constexpr int BATCH_SPMV_RW = 16;   // rows per SpMV tile of a batch member

inline int batch_spmv_tiles(int nr, int nz)
{
    return ((nr + BATCH_SPMV_RW - 1) / BATCH_SPMV_RW) * ((nz + SPMV_CHUNK - 1) / SPMV_CHUNK);
}

template <bool PR>
__device__ __forceinline__ void b_spmv_item(const ProbDesc *__restrict__ d, int n, int g, int parity)
{
    const int p = find_problem(d, n, g, RANGE_SP);
    const ProbDesc &P = d[p];
    const double *pold = parity ? P.p1 : P.p0;
    double *pnew = parity ? P.p0 : P.p1;
    spmv_tiles<PR, BATCH_SPMV_RW>(P.z, pold, pnew, P.q, P.D, P.CR, P.CZ, P.nr, P.nz, P.state, P.partials, P.n_tr,
                                  g - P.sp_start, P.n_sp);
}

__device__ __forceinline__ void b_init_item(const ProbDesc *__restrict__ d, int n, int g)
{
    const int p = find_problem(d, n, g, RANGE_ROWS);
    const ProbDesc &P = d[p];
    init_body(P.b, P.x, P.r, P.D, P.CR, P.CZ, P.nr, P.nz, P.partials, g - P.row_start, P.nr);
}

// Chebyshev step on one row of a member (d in its p0 buffer).
__device__ __forceinline__ void b_cheb_item(const ProbDesc *__restrict__ d, int n, int g)
{
    const int p = find_problem(d, n, g, RANGE_ROWS);
    const ProbDesc &P = d[p];
    cheb_update_body(P.p0, P.x, P.r, P.D, P.CR, P.CZ, P.nr, P.nz, P.state, P.partials, g - P.row_start, P.nr);
}

// x = 0 on the row when the problem's b = 0 (after the start test).
__device__ __forceinline__ void b_zero_item(const ProbDesc *__restrict__ d, int n, int g)
{
    const int p = find_problem(d, n, g, RANGE_ROWS);
    const ProbDesc &P = d[p];
    if (P.state->done != ST_BZERO) return;
    const int i = g - P.row_start;
    for (int k = threadIdx.x; k < P.nz; k += blockDim.x) P.x[(size_t)i * P.nz + k] = 0.0;
}

}  // namespace
}  // namespace axipcg
