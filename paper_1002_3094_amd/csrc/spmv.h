// Device bodies of the PCG step's SpMV (§2.2 eq. (8) with conjugate-
// gradient parameters; the operator of §2.1) that more than one launch form
// shares: the 5-point r-weighted stencil, the row-per-workgroup SpMV with the
// p update and p.q partials, and the start r = b - A x.  Each body takes its
// work item (vb, of vnb) as an argument.
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

// rho_k, beta; p_new = z + beta p_old; q = A p_new; p_new . q partials.
// A z and A p_old are formed first (no scalar needed), so the loads overlap
// the reduction of the r.z partials; q = A z + beta A p_old is the same
// product up to rounding (no recurrence: both terms are recomputed from the
// stored vectors every iteration).  A thread handles pairs of adjacent points
// (16-byte loads and stores; the z-neighbours k-1 and k+2 are 8-byte loads
// that hit the lines its wave already fetched).
constexpr int SPMV_PAIRS = 4;   // pairs per thread per row (nz <= 2048, 256 threads)

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

template <bool PR>
__device__ __forceinline__ void spmv_body(const double *__restrict__ z, const double *__restrict__ pold,
                                          double *__restrict__ pnew, double *__restrict__ q,
                                          const double *__restrict__ D, const double *__restrict__ CR,
                                          const double *__restrict__ CZ, int nr, int nz, PcgState *st,
                                          double *__restrict__ partials, int n_rz, int vb, int vnb)
{
    __shared__ double red[8];
    double acc = 0.0;
    double beta = 0.0;
    bool have_beta = false;
    int k_it = 0;
    for (int b = vb; b < nr; b += vnb) {
        const int i = xcd_swizzle(b, nr);
        Pair az[SPMV_PAIRS], ap[SPMV_PAIRS], zc[SPMV_PAIRS], pc[SPMV_PAIRS];
#pragma unroll
        for (int j = 0; j < SPMV_PAIRS; ++j) {
            const int k = 2 * (threadIdx.x + j * 256);
            if (k < nz) {
                const size_t e = (size_t)i * nz + k;
                zc[j] = ld2(z + e);
                pc[j] = ld2(pold + e);
                az[j] = stencil2(z, D, CR, CZ, e, i, k, nr, nz, zc[j]);
                ap[j] = stencil2(pold, D, CR, CZ, e, i, k, nr, nz, pc[j]);
            }
        }
        if (!have_beta) {   // scalars once per workgroup, after the first row's loads
            if (st->done) return;
            k_it = st->iters;
            const double rho = block_total(partials + SLOT_RZ * MAX_PARTIALS, n_rz, red);
            if (k_it > 0) {
                double num = rho;
                if (PR) num -= block_total(partials + SLOT_RZOLD * MAX_PARTIALS, n_rz, red);
                beta = num / st->rho[(k_it - 1) & 1];
            }
            if (vb == 0 && threadIdx.x == 0) st->rho[k_it & 1] = rho;
            have_beta = true;
        }
#pragma unroll
        for (int j = 0; j < SPMV_PAIRS; ++j) {
            const int k = 2 * (threadIdx.x + j * 256);
            if (k < nz) {
                const size_t e = (size_t)i * nz + k;
                double2 pn, qn;
                pn.x = (k_it > 0) ? zc[j].a + beta * pc[j].a : zc[j].a;
                pn.y = (k_it > 0) ? zc[j].b + beta * pc[j].b : zc[j].b;
                qn.x = (k_it > 0) ? az[j].a + beta * ap[j].a : az[j].a;
                qn.y = (k_it > 0) ? az[j].b + beta * ap[j].b : az[j].b;
                *reinterpret_cast<double2 *>(pnew + e) = pn;
                *reinterpret_cast<double2 *>(q + e) = qn;
                acc += pn.x * qn.x;
                acc += pn.y * qn.y;
            }
        }
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[SLOT_PQ * MAX_PARTIALS + vb] = s;
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
// One row of a batched phase, `g` its index over the rows of the whole batch
// (a launch passes its workgroup index; the single-launch batch deals the
// rows to its resident workgroups).
template <bool PR>
__device__ __forceinline__ void b_spmv_item(const ProbDesc *__restrict__ d, int n, int g, int parity)
{
    const int p = find_problem(d, n, g, RANGE_ROWS);
    const ProbDesc &P = d[p];
    const double *pold = parity ? P.p1 : P.p0;
    double *pnew = parity ? P.p0 : P.p1;
    spmv_body<PR>(P.z, pold, pnew, P.q, P.D, P.CR, P.CZ, P.nr, P.nz, P.state, P.partials, P.n_tr, g - P.row_start,
                  P.nr);
}

__device__ __forceinline__ void b_init_item(const ProbDesc *__restrict__ d, int n, int g)
{
    const int p = find_problem(d, n, g, RANGE_ROWS);
    const ProbDesc &P = d[p];
    init_body(P.b, P.x, P.r, P.D, P.CR, P.CZ, P.nr, P.nz, P.partials, g - P.row_start, P.nr);
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
