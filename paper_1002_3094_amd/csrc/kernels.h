// Host-side launchers shared between the library's translation units.
#pragma once

#include "common.h"

namespace axipcg {

// Forward z-transform of every r-row (§4.2 eq. (38)).
//  plain: spec = S rin (with `state` set: skipped once the stop test has fired)
//  fused PCG step (after the SpMV kernel): alpha = rho / p.q from the SpMV
//    partials (p.q <= 0 marks a breakdown), x += alpha p, r -= alpha q,
//    one ||r||^2 partial per workgroup, then spec = S r.
struct ZfwdArgs {
    const double *rin = nullptr;           // plain mode input
    double *x = nullptr, *r = nullptr;     // fused mode
    const double *p = nullptr, *q = nullptr;
    PcgState *state = nullptr;             // fused: gate + scalars
    int n_pq = 0;                          // fused: number of p.q partials
    bool fused = false;
};
void launch_zfwd(const Operator &op, int prec, const ZfwdArgs &a, hipStream_t s);

// Workgroups (= partial sums) of the transform launches for this operator.
int transform_blocks(const Operator &op, int prec);

// One r-tridiagonal solve per z-mode, in place on op.spec (§4.2 eq. (39)).
//  mode 0: plain;
//  mode 1: PCG step: ||r||^2 from the forward kernel's partials -> stop test
//          (workgroup 0 records it), then solve unless stopped;
//  mode 2: PCG start: ||r||^2 and ||b||^2 from the start kernel's partials ->
//          state initialised, start test, then solve unless stopped.
//  With `mirror`, workgroup 0 also publishes the outcome to the host
//  (HostMirror) when the test stops the solve, or always when `report`.
struct TriGate {
    int mode = 0;
    PcgState *state = nullptr;
    int n_rr = 0;          // partials of ||r||^2 (and of ||b||^2 in mode 2)
    double rtol2 = 0.0;    // mode 2
    int maxit = 0, flags = 0;
    HostMirror *mirror = nullptr;
    unsigned seq = 0;
    int report = 0;
    int rr_rows = 0;       // batched mode 1: one ||r||^2 partial per row (the Chebyshev update's)
};
void launch_tridiag(const Operator &op, int prec, const TriGate &g, hipStream_t s);

// Inverse z-transform of every row: zout = S^T spec.
//  mode 0: plain;  modes 1 (PCG step) and 2 (PCG start): skipped once the
//  stop test has fired, one r.z partial per workgroup (and r.z_old for the
//  Polak-Ribiere form), reduced by the next SpMV kernel.
//  modes 3 (Chebyshev step) and 4 (Chebyshev start): z is not stored; it
//  forms the increment of eq. (8) in Chebyshev form instead,
//  d = (alpha_m - 1) d + alpha_m tau z with m = iterations done + 1
//  (mode 4: d = tau z), skipped once the stop test has fired.
struct ZinvArgs {
    double *zout = nullptr;
    const double *r = nullptr;
    PcgState *state = nullptr;
    int mode = 0;
    bool pr = false;   // also reduce r.z_old (Polak-Ribiere)
    double *d = nullptr;           // modes 3, 4
    double tau = 0.0, rho2 = 0.0;  // modes 3, 4: Chebyshev parameters
};
void launch_zinv(const Operator &op, int prec, const ZinvArgs &a, hipStream_t s);

// Strip-partitioned form of the same three launches (strip.hip): forward
// transform + local elimination of strips of `rows` rows, the reduced
// systems of the strips' boundary rows, back substitution + inverse
// transform.  The launch_* functions above route to it with the handle's
// strip height when strip_usable holds for it.
bool strip_usable(const Operator &op, int prec, int rows);
// The strip height of the solves' launches for this precision (0: per-mode).
int strip_solve_rows(const Operator &op, int prec);
size_t strip_red_bytes(int nr, int nz);
void strip_fwd(const Operator &op, int prec, int rows, const ZfwdArgs &a, hipStream_t s);
void strip_reduced(const Operator &op, int prec, int rows, const TriGate &g, hipStream_t s);
void strip_inv(const Operator &op, int prec, int rows, const ZinvArgs &a, hipStream_t s);

// z = B^{-1} r with three launches (forward, r-solves, inverse).
void precond_apply_impl(const Operator &op, const double *r, double *z, int prec, hipStream_t s);

// The strip form in one cooperative launch (pfused.hip), FP32, when
// pfused_plan accepts the operator for the kind of launch (0 standalone
// apply, 1 PCG iteration: the forward kernel's x, r update, the r-solve
// launch's stop test and the inverse's r.z partials in the same launch).
bool pfused_plan(Operator &op, int kind);
void pfused_apply(Operator &op, const double *r, double *z, hipStream_t s);
void pfused_pcg_step(Operator &op, const ZfwdArgs &fa, const TriGate &g, const ZinvArgs &ia, hipStream_t s);

// ---- batched solve: one launch per PCG phase covers every problem ----------
void batch_tri_geom(int nr, int prec, int M, int *S, int *L, int *Lp, int *pitch, size_t *shm);
void launch_b_init(const ProbDesc *d, int n, int rows, hipStream_t s);
void launch_b_zero(const ProbDesc *d, int n, int rows, hipStream_t s);
void launch_b_spmv(const ProbDesc *d, int n, int tiles, bool pr, int parity, hipStream_t s);
// Chebyshev step of every member (one workgroup per row): x += d, r -= A d,
// ||r||^2 partials; d is the member's p0 buffer.
void launch_b_cheb(const ProbDesc *d, int n, int rows, hipStream_t s);
// One batched transform launch covers the problems d[off, off + n) of an
// array sorted by transform plan: r2 = N / 128 for the one-wave plans, 0 for
// the block-wide kernels (one row per workgroup); `blocks` workgroups in all.
struct BatchPlan {
    int r2 = 0, off = 0, n = 0, blocks = 0, nz_max = 0;
};
// Plan of a batch member with nz points per row: returns r2 and sets the rows
// per transform workgroup.
int batch_transform_plan(int nz, int prec, int *rows_per_wg);
// kind 0: start (plain transform of r); 1: PCG step (alpha, x and r update,
// transform); 2: Chebyshev step (plain transform of r, skipped once stopped).
enum { BZ_START = 0, BZ_PCG = 1, BZ_CHEB = 2 };
void launch_b_zfwd(const ProbDesc *d, const BatchPlan &pl, int prec, int kind, int parity, hipStream_t s);
void launch_b_tridiag(const ProbDesc *d, int n, int blocks, int prec, const TriGate &g, int M, size_t shm,
                      hipStream_t s);
// mode as for launch_zinv (1, 2: PCG; 3, 4: Chebyshev, d in each member's p0)
void launch_b_zinv(const ProbDesc *d, const BatchPlan &pl, int prec, int mode, bool pr, hipStream_t s);
void launch_b_gather(const ProbDesc *d, int n, PcgState *out, hipStream_t s);
// Dynamic LDS of a transform plan's workgroup; *twl: twiddles staged in LDS
// (block-wide plans).
size_t batch_plan_lds(const BatchPlan &pl, int prec, bool *twl);

// The whole batched solve in one cooperative launch (bsingle.hip): the
// phases above dealt to resident workgroups, grid barriers between them.
struct BatchSingle {
    const ProbDesc *d = nullptr;    // by problem
    const ProbDesc *dp = nullptr;   // by transform plan
    int n = 0, rows = 0, tri = 0, spt = 0, nplan = 0;   // items: rows, mode groups, SpMV tiles
    BatchPlan plans[5];
    bool twl[5] = {};
    TriGate g_start, g_step;
    int M = 4, maxit = 0;
    unsigned *bar = nullptr;   // 1 + grid words, zero before the launch
    int *err = nullptr;        // set when a barrier gives up
    PcgState *out = nullptr;   // the n states at the end
};
// Workgroups of the single launch (all resident) for `shm` bytes of LDS;
// rmax: the batch's largest one-wave transform plan (BatchPlan::r2).
int batch_single_grid(int prec, int rmax, bool pr, size_t shm);
void launch_b_single(const BatchSingle &b, int prec, int rmax, bool pr, int grid, size_t shm, hipStream_t s);
void resid_impl(const Operator &op, const double *b, const double *x, double *out_dev, hipStream_t s);

// Flattened grid geometry for pointwise kernels.
inline unsigned pointwise_blocks(size_t n, int threads = 256)
{
    size_t b = (n + threads - 1) / threads;
    if (b > (size_t)MAX_PARTIALS) b = MAX_PARTIALS;
    return (unsigned)b;
}

// The guard of axipcg_guess_poly (nn NULL) or axipcg_nn_guess_poly with a
// cache of A u: ah[j] holds A hist[j] for 1 <= j < K on entry, and A hist[0]
// is written to ah[0] (each array nr * nz).  Same choice and x as the
// uncached calls.
void guess_poly_cached(Operator &op, axipcg_nn_t nn, const double *b, const double *const *hist, int K,
                       double *const *ah, const double *kappa, double *x, hipStream_t s);
// y = A v with the guard's arithmetic (to fill that cache).
void apply_a_pairs(const Operator &op, const double *v, double *y, hipStream_t s);

// The solve entry points behind axipcg_pcg_solve / axipcg_cheb_solve (which
// pass sync_end = true).  With sync_end = false the call returns as soon as
// the host has seen the stop test's outcome: launches of the last chunk may
// still be queued, so later work on the stream is ordered after them while
// the host has not waited for them.
int pcg_solve_entry(axipcg_op_t h, const double *b, double *x, double rtol, int maxit, int prec, unsigned flags,
                    axipcg_stats *st, void *stream, bool sync_end);
int cheb_solve_entry(axipcg_op_t h, const double *b, double *x, double gamma1, double gamma2, double rtol,
                     int maxit, int prec, axipcg_stats *st, void *stream, bool sync_end);

}  // namespace axipcg
