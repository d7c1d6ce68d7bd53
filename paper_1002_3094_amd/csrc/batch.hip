// Batched PCG over independent problems of different sizes (§2.2 eq. (8) for
// each; the series setting of §1 eq. (1) with one operator per problem).
//
// Every PCG phase is one launch that covers the whole batch: the launch's
// workgroups are dealt out to the problems by prefix sums of their row (or
// mode-group) counts, each problem keeps its own device state, partial sums
// and stop flag, and a finished problem's workgroups return at once.  The
// number of launches per iteration does not grow with the number of problems
// (four, plus one transform launch per extra transform plan present), and the
// host reads all states back once per chunk of iterations.
//
// With AXIPCG_FLAG_SINGLE_LAUNCH the same phases run in one cooperative
// launch for the whole solve (bsingle.hip), the host reading the states back
// once at the end; the operations and their order are those of the launches
// above.  The Chebyshev form of eq. (8) (axipcg_batch_cheb_solve) runs the
// same way, one launch per phase, with the update x += d, r -= A d in place
// of the SpMV and no inner products but ||r||^2.
#include <cmath>
#include <vector>

#include "kernels.h"
#include "spmv.h"

namespace axipcg {
namespace {

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

// Descriptors of one batched solve, grouped by problem and by transform
// plan, with their device copies and the states' read-back buffers.
struct BatchSetup {
    static constexpr int M = 4;   // modes per r-solve workgroup, one per wave (256 threads)
    std::vector<ProbDesc> h, hp;
    std::vector<BatchPlan> plans;
    int rows = 0, tri = 0, spt = 0;
    size_t tri_shm = 0;
    DevBuf dd, ds;
    PcgState *hs = nullptr;   // pinned host copy of the states
    const ProbDesc *d = nullptr, *dp = nullptr;
    PcgState *dstates = nullptr;
    BatchSetup() = default;
    BatchSetup(const BatchSetup &) = delete;
    BatchSetup &operator=(const BatchSetup &) = delete;
    ~BatchSetup() { if (hs) (void)hipHostFree(hs); }
};

// tau, rho2: the Chebyshev parameters of each member (NULL for PCG).
void batch_setup(BatchSetup &B, int n, Operator *const *ops, const double *const *b, double *const *x, int prec,
                 const double *tau, const double *rho2, hipStream_t s)
{
    B.h.resize(n);
    std::vector<int> plan(n);
    for (int p = 0; p < n; ++p) {
        const Operator &op = *ops[p];
        ProbDesc &d = B.h[p];
        d.nr = op.nr;
        d.nz = op.nz;
        d.bc_z = op.bc_z;
        d.row_start = B.rows;
        d.tri_start = B.tri;
        d.sp_start = B.spt;
        d.n_sp = batch_spmv_tiles(op.nr, op.nz);
        B.spt += d.n_sp;
        size_t shm = 0;
        batch_tri_geom(op.nr, prec, BatchSetup::M, &d.tri_S, &d.tri_L, &d.tri_Lp, &d.tri_pitch, &shm);
        B.rows += op.nr;
        B.tri += op.nz / BatchSetup::M;
        if (shm > B.tri_shm) B.tri_shm = shm;
        int wr = 1;
        plan[p] = batch_transform_plan(op.nz, prec, &wr);
        d.n_tr = (op.nr + wr - 1) / wr;
        d.tau = tau ? tau[p] : 0.0;
        d.rho2 = rho2 ? rho2[p] : 0.0;
        d.b = b[p];
        d.x = x[p];
        d.D = op.D; d.CR = op.CR; d.CZ = op.CZ;
        d.r = op.r; d.z = op.z; d.p0 = op.p0; d.p1 = op.p1; d.q = op.q;
        d.spec = op.spec;
        d.partials = op.partials;
        d.state = op.state;
        d.cb32 = op.cb32; d.db32 = op.db32; d.rw32 = op.rw32; d.lam32 = op.lam32;
        d.cb64 = op.cb64; d.db64 = op.db64; d.rw64 = op.rw64; d.lam64 = op.lam64;
        d.tw32 = op.tw32; d.pt32 = op.pt32; d.tw64 = op.tw64; d.pt64 = op.pt64;
    }
    AXI_REQUIRE(B.tri_shm <= 65536, "a batch member's r-solve tile exceeds the LDS budget");
    // a second copy of the descriptors, grouped by transform plan: one
    // transform launch per plan present
    B.hp.reserve(n);
    for (const int r2 : {0, 2, 4, 8, 16}) {
        BatchPlan pl;
        pl.r2 = r2;
        pl.off = (int)B.hp.size();
        for (int p = 0; p < n; ++p) {
            if (plan[p] != r2) continue;
            ProbDesc e = B.h[p];
            e.tr_start = pl.blocks;
            pl.blocks += e.n_tr;
            if (e.nz > pl.nz_max) pl.nz_max = e.nz;
            B.hp.push_back(e);
            ++pl.n;
        }
        if (pl.n > 0) B.plans.push_back(pl);
    }
    AXI_REQUIRE((int)B.hp.size() == n, "unknown transform plan");
    AXI_CHECK_HIP(hipMalloc(&B.dd.p, 2 * sizeof(ProbDesc) * n));
    AXI_CHECK_HIP(hipMalloc(&B.ds.p, sizeof(PcgState) * n));
    AXI_CHECK_HIP(hipHostMalloc((void **)&B.hs, sizeof(PcgState) * n, hipHostMallocDefault));
    B.d = static_cast<const ProbDesc *>(B.dd.p);
    B.dp = B.d + n;
    B.dstates = static_cast<PcgState *>(B.ds.p);
    AXI_CHECK_HIP(hipMemcpyAsync(B.dd.p, B.h.data(), sizeof(ProbDesc) * n, hipMemcpyHostToDevice, s));
    AXI_CHECK_HIP(hipMemcpyAsync((void *)B.dp, B.hp.data(), sizeof(ProbDesc) * n, hipMemcpyHostToDevice, s));
}

// Iterations in chunks (16, then 4) of `step` launches, the states read back
// after each chunk, until every member has stopped or maxit.
template <typename Step>
void batch_iterate(BatchSetup &B, int n, int maxit, hipStream_t s, Step step)
{
    int launched = 0, chunk = 16;
    for (;;) {
        if (chunk > maxit - launched) chunk = maxit - launched;
        for (int it = 0; it < chunk; ++it) step(launched + it);
        launched += chunk;
        launch_b_gather(B.d, n, B.dstates, s);
        AXI_CHECK_HIP(hipMemcpyAsync(B.hs, B.dstates, sizeof(PcgState) * n, hipMemcpyDeviceToHost, s));
        AXI_CHECK_HIP(hipStreamSynchronize(s));
        bool all = true;
        for (int p = 0; p < n; ++p) all = all && B.hs[p].done != ST_RUN;
        if (all || launched >= maxit) break;
        chunk = 4;
    }
}

// Statuses and statistics from the read-back states; the true residuals on
// request.  Returns the worst status.
int batch_finish(const BatchSetup &B, int n, Operator *const *ops, const double *const *b, double *const *x,
                 bool true_residual, axipcg_stats *st, hipStream_t s)
{
    int worst = AXIPCG_OK;
    for (int p = 0; p < n; ++p) {
        const PcgState &q = B.hs[p];
        int status;
        if (q.done == ST_CONV || q.done == ST_BZERO) status = AXIPCG_OK;
        else if (q.done == ST_BREAK) status = AXIPCG_EBREAKDOWN;
        else status = AXIPCG_ENOTCONV;
        if (status == AXIPCG_EBREAKDOWN) worst = AXIPCG_EBREAKDOWN;
        else if (status == AXIPCG_ENOTCONV && worst == AXIPCG_OK) worst = AXIPCG_ENOTCONV;
        ops[p]->last_iters = q.iters;
        if (st) {
            st[p].iters = q.iters;
            st[p].status = status;
            st[p].relres_rec = (q.bb > 0) ? std::sqrt(q.rr / q.bb) : 0.0;
            st[p].relres_true = -1.0;
        }
    }
    if (st && true_residual) {
        for (int p = 0; p < n; ++p) {
            if (B.hs[p].bb > 0) {
                resid_impl(*ops[p], b[p], x[p], ops[p]->dscal, s);
                AXI_CHECK_HIP(hipMemcpyAsync(ops[p]->scratch_host, ops[p]->dscal, 2 * sizeof(double),
                                             hipMemcpyDeviceToHost, s));
                AXI_CHECK_HIP(hipStreamSynchronize(s));
                st[p].relres_true = std::sqrt(ops[p]->scratch_host[0] / ops[p]->scratch_host[1]);
            } else {
                st[p].relres_true = 0.0;
            }
        }
    }
    return worst;
}

// The start of both forms: r = b - A x and z = B^{-1} r, the r-solve launch
// initialising each state and running the start test; x = 0 where b = 0;
// then the inverse transform in `zinv_mode` (2: PCG, z and r.z; 4:
// Chebyshev, d = tau z).
void batch_start(const BatchSetup &B, int n, int prec, const TriGate &g, int zinv_mode, hipStream_t s)
{
    launch_b_init(B.d, n, B.rows, s);
    for (const BatchPlan &pl : B.plans) launch_b_zfwd(B.dp, pl, prec, BZ_START, 0, s);
    launch_b_tridiag(B.d, n, B.tri, prec, g, BatchSetup::M, B.tri_shm, s);
    launch_b_zero(B.d, n, B.rows, s);
    for (const BatchPlan &pl : B.plans) launch_b_zinv(B.dp, pl, prec, zinv_mode, false, s);
}

int batch_impl(int n, Operator *const *ops, const double *const *b, double *const *x, double rtol, int maxit,
               int prec, unsigned flags, axipcg_stats *st, hipStream_t s)
{
    const bool single = (flags & AXIPCG_FLAG_SINGLE_LAUNCH) != 0;
    const bool pr = (flags & AXIPCG_FLAG_POLAK_RIBIERE) != 0;
    BatchSetup B;
    batch_setup(B, n, ops, b, x, prec, nullptr, nullptr, s);
    TriGate g;
    g.mode = 2;
    g.rtol2 = rtol * rtol;
    g.maxit = maxit;
    g.flags = (int)flags;
    TriGate gi;
    gi.mode = 1;
    if (single) {
        BatchSingle bs;
        bs.d = B.d;
        bs.dp = B.dp;
        bs.n = n;
        bs.rows = B.rows;
        bs.tri = B.tri;
        bs.spt = B.spt;
        bs.nplan = (int)B.plans.size();
        size_t shm = B.tri_shm;
        for (int i = 0; i < bs.nplan; ++i) {
            bs.plans[i] = B.plans[i];
            const size_t lds = batch_plan_lds(B.plans[i], prec, &bs.twl[i]);
            if (lds > shm) shm = lds;
        }
        bs.g_start = g;
        bs.g_step = gi;
        bs.M = BatchSetup::M;
        bs.maxit = maxit;
        int rmax = 2;
        for (const BatchPlan &pl : B.plans) rmax = pl.r2 > rmax ? pl.r2 : rmax;
        const int grid = batch_single_grid(prec, rmax, pr, shm);
        // barrier words (1 + grid) and the error word, zero before the launch
        DevBuf db;
        AXI_CHECK_HIP(hipMalloc(&db.p, sizeof(unsigned) * (grid + 2)));
        const std::vector<unsigned> zero(grid + 2, 0u);
        AXI_CHECK_HIP(hipMemcpyAsync(db.p, zero.data(), sizeof(unsigned) * (grid + 2), hipMemcpyHostToDevice, s));
        bs.bar = static_cast<unsigned *>(db.p);
        bs.err = reinterpret_cast<int *>(bs.bar + grid + 1);
        bs.out = B.dstates;
        launch_b_single(bs, prec, rmax, pr, grid, shm, s);
        AXI_CHECK_HIP(hipMemcpyAsync(B.hs, B.dstates, sizeof(PcgState) * n, hipMemcpyDeviceToHost, s));
        int err = 0;
        AXI_CHECK_HIP(hipMemcpyAsync(&err, bs.err, sizeof(int), hipMemcpyDeviceToHost, s));
        AXI_CHECK_HIP(hipStreamSynchronize(s));
        if (err) throw Error{AXIPCG_EDEVICE, "a grid barrier of the single-launch batch gave up"};
    } else {
        batch_start(B, n, prec, g, 2, s);
        batch_iterate(B, n, maxit, s, [&](int it) {
            const int parity = it & 1;
            launch_b_spmv(B.d, n, B.spt, pr, parity, s);
            for (const BatchPlan &pl : B.plans) launch_b_zfwd(B.dp, pl, prec, BZ_PCG, parity, s);
            launch_b_tridiag(B.d, n, B.tri, prec, gi, BatchSetup::M, B.tri_shm, s);
            for (const BatchPlan &pl : B.plans) launch_b_zinv(B.dp, pl, prec, 1, pr, s);
        });
    }
    return batch_finish(B, n, ops, b, x, (flags & AXIPCG_FLAG_TRUE_RESIDUAL) != 0, st, s);
}

// Chebyshev form of eq. (8) for every member, with its bounds gamma1 <=
// gamma2: start d = tau z; per iteration x += d, r -= A d (||r||^2 partials,
// one per row), forward transform, stop test and r-solves, inverse transform
// forming the next d.  The increment lives in each member's p0 buffer.
int batch_cheb_impl(int n, Operator *const *ops, const double *const *b, double *const *x, const double *g1,
                    const double *g2, double rtol, int maxit, int prec, bool true_residual, axipcg_stats *st,
                    hipStream_t s)
{
    std::vector<double> tau(n), rho2(n);
    for (int p = 0; p < n; ++p) {
        tau[p] = 2.0 / (g1[p] + g2[p]);
        const double xi = g1[p] / g2[p];
        rho2[p] = ((1.0 - xi) / (1.0 + xi)) * ((1.0 - xi) / (1.0 + xi));
    }
    BatchSetup B;
    batch_setup(B, n, ops, b, x, prec, tau.data(), rho2.data(), s);
    TriGate g;
    g.mode = 2;
    g.rtol2 = rtol * rtol;
    g.maxit = maxit;
    batch_start(B, n, prec, g, 4, s);
    TriGate gi;
    gi.mode = 1;
    gi.rr_rows = 1;
    batch_iterate(B, n, maxit, s, [&](int) {
        launch_b_cheb(B.d, n, B.rows, s);
        for (const BatchPlan &pl : B.plans) launch_b_zfwd(B.dp, pl, prec, BZ_CHEB, 0, s);
        launch_b_tridiag(B.d, n, B.tri, prec, gi, BatchSetup::M, B.tri_shm, s);
        for (const BatchPlan &pl : B.plans) launch_b_zinv(B.dp, pl, prec, 3, false, s);
    });
    return batch_finish(B, n, ops, b, x, true_residual, st, s);
}

// The checks both batched entry points make on their members.
std::vector<Operator *> batch_members(int n, const axipcg_op_t *ops, const double *const *b, double *const *x,
                                      int nz_max)
{
    AXI_REQUIRE(n >= 1 && n <= 4096, "n must be in [1, 4096]");
    AXI_REQUIRE(ops && b && x, "NULL argument");
    std::vector<Operator *> v(n);
    long rows = 0;
    for (int p = 0; p < n; ++p) {
        v[p] = reinterpret_cast<Operator *>(ops[p]);
        AXI_REQUIRE(v[p] && b[p] && x[p], "NULL operator or vector in the batch");
        AXI_REQUIRE(b[p] != x[p], "b and x must not alias");
        AXI_REQUIRE(v[p]->nr <= 1024, "batch members need nr <= 1024");
        AXI_REQUIRE(v[p]->nz % 4 == 0 && v[p]->nz <= 2048, "batch members need nz in [4, 2048]");
        AXI_REQUIRE(v[p]->nz <= nz_max, "the single-launch batch takes members with nz <= 1024");
        for (int q = 0; q < p; ++q) AXI_REQUIRE(v[q] != v[p], "an operator appears twice in the batch");
        rows += v[p]->nr;
    }
    AXI_REQUIRE(rows <= 2147483647L, "batch too large");
    return v;
}

}  // namespace
}  // namespace axipcg

using namespace axipcg;

extern "C" int axipcg_batch_solve(int n, const axipcg_op_t *ops, const double *const *b, double *const *x,
                                  double rtol, int maxit, int prec, unsigned flags, axipcg_stats *st, void *stream)
{
    return guarded([&] {
        AXI_REQUIRE(std::isfinite(rtol) && rtol > 0, "rtol must be > 0");
        AXI_REQUIRE(maxit >= 1 && maxit <= 100000, "maxit must be in [1, 100000]");
        AXI_REQUIRE(prec == AXIPCG_PREC_FP32 || prec == AXIPCG_PREC_FP64, "prec must be 0 or 1");
        AXI_REQUIRE((flags & ~7u) == 0, "unknown flags");
        std::vector<Operator *> v =
            batch_members(n, ops, b, x, (flags & AXIPCG_FLAG_SINGLE_LAUNCH) ? 1024 : 2048);
        return batch_impl(n, v.data(), b, x, rtol, maxit, prec, flags, st, (hipStream_t)stream);
    });
}

extern "C" int axipcg_batch_cheb_solve(int n, const axipcg_op_t *ops, const double *const *b, double *const *x,
                                       const double *gamma1, const double *gamma2, double rtol, int maxit, int prec,
                                       unsigned flags, axipcg_stats *st, void *stream)
{
    return guarded([&] {
        AXI_REQUIRE(std::isfinite(rtol) && rtol > 0 && rtol < 1, "rtol must be in (0, 1)");
        AXI_REQUIRE(maxit >= 1 && maxit <= 100000, "maxit must be in [1, 100000]");
        AXI_REQUIRE(prec == AXIPCG_PREC_FP32 || prec == AXIPCG_PREC_FP64, "prec must be 0 or 1");
        AXI_REQUIRE((flags & ~(unsigned)AXIPCG_FLAG_TRUE_RESIDUAL) == 0, "unknown flags");
        std::vector<Operator *> v = batch_members(n, ops, b, x, 2048);
        std::vector<double> g1(n), g2(n);
        for (int p = 0; p < n; ++p) {
            g1[p] = gamma1 ? gamma1[p] : 0.0;
            g2[p] = gamma2 ? gamma2[p] : 0.0;
            if (g1[p] <= 0 && g2[p] <= 0) {
                g1[p] = v[p]->gamma1;
                g2[p] = v[p]->gamma2;
            }
            AXI_REQUIRE(std::isfinite(g1[p]) && std::isfinite(g2[p]) && g1[p] > 0 && g1[p] <= g2[p],
                        "need 0 < gamma1 <= gamma2 for every member (the operator's own bounds have gamma1 = 0 "
                        "when some q is 0 while qbar > 0)");
        }
        return batch_cheb_impl(n, v.data(), b, x, g1.data(), g2.data(), rtol, maxit, prec,
                               (flags & AXIPCG_FLAG_TRUE_RESIDUAL) != 0, st, (hipStream_t)stream);
    });
}
