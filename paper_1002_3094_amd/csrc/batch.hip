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
// above.
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

int batch_impl(int n, Operator *const *ops, const double *const *b, double *const *x, double rtol, int maxit,
               int prec, unsigned flags, axipcg_stats *st, hipStream_t s)
{
    const bool single = (flags & AXIPCG_FLAG_SINGLE_LAUNCH) != 0;
    // modes per r-solve workgroup, one per wave: 256 threads, as every
    // workgroup of the single launch has
    const int M = 4;
    std::vector<ProbDesc> h(n);
    std::vector<int> plan(n);
    int rows = 0, tri = 0, spt = 0;
    size_t tri_shm = 0;
    for (int p = 0; p < n; ++p) {
        const Operator &op = *ops[p];
        ProbDesc &d = h[p];
        d.nr = op.nr;
        d.nz = op.nz;
        d.bc_z = op.bc_z;
        d.row_start = rows;
        d.tri_start = tri;
        d.sp_start = spt;
        d.n_sp = batch_spmv_tiles(op.nr, op.nz);
        spt += d.n_sp;
        size_t shm = 0;
        batch_tri_geom(op.nr, prec, M, &d.tri_S, &d.tri_L, &d.tri_Lp, &d.tri_pitch, &shm);
        rows += op.nr;
        tri += op.nz / M;
        if (shm > tri_shm) tri_shm = shm;
        int wr = 1;
        plan[p] = batch_transform_plan(op.nz, prec, &wr);
        d.n_tr = (op.nr + wr - 1) / wr;
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
    AXI_REQUIRE(tri_shm <= 65536, "a batch member's r-solve tile exceeds the LDS budget");
    // a second copy of the descriptors, grouped by transform plan: one
    // transform launch per plan present
    std::vector<ProbDesc> hp;
    std::vector<BatchPlan> plans;
    hp.reserve(n);
    for (const int r2 : {0, 2, 4, 8, 16}) {
        BatchPlan pl;
        pl.r2 = r2;
        pl.off = (int)hp.size();
        for (int p = 0; p < n; ++p) {
            if (plan[p] != r2) continue;
            ProbDesc e = h[p];
            e.tr_start = pl.blocks;
            pl.blocks += e.n_tr;
            if (e.nz > pl.nz_max) pl.nz_max = e.nz;
            hp.push_back(e);
            ++pl.n;
        }
        if (pl.n > 0) plans.push_back(pl);
    }
    AXI_REQUIRE((int)hp.size() == n, "unknown transform plan");

    DevBuf dd, ds;
    AXI_CHECK_HIP(hipMalloc(&dd.p, 2 * sizeof(ProbDesc) * n));
    AXI_CHECK_HIP(hipMalloc(&ds.p, sizeof(PcgState) * n));
    PcgState *hs = nullptr;
    AXI_CHECK_HIP(hipHostMalloc((void **)&hs, sizeof(PcgState) * n, hipHostMallocDefault));
    struct HostFree {
        PcgState *p;
        ~HostFree() { if (p) (void)hipHostFree(p); }
    } hf{hs};
    const ProbDesc *d = static_cast<const ProbDesc *>(dd.p);
    const ProbDesc *dp = d + n;
    PcgState *dstates = static_cast<PcgState *>(ds.p);
    AXI_CHECK_HIP(hipMemcpyAsync(dd.p, h.data(), sizeof(ProbDesc) * n, hipMemcpyHostToDevice, s));
    AXI_CHECK_HIP(hipMemcpyAsync((void *)dp, hp.data(), sizeof(ProbDesc) * n, hipMemcpyHostToDevice, s));

    const bool pr = (flags & AXIPCG_FLAG_POLAK_RIBIERE) != 0;
    TriGate g;
    g.mode = 2;
    g.rtol2 = rtol * rtol;
    g.maxit = maxit;
    g.flags = (int)flags;
    if (!single) {
        // start: r = b - A x, z = B^{-1} r (the r-solve launch initialises each state)
        launch_b_init(d, n, rows, s);
        for (const BatchPlan &pl : plans) launch_b_zfwd(dp, pl, prec, false, 0, s);
        launch_b_tridiag(d, n, tri, prec, g, M, tri_shm, s);
        launch_b_zero(d, n, rows, s);
        for (const BatchPlan &pl : plans) launch_b_zinv(dp, pl, prec, 2, false, s);
    }

    TriGate gi;
    gi.mode = 1;
    if (single) {
        BatchSingle bs;
        bs.d = d;
        bs.dp = dp;
        bs.n = n;
        bs.rows = rows;
        bs.tri = tri;
        bs.spt = spt;
        bs.nplan = (int)plans.size();
        size_t shm = tri_shm;
        for (int i = 0; i < bs.nplan; ++i) {
            bs.plans[i] = plans[i];
            const size_t b = batch_plan_lds(plans[i], prec, &bs.twl[i]);
            if (b > shm) shm = b;
        }
        bs.g_start = g;
        bs.g_step = gi;
        bs.M = M;
        bs.maxit = maxit;
        int rmax = 2;
        for (const BatchPlan &pl : plans) rmax = pl.r2 > rmax ? pl.r2 : rmax;
        const int grid = batch_single_grid(prec, rmax, pr, shm);
        // barrier words (1 + grid) and the error word, zero before the launch
        DevBuf db;
        AXI_CHECK_HIP(hipMalloc(&db.p, sizeof(unsigned) * (grid + 2)));
        const std::vector<unsigned> zero(grid + 2, 0u);
        AXI_CHECK_HIP(hipMemcpyAsync(db.p, zero.data(), sizeof(unsigned) * (grid + 2), hipMemcpyHostToDevice, s));
        bs.bar = static_cast<unsigned *>(db.p);
        bs.err = reinterpret_cast<int *>(bs.bar + grid + 1);
        bs.out = dstates;
        launch_b_single(bs, prec, rmax, pr, grid, shm, s);
        AXI_CHECK_HIP(hipMemcpyAsync(hs, dstates, sizeof(PcgState) * n, hipMemcpyDeviceToHost, s));
        int err = 0;
        AXI_CHECK_HIP(hipMemcpyAsync(&err, bs.err, sizeof(int), hipMemcpyDeviceToHost, s));
        AXI_CHECK_HIP(hipStreamSynchronize(s));
        if (err) throw Error{AXIPCG_EDEVICE, "a grid barrier of the single-launch batch gave up"};
    } else {
        int launched = 0, parity = 0, chunk = 16;
        for (;;) {
            if (chunk > maxit - launched) chunk = maxit - launched;
            for (int it = 0; it < chunk; ++it) {
                launch_b_spmv(d, n, spt, pr, parity, s);
                for (const BatchPlan &pl : plans) launch_b_zfwd(dp, pl, prec, true, parity, s);
                launch_b_tridiag(d, n, tri, prec, gi, M, tri_shm, s);
                for (const BatchPlan &pl : plans) launch_b_zinv(dp, pl, prec, 1, pr, s);
                parity ^= 1;
            }
            launched += chunk;
            launch_b_gather(d, n, dstates, s);
            AXI_CHECK_HIP(hipMemcpyAsync(hs, dstates, sizeof(PcgState) * n, hipMemcpyDeviceToHost, s));
            AXI_CHECK_HIP(hipStreamSynchronize(s));
            bool all = true;
            for (int p = 0; p < n; ++p) all = all && hs[p].done != ST_RUN;
            if (all || launched >= maxit) break;
            chunk = 4;
        }
    }

    int worst = AXIPCG_OK;
    for (int p = 0; p < n; ++p) {
        const PcgState &q = hs[p];
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
    if (st && (flags & AXIPCG_FLAG_TRUE_RESIDUAL)) {
        for (int p = 0; p < n; ++p) {
            if (hs[p].bb > 0) {
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

}  // namespace
}  // namespace axipcg

using namespace axipcg;

extern "C" int axipcg_batch_solve(int n, const axipcg_op_t *ops, const double *const *b, double *const *x,
                                  double rtol, int maxit, int prec, unsigned flags, axipcg_stats *st, void *stream)
{
    return guarded([&] {
        AXI_REQUIRE(n >= 1 && n <= 4096, "n must be in [1, 4096]");
        AXI_REQUIRE(ops && b && x, "NULL argument");
        AXI_REQUIRE(std::isfinite(rtol) && rtol > 0, "rtol must be > 0");
        AXI_REQUIRE(maxit >= 1 && maxit <= 100000, "maxit must be in [1, 100000]");
        AXI_REQUIRE(prec == AXIPCG_PREC_FP32 || prec == AXIPCG_PREC_FP64, "prec must be 0 or 1");
        AXI_REQUIRE((flags & ~7u) == 0, "unknown flags");
        std::vector<Operator *> v(n);
        long rows = 0;
        for (int p = 0; p < n; ++p) {
            v[p] = reinterpret_cast<Operator *>(ops[p]);
            AXI_REQUIRE(v[p] && b[p] && x[p], "NULL operator or vector in the batch");
            AXI_REQUIRE(b[p] != x[p], "b and x must not alias");
            AXI_REQUIRE(v[p]->nr <= 1024, "batch members need nr <= 1024");
            AXI_REQUIRE(v[p]->nz % 4 == 0 && v[p]->nz <= 2048, "batch members need nz in [4, 2048]");
            AXI_REQUIRE(!(flags & AXIPCG_FLAG_SINGLE_LAUNCH) || v[p]->nz <= 1024,
                        "the single-launch batch takes members with nz <= 1024");
            for (int q = 0; q < p; ++q) AXI_REQUIRE(v[q] != v[p], "an operator appears twice in the batch");
            rows += v[p]->nr;
        }
        AXI_REQUIRE(rows <= 2147483647L, "batch too large");
        return batch_impl(n, v.data(), b, x, rtol, maxit, prec, flags, st, (hipStream_t)stream);
    });
}
