// PCG (§2.2 eq. (8) with conjugate-gradient parameters) on gfx950.
//
// One iteration is four stream-ordered launches; every scalar lives in device
// memory (PcgState) and is produced by the last workgroup of the kernel that
// completes its reduction, so the host never waits inside an iteration:
//   1. p = z + beta p_old (ping-pong), q = A p, p.q  -> alpha = rho / p.q
//   2. x += alpha p, r -= alpha q, ||r||^2 -> stop test; forward z-transform of r
//   3. r-tridiagonal solves of the preconditioner
//   4. inverse z-transform -> z, r.z -> beta, rho
// After the stop test fires, the remaining launches of the chunk return at
// once.  The host reads the state back once per chunk of iterations.
#include <cmath>

#include "kernels.h"

namespace axipcg {

void apply_impl(const Operator &op, const double *x, double *y, hipStream_t s);
void resid_impl(const Operator &op, const double *b, const double *x, double *out_dev, hipStream_t s);

namespace {

// p_new = z + beta p_old; q = A p_new; reduce p_new . q.
__global__ void __launch_bounds__(256)
k_pcg_spmv(const double *__restrict__ z, const double *__restrict__ pold, double *__restrict__ pnew,
           double *__restrict__ q, const double *__restrict__ D, const double *__restrict__ CR,
           const double *__restrict__ CZ, int nr, int nz, PcgState *st, double *partials, unsigned *tickets)
{
    if (st->done) return;
    __shared__ double red[8];
    const double beta = st->beta;
    const size_t n = (size_t)nr * nz;
    double acc = 0.0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / nz), k = (int)(e - (size_t)i * nz);
        const double pc = z[e] + beta * pold[e];
        double v = D[e] * pc;
        if (i + 1 < nr) v -= CR[e] * (z[e + nz] + beta * pold[e + nz]);
        if (i > 0) v -= CR[e - nz] * (z[e - nz] + beta * pold[e - nz]);
        if (k + 1 < nz) v -= CZ[e] * (z[e + 1] + beta * pold[e + 1]);
        if (k > 0) v -= CZ[e - 1] * (z[e - 1] + beta * pold[e - 1]);
        pnew[e] = pc;
        q[e] = v;
        acc += pc * v;
    }
    const double s = block_sum(acc, red);
    if (publish_partial(s, partials + SLOT_PQ * MAX_PARTIALS, tickets + SLOT_PQ * 16, gridDim.x, blockIdx.x)) {
        const double pq = sum_partials(partials + SLOT_PQ * MAX_PARTIALS, gridDim.x, red);
        if (threadIdx.x == 0) {
            if (!(pq > 0.0) || !(pq < 1e308)) st->done = 2;
            else st->alpha = st->rho / pq;
        }
    }
}

// r = b - A x; ||r||^2 and ||b||^2; initial state.
__global__ void __launch_bounds__(256)
k_pcg_init(const double *__restrict__ b, const double *__restrict__ x, double *__restrict__ r,
           const double *__restrict__ D, const double *__restrict__ CR, const double *__restrict__ CZ, int nr,
           int nz, PcgState *st, double *partials, unsigned *tickets, double rtol2, int maxit, int flags)
{
    __shared__ double red[8];
    const size_t n = (size_t)nr * nz;
    double s_r = 0.0, s_b = 0.0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / nz), k = (int)(e - (size_t)i * nz);
        double v = D[e] * x[e];
        if (i + 1 < nr) v -= CR[e] * x[e + nz];
        if (i > 0) v -= CR[e - nz] * x[e - nz];
        if (k + 1 < nz) v -= CZ[e] * x[e + 1];
        if (k > 0) v -= CZ[e - 1] * x[e - 1];
        const double bv = b[e];
        const double d = bv - v;
        r[e] = d;
        s_r += d * d;
        s_b += bv * bv;
    }
    const double tb = block_sum(s_b, red);
    if (threadIdx.x == 0)
        __hip_atomic_store(reinterpret_cast<unsigned long long *>(partials + SLOT_MISC * MAX_PARTIALS + blockIdx.x),
                           (unsigned long long)__double_as_longlong(tb), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double tr = block_sum(s_r, red);
    if (publish_partial(tr, partials + SLOT_RR * MAX_PARTIALS, tickets + SLOT_RR * 16, gridDim.x, blockIdx.x)) {
        const double rr = sum_partials(partials + SLOT_RR * MAX_PARTIALS, gridDim.x, red);
        const double bb = sum_partials(partials + SLOT_MISC * MAX_PARTIALS, gridDim.x, red);
        if (threadIdx.x == 0) {
            st->rr = rr;
            st->bb = bb;
            st->tol2 = rtol2 * bb;
            st->iters = 0;
            st->maxit = maxit;
            st->flags = flags;
            st->alpha = 0.0;
            st->beta = 0.0;
            st->rho = 0.0;
            if (bb == 0.0) st->done = 4;               // b = 0: x = 0 is the answer
            else if (!(rr == rr)) st->done = 2;
            else st->done = (rr <= st->tol2) ? 1 : 0;
        }
    }
}

// x = 0 when b = 0 (state->done == 4).
__global__ void k_zero_if_b_zero(double *__restrict__ x, size_t n, const PcgState *st)
{
    if (st->done != 4) return;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        x[e] = 0.0;
}

__global__ void k_copy_gated(const double *__restrict__ a, double *__restrict__ b, size_t n, const PcgState *st)
{
    if (st->done) return;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        b[e] = a[e];
}

struct SolveCtx {
    Operator *op;
    const double *b;
    double *x;
    int prec;
    hipStream_t s;
};

// Event pair around one launch of the profiled kernel class.
struct ProfScope {
    Operator &op;
    hipStream_t s;
    bool on;
    size_t slot = 0;
    ProfScope(Operator &o, hipStream_t st, int kernel, int iter) : op(o), s(st), on(o.prof_kernel == kernel)
    {
        if (!on) return;
        slot = op.prof_used++;
        while (op.prof_events.size() < 2 * op.prof_used) {
            hipEvent_t e;
            AXI_CHECK_HIP(hipEventCreate(&e));
            op.prof_events.push_back(e);
        }
        if (op.prof_iter.size() < op.prof_used) op.prof_iter.resize(op.prof_used);
        op.prof_iter[slot] = iter;
        AXI_CHECK_HIP(hipEventRecord(op.prof_events[2 * slot], s));
    }
    ~ProfScope() noexcept(false)
    {
        if (on) AXI_CHECK_HIP(hipEventRecord(op.prof_events[2 * slot + 1], s));
    }
};

void launch_iteration(const SolveCtx &c, int parity, int iter)
{
    Operator &op = *c.op;
    const size_t n = (size_t)op.nr * op.nz;
    double *pold = parity ? op.p1 : op.p0;
    double *pnew = parity ? op.p0 : op.p1;
    {
        ProfScope ps(op, c.s, AXIPCG_KERNEL_SPMV, iter);
        hipLaunchKernelGGL(k_pcg_spmv, dim3(pointwise_blocks(n)), dim3(256), 0, c.s, op.z, pold, pnew, op.q,
                           op.D, op.CR, op.CZ, op.nr, op.nz, op.state, op.partials, op.tickets);
        AXI_CHECK_HIP(hipGetLastError());
    }
    ZfwdArgs fa;
    fa.fused = true;
    fa.x = c.x;
    fa.r = op.r;
    fa.p = pnew;
    fa.q = op.q;
    fa.state = op.state;
    {
        ProfScope ps(op, c.s, AXIPCG_KERNEL_ZFWD, iter);
        launch_zfwd(op, c.prec, fa, c.s);
    }
    {
        ProfScope ps(op, c.s, AXIPCG_KERNEL_TRIDIAG, iter);
        launch_tridiag(op, c.prec, op.state, c.s);
    }
    ZinvArgs ia;
    ia.zout = op.z;
    ia.r = op.r;
    ia.state = op.state;
    ia.mode = 1;
    {
        ProfScope ps(op, c.s, AXIPCG_KERNEL_ZINV, iter);
        launch_zinv(op, c.prec, ia, c.s);
    }
}

// Add the timed launches that did work: the SpMV and forward kernels of
// iterations 0..iters-1, the r-solve and inverse of iterations 0..iters-2
// (the stop test fires inside the forward kernel).
void collect_profile(Operator &op, int iters)
{
    for (size_t k = 0; k < op.prof_used; ++k) {
        const int it = op.prof_iter[k];
        const int limit = (op.prof_kernel == AXIPCG_KERNEL_SPMV || op.prof_kernel == AXIPCG_KERNEL_ZFWD)
                              ? iters : iters - 1;
        if (it >= limit) continue;
        float ms = 0.f;
        AXI_CHECK_HIP(hipEventElapsedTime(&ms, op.prof_events[2 * k], op.prof_events[2 * k + 1]));
        op.prof_ms += ms;
        op.prof_count += 1;
    }
    op.prof_used = 0;
}

int solve_impl(Operator &op, const double *b, double *x, double rtol, int maxit, int prec, unsigned flags,
               axipcg_stats *st, hipStream_t s)
{
    const size_t n = (size_t)op.nr * op.nz;
    SolveCtx c{&op, b, x, prec, s};
    // start: r = b - A x, z = B^{-1} r, rho = r.z, p_0 = z
    hipLaunchKernelGGL(k_pcg_init, dim3(pointwise_blocks(n)), dim3(256), 0, s, b, x, op.r, op.D, op.CR, op.CZ,
                       op.nr, op.nz, op.state, op.partials, op.tickets, rtol * rtol, maxit, (int)flags);
    AXI_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_zero_if_b_zero, dim3(pointwise_blocks(n)), dim3(256), 0, s, x, n, op.state);
    AXI_CHECK_HIP(hipGetLastError());
    ZfwdArgs fa;
    fa.rin = op.r;
    launch_zfwd(op, prec, fa, s);
    launch_tridiag(op, prec, op.state, s);
    ZinvArgs ia;
    ia.zout = op.z;
    ia.r = op.r;
    ia.state = op.state;
    ia.mode = 2;
    launch_zinv(op, prec, ia, s);
    hipLaunchKernelGGL(k_copy_gated, dim3(pointwise_blocks(n)), dim3(256), 0, s, op.z, op.p0, n, op.state);
    AXI_CHECK_HIP(hipGetLastError());

    // iterations, in chunks; the first chunk is sized from the previous solve
    int launched = 0;
    int parity = 0;
    op.prof_used = 0;
    int chunk = op.last_iters > 2 ? op.last_iters - 1 : 4;
    for (;;) {
        if (chunk > maxit - launched) chunk = maxit - launched;
        for (int it = 0; it < chunk; ++it) {
            launch_iteration(c, parity, launched + it);
            parity ^= 1;
        }
        launched += chunk;
        AXI_CHECK_HIP(hipMemcpyAsync(op.state_host, op.state, sizeof(PcgState), hipMemcpyDeviceToHost, s));
        AXI_CHECK_HIP(hipStreamSynchronize(s));
        if (op.state_host->done || launched >= maxit) break;
        chunk = 2;
    }
    const PcgState h = *op.state_host;
    op.last_iters = h.iters;
    if (op.prof_kernel >= 0) collect_profile(op, h.iters);
    int status;
    if (h.done == 1 || h.done == 4) status = AXIPCG_OK;
    else if (h.done == 2) status = AXIPCG_EBREAKDOWN;
    else status = AXIPCG_ENOTCONV;
    if (st) {
        st->iters = h.iters;
        st->status = status;
        st->relres_rec = (h.bb > 0) ? std::sqrt(h.rr / h.bb) : 0.0;
        st->relres_true = -1.0;
        if (flags & AXIPCG_FLAG_TRUE_RESIDUAL) {
            if (h.bb > 0) {
                resid_impl(op, b, x, op.dscal, s);
                AXI_CHECK_HIP(hipMemcpyAsync(op.scratch_host, op.dscal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
                AXI_CHECK_HIP(hipStreamSynchronize(s));
                st->relres_true = std::sqrt(op.scratch_host[0] / op.scratch_host[1]);
            } else {
                st->relres_true = 0.0;
            }
        }
    }
    return status;
}

}  // namespace

}  // namespace axipcg

using namespace axipcg;

extern "C" int axipcg_profile_select(axipcg_op_t h, int kernel)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(h);
        AXI_REQUIRE(op != nullptr, "op is NULL");
        AXI_REQUIRE(kernel >= AXIPCG_KERNEL_NONE && kernel <= AXIPCG_KERNEL_ZINV, "unknown kernel class");
        op->prof_kernel = kernel;
        op->prof_used = 0;
        return AXIPCG_OK;
    });
}

extern "C" int axipcg_profile_read(axipcg_op_t h, double *total_ms, long long *launches, int reset)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(h);
        AXI_REQUIRE(op != nullptr, "op is NULL");
        if (total_ms) *total_ms = op->prof_ms;
        if (launches) *launches = op->prof_count;
        if (reset) {
            op->prof_ms = 0.0;
            op->prof_count = 0;
        }
        return AXIPCG_OK;
    });
}

extern "C" int axipcg_pcg_solve(axipcg_op_t h, const double *b, double *x, double rtol, int maxit, int prec,
                                unsigned flags, axipcg_stats *st, void *stream)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(h);
        AXI_REQUIRE(op && b && x, "NULL argument");
        AXI_REQUIRE(b != x, "b and x must not alias");
        AXI_REQUIRE(std::isfinite(rtol) && rtol > 0, "rtol must be > 0");
        AXI_REQUIRE(maxit >= 1 && maxit <= 100000, "maxit must be in [1, 100000]");
        AXI_REQUIRE(prec == AXIPCG_PREC_FP32 || prec == AXIPCG_PREC_FP64, "prec must be 0 or 1");
        AXI_REQUIRE((flags & ~3u) == 0, "unknown flags");
        return solve_impl(*op, b, x, rtol, maxit, prec, flags, st, (hipStream_t)stream);
    });
}
