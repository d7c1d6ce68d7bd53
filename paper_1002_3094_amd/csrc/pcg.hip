// PCG (§2.2 eq. (8) with conjugate-gradient parameters) on gfx950.
//
// One iteration k is four stream-ordered launches.  Each kernel writes one
// partial sum per workgroup; the next kernel's workgroups each sum those
// partials in the same fixed order and take the same decision, so the host
// never waits inside an iteration and no atomics are needed:
//   1. SpMV:    rho_k = sum(r.z partials), beta = rho_k / rho_{k-1};
//               p = z + beta p_old (ping-pong buffers), q = A p, p.q partials
//   2. forward: alpha = rho_k / p.q; x += alpha p, r -= alpha q, ||r||^2
//               partials; z-transform of r
//   3. r-solve: ||r||^2 -> stop test (sets `done`); r-tridiagonal solves
//   4. inverse: inverse z-transform -> z, r.z partials
// After the stop test fires, the remaining launches of the chunk return at
// once.  The host follows the solve through a progress record that the stop
// test publishes to pinned host memory (HostMirror), normally once per solve.
#include <atomic>
#include <cmath>

#include <hip/hip_ext.h>

#include <climits>

#include "kernels.h"
#include "spmv.h"

namespace axipcg {

void resid_impl(const Operator &op, const double *b, const double *x, double *out_dev, hipStream_t s);

namespace {

inline unsigned row_blocks(int nr) { return (unsigned)(nr < MAX_PARTIALS ? nr : MAX_PARTIALS); }

template <bool PR, int RW>
__global__ void __launch_bounds__(256)
k_pcg_spmv(const double *__restrict__ z, const double *__restrict__ pold, double *__restrict__ pnew,
           double *__restrict__ q, const double *__restrict__ D, const double *__restrict__ CR,
           const double *__restrict__ CZ, int nr, int nz, PcgState *st, double *__restrict__ partials, int n_rz)
{
    spmv_tiles<PR, RW>(z, pold, pnew, q, D, CR, CZ, nr, nz, st, partials, n_rz, blockIdx.x, gridDim.x);
}

// Rows per SpMV tile: 16 when that still leaves 512 tiles or more (long
// windows: the halo is 2/16 of the rows), else 2 (more tiles to fill the
// chip); the workgroups, at most MAX_PARTIALS, loop over the tiles.
int spmv_rows(int nr, int nz)
{
    const long nc = (nz + SPMV_CHUNK - 1) / SPMV_CHUNK;
    return ((long)(nr / 16) * nc >= 512) ? 16 : 2;
}

unsigned spmv_blocks(int nr, int nz)
{
    const int rw = spmv_rows(nr, nz);
    const long tiles = (long)((nr + rw - 1) / rw) * ((nz + SPMV_CHUNK - 1) / SPMV_CHUNK);
    return (unsigned)(tiles < MAX_PARTIALS ? tiles : MAX_PARTIALS);
}

// Chebyshev step of eq. (8) (spmv.h), the workgroups looping over the rows.
__global__ void __launch_bounds__(256)
k_cheb_update(const double *__restrict__ d, double *__restrict__ x, double *__restrict__ r,
              const double *__restrict__ D, const double *__restrict__ CR, const double *__restrict__ CZ, int nr,
              int nz, PcgState *st, double *__restrict__ partials)
{
    cheb_update_body(d, x, r, D, CR, CZ, nr, nz, st, partials, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(256)
k_pcg_init(const double *__restrict__ b, const double *__restrict__ x, double *__restrict__ r,
           const double *__restrict__ D, const double *__restrict__ CR, const double *__restrict__ CZ, int nr,
           int nz, double *__restrict__ partials)
{
    init_body(b, x, r, D, CR, CZ, nr, nz, partials, blockIdx.x, gridDim.x);
}

// ---- batched launches: one launch covers every problem of a batch --------
// One work item (spmv.h) per workgroup.
template <bool PR>
__global__ void __launch_bounds__(256) k_b_spmv(const ProbDesc *__restrict__ d, int n, int parity)
{
    b_spmv_item<PR>(d, n, blockIdx.x, parity);
}

__global__ void __launch_bounds__(256) k_b_cheb(const ProbDesc *__restrict__ d, int n)
{
    b_cheb_item(d, n, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_b_init(const ProbDesc *__restrict__ d, int n)
{
    b_init_item(d, n, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_b_zero_if_b_zero(const ProbDesc *__restrict__ d, int n)
{
    b_zero_item(d, n, blockIdx.x);
}

// Copy every problem's state into one array (one read-back per chunk).
__global__ void k_b_gather(const ProbDesc *__restrict__ d, int n, PcgState *out)
{
    for (int p = threadIdx.x; p < n; p += blockDim.x) out[p] = *d[p].state;
}

// x = 0 when b = 0.
__global__ void k_zero_if_b_zero(double *__restrict__ x, size_t n, const PcgState *st)
{
    if (st->done != ST_BZERO) return;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        x[e] = 0.0;
}

struct SolveCtx {
    Operator *op;
    double *x;
    int prec;
    bool pr;
    hipStream_t s;
    int n_tr;   // workgroups (partials) of the transform kernels
    unsigned seq = 0;     // solve number published through the host mirror
    int report_it = -1;   // iteration whose stop test publishes even without a stop
    bool one = false;     // iterations through the single-launch preconditioner
};

// Event pair around one launch of the profiled kernel class.  With `ext`
// the launch site hands the pair to hipExtLaunchKernelGGL, which stamps them
// from the dispatch itself (no separate event packets around the kernel);
// otherwise the events are recorded on the stream before and after it.
struct ProfScope {
    Operator &op;
    hipStream_t s;
    bool on;
    bool ext;
    size_t slot = 0;
    ProfScope(Operator &o, hipStream_t st, int kernel, int iter, bool ext_launch = false)
        : op(o), s(st), on(o.prof_kernel == kernel && (o.prof_seen++ % o.prof_every) == 0), ext(ext_launch)
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
        if (!ext) AXI_CHECK_HIP(hipEventRecord(op.prof_events[2 * slot], s));
    }
    hipEvent_t start() const { return on ? op.prof_events[2 * slot] : nullptr; }
    hipEvent_t stop() const { return on ? op.prof_events[2 * slot + 1] : nullptr; }
    // Never throws (it may run during unwinding): a failed stop record drops
    // the sample and marks the profile, which axipcg_profile_read reports.
    ~ProfScope() noexcept
    {
        if (on && !ext && hipEventRecord(op.prof_events[2 * slot + 1], s) != hipSuccess) {
            op.prof_error = true;
            op.prof_iter[slot] = INT_MAX;   // dropped by collect_profile
        }
    }
};

void launch_iteration(const SolveCtx &c, int parity, int iter)
{
    Operator &op = *c.op;
    double *pold = parity ? op.p1 : op.p0;
    double *pnew = parity ? op.p0 : op.p1;
    const unsigned gs = spmv_blocks(op.nr, op.nz);
    {
        ProfScope ps(op, c.s, AXIPCG_KERNEL_SPMV, iter, true);
#define AXI_SPMV(PRV, RWV)                                                                                           \
    hipExtLaunchKernelGGL((k_pcg_spmv<PRV, RWV>), dim3(gs), dim3(256), 0, c.s, ps.start(), ps.stop(), 0, op.z, pold, \
                          pnew, op.q, op.D, op.CR, op.CZ, op.nr, op.nz, op.state, op.partials, c.n_tr)
        const bool long_tiles = spmv_rows(op.nr, op.nz) == 16;
        if (c.pr) {
            if (long_tiles) AXI_SPMV(true, 16);
            else AXI_SPMV(true, 2);
        } else {
            if (long_tiles) AXI_SPMV(false, 16);
            else AXI_SPMV(false, 2);
        }
#undef AXI_SPMV
        AXI_CHECK_HIP(hipGetLastError());
    }
    ZfwdArgs fa;
    fa.fused = true;
    fa.x = c.x;
    fa.r = op.r;
    fa.p = pnew;
    fa.q = op.q;
    fa.state = op.state;
    fa.n_pq = (int)gs;
    TriGate g;
    g.mode = 1;
    g.state = op.state;
    g.n_rr = c.n_tr;
    g.mirror = op.mirror_dev;
    g.seq = c.seq;
    g.report = iter == c.report_it;
    ZinvArgs ia;
    ia.zout = op.z;
    ia.r = op.r;
    ia.state = op.state;
    ia.mode = 1;
    ia.pr = c.pr;
    if (c.one) {
        // the preconditioner phases in one cooperative launch (timed as the
        // forward-transform class)
        ProfScope ps(op, c.s, AXIPCG_KERNEL_ZFWD, iter);
        pfused_pcg_step(op, fa, g, ia, c.s);
        return;
    }
    {
        ProfScope ps(op, c.s, AXIPCG_KERNEL_ZFWD, iter);
        launch_zfwd(op, c.prec, fa, c.s);
    }
    {
        ProfScope ps(op, c.s, AXIPCG_KERNEL_TRIDIAG, iter);
        launch_tridiag(op, c.prec, g, c.s);
    }
    {
        ProfScope ps(op, c.s, AXIPCG_KERNEL_ZINV, iter);
        launch_zinv(op, c.prec, ia, c.s);
    }
}

// Add the timed launches that did work: the SpMV and forward kernels of
// iterations 0..iters-1, the r-solve and inverse of iterations 0..iters-2
// (the last r-solve launch only runs the stop test).
void collect_profile(Operator &op, int iters)
{
    for (size_t k = 0; k < op.prof_used; ++k) {
        const int it = op.prof_iter[k];
        const int limit = (op.prof_kernel == AXIPCG_KERNEL_SPMV || op.prof_kernel == AXIPCG_KERNEL_ZFWD)
                              ? iters : iters - 1;
        if (it >= limit) continue;
        float ms = 0.f;
        // complete (they precede the stop test in stream order); the wait
        // only covers the completion notice reaching the runtime
        AXI_CHECK_HIP(hipEventSynchronize(op.prof_events[2 * k + 1]));
        AXI_CHECK_HIP(hipEventElapsedTime(&ms, op.prof_events[2 * k], op.prof_events[2 * k + 1]));
        op.prof_ms += ms;
        op.prof_count += 1;
    }
    op.prof_used = 0;
}

// Wait until solve `seq` has published a stop, or (need >= 0) at least
// `need` finished iterations, through the host mirror.  Should the stream
// drain first (a stop that no r-solve launch publishes, such as a breakdown
// found by the forward transform), the device state is read instead.
PcgState wait_progress(Operator &op, hipStream_t s, unsigned seq, int need)
{
    const volatile unsigned long long *w = &op.mirror_host->word;
    for (unsigned spin = 1;; ++spin) {
        const unsigned long long v = *w;
        if ((unsigned)(v >> 32) == seq) {
            const int done = (int)(v & 0xffu), iters = (int)((v >> 8) & 0xffffffu);
            if (done != ST_RUN || (need >= 0 && iters >= need)) {
                std::atomic_thread_fence(std::memory_order_acquire);
                PcgState h{};
                h.done = done;
                h.iters = iters;
                h.rr = static_cast<const volatile double &>(op.mirror_host->rr);
                h.bb = static_cast<const volatile double &>(op.mirror_host->bb);
                return h;
            }
        }
        if ((spin & 31u) == 0) {
            const hipError_t e = hipStreamQuery(s);
            if (e == hipSuccess) {
                AXI_CHECK_HIP(hipMemcpyAsync(op.state_host, op.state, sizeof(PcgState), hipMemcpyDeviceToHost, s));
                AXI_CHECK_HIP(hipStreamSynchronize(s));
                return *op.state_host;
            }
            if (e != hipErrorNotReady) AXI_CHECK_HIP(e);
        }
        __builtin_ia32_pause();
    }
}

int solve_impl(Operator &op, const double *b, double *x, double rtol, int maxit, int prec, unsigned flags,
               axipcg_stats *st, hipStream_t s, bool sync_end)
{
    const size_t n = (size_t)op.nr * op.nz;
    SolveCtx c{&op, x, prec, (flags & AXIPCG_FLAG_POLAK_RIBIERE) != 0, s, transform_blocks(op, prec)};
    c.seq = ++op.mirror_seq;
    // the single launch keeps the three-launch strips' partial counts (4-row
    // strips), and has no Polak-Ribiere form
    c.one = op.fused_enabled && prec == AXIPCG_PREC_FP32 && !c.pr && pfused_plan(op, AXIPCG_FUSED_PCG) &&
            op.pf[AXIPCG_FUSED_PCG].G == c.n_tr;
    op.prof_used = 0;
    // start: r = b - A x; z = B^{-1} r (the r-solve launch runs the start test)
    const unsigned gi = row_blocks(op.nr);
    hipLaunchKernelGGL(k_pcg_init, dim3(gi), dim3(256), 0, s, b, x, op.r, op.D, op.CR, op.CZ, op.nr, op.nz,
                       op.partials);
    AXI_CHECK_HIP(hipGetLastError());
    ZfwdArgs fa;
    fa.rin = op.r;
    launch_zfwd(op, prec, fa, s);
    TriGate g;
    g.mode = 2;
    g.state = op.state;
    g.n_rr = (int)gi;
    g.rtol2 = rtol * rtol;
    g.maxit = maxit;
    g.flags = (int)flags;
    g.mirror = op.mirror_dev;
    g.seq = c.seq;
    launch_tridiag(op, prec, g, s);
    hipLaunchKernelGGL(k_zero_if_b_zero, dim3(pointwise_blocks(n)), dim3(256), 0, s, x, n, op.state);
    AXI_CHECK_HIP(hipGetLastError());
    ZinvArgs ia;
    ia.zout = op.z;
    ia.r = op.r;
    ia.state = op.state;
    ia.mode = 2;
    launch_zinv(op, prec, ia, s);

    // iterations, in chunks: the first one covers the previous solve's
    // count, so a series of similar solves needs one chunk each (the launches
    // past the stop test return at once, but still cost a few microseconds
    // each).  The host follows the solve through the mirror: the stop test
    // publishes a stop at once, and the last iteration of a chunk publishes
    // its progress; only then is a further chunk queued, which leaves a short
    // gap but never more than one iteration of no-op launches.
    int launched = 0;
    int parity = 0;
    int chunk = op.last_iters > 0 ? op.last_iters : 4;
    PcgState h{};
    for (;;) {
        if (chunk > maxit - launched) chunk = maxit - launched;
        c.report_it = launched + chunk - 1;
        for (int it = 0; it < chunk; ++it) {
            launch_iteration(c, parity, launched + it);
            parity ^= 1;
        }
        launched += chunk;
        h = wait_progress(op, s, c.seq, launched >= maxit ? -1 : c.report_it + 1);
        if (h.done != ST_RUN || launched >= maxit) break;
        chunk = 2;
    }
    op.last_iters = h.iters;
    if (op.prof_kernel >= 0) collect_profile(op, h.iters);
    int status;
    if (h.done == ST_CONV || h.done == ST_BZERO) status = AXIPCG_OK;
    else if (h.done == ST_BREAK) status = AXIPCG_EBREAKDOWN;
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
    if (sync_end) AXI_CHECK_HIP(hipStreamSynchronize(s));
    return status;
}

// Chebyshev form of eq. (8): start r = b - A x, z = B^{-1} r (start test),
// d = tau z; then per iteration x += d, r -= A d (||r||^2), forward
// transform, r-solves (stop test), inverse transform forming the next d.  No
// dot products beyond ||r||^2 for the stop test.
int cheb_solve_impl(Operator &op, const double *b, double *x, double gamma1, double gamma2, double rtol, int maxit,
                    int prec, axipcg_stats *st, hipStream_t s, bool sync_end)
{
    const unsigned seq = ++op.mirror_seq;
    const size_t n = (size_t)op.nr * op.nz;
    const double tau = 2.0 / (gamma1 + gamma2);
    const double xi = gamma1 / gamma2;
    const double rho2 = ((1.0 - xi) / (1.0 + xi)) * ((1.0 - xi) / (1.0 + xi));
    double *d = op.p0;   // the increment lives in the first search-direction buffer
    const unsigned gi = row_blocks(op.nr);
    hipLaunchKernelGGL(k_pcg_init, dim3(gi), dim3(256), 0, s, b, x, op.r, op.D, op.CR, op.CZ, op.nr, op.nz,
                       op.partials);
    AXI_CHECK_HIP(hipGetLastError());
    ZfwdArgs fa;
    fa.rin = op.r;
    launch_zfwd(op, prec, fa, s);
    TriGate g;
    g.mode = 2;
    g.state = op.state;
    g.n_rr = (int)gi;
    g.rtol2 = rtol * rtol;
    g.maxit = maxit;
    g.flags = 0;
    g.mirror = op.mirror_dev;
    g.seq = seq;
    launch_tridiag(op, prec, g, s);
    hipLaunchKernelGGL(k_zero_if_b_zero, dim3(pointwise_blocks(n)), dim3(256), 0, s, x, n, op.state);
    AXI_CHECK_HIP(hipGetLastError());
    ZinvArgs ia;
    ia.state = op.state;
    ia.mode = 4;
    ia.d = d;
    ia.tau = tau;
    ia.rho2 = rho2;
    launch_zinv(op, prec, ia, s);

    ZfwdArgs ga;
    ga.rin = op.r;
    ga.state = op.state;
    TriGate g1;
    g1.mode = 1;
    g1.state = op.state;
    g1.n_rr = (int)gi;
    g1.mirror = op.mirror_dev;
    g1.seq = seq;
    ZinvArgs ib = ia;
    ib.mode = 3;
    int launched = 0;
    int chunk = op.last_iters > 0 ? op.last_iters : 4;
    PcgState h{};
    for (;;) {
        if (chunk > maxit - launched) chunk = maxit - launched;
        const int report_it = launched + chunk - 1;
        for (int it = 0; it < chunk; ++it) {
            hipLaunchKernelGGL(k_cheb_update, dim3(gi), dim3(256), 0, s, d, x, op.r, op.D, op.CR, op.CZ, op.nr, op.nz,
                               op.state, op.partials);
            AXI_CHECK_HIP(hipGetLastError());
            launch_zfwd(op, prec, ga, s);
            g1.report = launched + it == report_it;
            launch_tridiag(op, prec, g1, s);
            launch_zinv(op, prec, ib, s);
        }
        launched += chunk;
        h = wait_progress(op, s, seq, launched >= maxit ? -1 : report_it + 1);
        if (h.done != ST_RUN || launched >= maxit) break;
        chunk = 2;
    }
    op.last_iters = h.iters;
    int status;
    if (h.done == ST_CONV || h.done == ST_BZERO) status = AXIPCG_OK;
    else if (h.done == ST_BREAK) status = AXIPCG_EBREAKDOWN;
    else status = AXIPCG_ENOTCONV;
    if (st) {
        st->iters = h.iters;
        st->status = status;
        st->relres_rec = (h.bb > 0) ? std::sqrt(h.rr / h.bb) : 0.0;
        st->relres_true = -1.0;
    }
    if (sync_end) AXI_CHECK_HIP(hipStreamSynchronize(s));
    return status;
}

}  // namespace

void launch_b_spmv(const ProbDesc *d, int n, int tiles, bool pr, int parity, hipStream_t s)
{
    if (pr) hipLaunchKernelGGL(k_b_spmv<true>, dim3(tiles), dim3(256), 0, s, d, n, parity);
    else hipLaunchKernelGGL(k_b_spmv<false>, dim3(tiles), dim3(256), 0, s, d, n, parity);
    AXI_CHECK_HIP(hipGetLastError());
}

void launch_b_cheb(const ProbDesc *d, int n, int rows, hipStream_t s)
{
    hipLaunchKernelGGL(k_b_cheb, dim3(rows), dim3(256), 0, s, d, n);
    AXI_CHECK_HIP(hipGetLastError());
}

void launch_b_init(const ProbDesc *d, int n, int rows, hipStream_t s)
{
    hipLaunchKernelGGL(k_b_init, dim3(rows), dim3(256), 0, s, d, n);
    AXI_CHECK_HIP(hipGetLastError());
}

void launch_b_zero(const ProbDesc *d, int n, int rows, hipStream_t s)
{
    hipLaunchKernelGGL(k_b_zero_if_b_zero, dim3(rows), dim3(256), 0, s, d, n);
    AXI_CHECK_HIP(hipGetLastError());
}

void launch_b_gather(const ProbDesc *d, int n, PcgState *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_b_gather, dim3(1), dim3(256), 0, s, d, n, out);
    AXI_CHECK_HIP(hipGetLastError());
}

}  // namespace axipcg

using namespace axipcg;

extern "C" int axipcg_profile_select(axipcg_op_t h, int kernel, int every)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(h);
        AXI_REQUIRE(op != nullptr, "op is NULL");
        AXI_REQUIRE(kernel >= AXIPCG_KERNEL_NONE && kernel <= AXIPCG_KERNEL_ZINV, "unknown kernel class");
        AXI_REQUIRE(every >= 1, "every must be >= 1");
        op->prof_kernel = kernel;
        op->prof_every = every;
        op->prof_seen = 0;
        op->prof_used = 0;
        return AXIPCG_OK;
    });
}

extern "C" int axipcg_profile_read(axipcg_op_t h, double *total_ms, long long *launches, int reset)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(h);
        AXI_REQUIRE(op != nullptr, "op is NULL");
        if (op->prof_error) {
            op->prof_error = false;
            throw Error{AXIPCG_EDEVICE, "a profiling event could not be recorded; samples were dropped"};
        }
        if (total_ms) *total_ms = op->prof_ms;
        if (launches) *launches = op->prof_count;
        if (reset) {
            op->prof_ms = 0.0;
            op->prof_count = 0;
        }
        return AXIPCG_OK;
    });
}

namespace axipcg {
int pcg_solve_entry(axipcg_op_t h, const double *b, double *x, double rtol, int maxit, int prec, unsigned flags,
                    axipcg_stats *st, void *stream, bool sync_end)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(h);
        AXI_REQUIRE(op && b && x, "NULL argument");
        AXI_REQUIRE(b != x, "b and x must not alias");
        AXI_REQUIRE(std::isfinite(rtol) && rtol > 0, "rtol must be > 0");
        AXI_REQUIRE(maxit >= 1 && maxit <= 100000, "maxit must be in [1, 100000]");
        AXI_REQUIRE(prec == AXIPCG_PREC_FP32 || prec == AXIPCG_PREC_FP64, "prec must be 0 or 1");
        AXI_REQUIRE((flags & ~3u) == 0, "unknown flags");
        return solve_impl(*op, b, x, rtol, maxit, prec, flags, st, (hipStream_t)stream, sync_end);
    });
}

int cheb_solve_entry(axipcg_op_t h, const double *b, double *x, double gamma1, double gamma2, double rtol,
                     int maxit, int prec, axipcg_stats *st, void *stream, bool sync_end)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(h);
        AXI_REQUIRE(op && b && x, "NULL argument");
        AXI_REQUIRE(b != x, "b and x must not alias");
        AXI_REQUIRE(prec == AXIPCG_PREC_FP32 || prec == AXIPCG_PREC_FP64, "prec must be 0 or 1");
        AXI_REQUIRE(rtol > 0 && rtol < 1, "rtol must be in (0, 1)");
        AXI_REQUIRE(maxit >= 1, "maxit must be >= 1");
        if (gamma1 <= 0 && gamma2 <= 0) {
            gamma1 = op->gamma1;
            gamma2 = op->gamma2;
        }
        AXI_REQUIRE(std::isfinite(gamma1) && std::isfinite(gamma2) && gamma1 > 0 && gamma1 <= gamma2,
                    "need 0 < gamma1 <= gamma2 (the operator's own bounds have gamma1 = 0 when some q is 0 "
                    "while qbar > 0)");
        return cheb_solve_impl(*op, b, x, gamma1, gamma2, rtol, maxit, prec, st, (hipStream_t)stream, sync_end);
    });
}
}  // namespace axipcg

extern "C" int axipcg_pcg_solve(axipcg_op_t h, const double *b, double *x, double rtol, int maxit, int prec,
                                unsigned flags, axipcg_stats *st, void *stream)
{
    return pcg_solve_entry(h, b, x, rtol, maxit, prec, flags, st, stream, true);
}

extern "C" int axipcg_cheb_solve(axipcg_op_t h, const double *b, double *x, double gamma1, double gamma2,
                                 double rtol, int maxit, int prec, axipcg_stats *st, void *stream)
{
    return cheb_solve_entry(h, b, x, gamma1, gamma2, rtol, maxit, prec, st, stream, true);
}
