// Shared declarations of the axipcg HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <new>
#include <string>
#include <vector>

#include "axipcg.h"

namespace axipcg {

// ---------------------------------------------------------------------------
// Errors: every ABI entry point returns a code; the message of the last
// failure is kept per host thread.
// ---------------------------------------------------------------------------
struct Error {
    int code;
    std::string msg;
};

void set_last_error(const std::string &msg);
void clear_last_error();

#define AXI_CHECK_HIP(expr)                                                          \
    do {                                                                             \
        hipError_t _e = (expr);                                                      \
        if (_e != hipSuccess)                                                        \
            throw ::axipcg::Error{AXIPCG_EDEVICE, std::string(#expr) + ": " +        \
                                                      hipGetErrorString(_e)};        \
    } while (0)

#define AXI_REQUIRE(cond, text)                                                      \
    do {                                                                             \
        if (!(cond)) throw ::axipcg::Error{AXIPCG_EINVAL, (text)};                   \
    } while (0)

// ---------------------------------------------------------------------------
// Device-side PCG scalars.  No kernel both reads and writes a field: every
// field is written by workgroup 0 of one kernel and read by later kernels
// (kernel boundaries order the accesses).  The scalars of a reduction are
// recomputed by every workgroup of the consuming kernel from the producer's
// per-workgroup partial sums, in a fixed order, so all workgroups agree.
// ---------------------------------------------------------------------------
struct PcgState {
    double rho[2];   // r.z of iteration k at slot k & 1 (SpMV kernel)
    double rr;       // ||r||^2 after the last update (r-solve kernel)
    double bb;       // ||b||^2 (start)
    double tol2;     // rtol^2 ||b||^2 (start)
    double pad[3];
    int done;        // 0 running, 1 converged, 2 breakdown, 3 maxit, 4 b = 0
    int iters;       // completed iterations (r-solve kernel)
    int cur;         // iteration being processed (forward kernel)
    int maxit;
    int flags;
    int pad2[3];
};

// Progress of a solve as the host sees it, in coherent pinned host memory:
// workgroup 0 of an r-solve launch writes it when the stop test fires, and at
// the one iteration of a chunk the host asks for, so that the host can follow
// a solve without draining the stream.  rr and bb first, then (after a
// system-scope fence) word = seq << 32 | iters << 8 | done.
struct HostMirror {
    double rr, bb;
    unsigned long long word;
    unsigned long long pad;
};
__host__ __device__ inline unsigned long long mirror_word(unsigned seq, int iters, int done)
{
    return ((unsigned long long)seq << 32) | ((unsigned long long)((unsigned)iters & 0xffffffu) << 8) |
           (unsigned long long)((unsigned)done & 0xffu);
}

// Reduction slots: each fused kernel owns one ticket counter and one
// partial-sum array in the operator's workspace.
enum Slot { SLOT_PQ = 0, SLOT_RR = 1, SLOT_RZ = 2, SLOT_MISC = 3, SLOT_RZOLD = 4, NUM_SLOTS = 5 };
// PCG kernel status codes stored in PcgState::done
enum { ST_RUN = 0, ST_CONV = 1, ST_BREAK = 2, ST_MAXIT = 3, ST_BZERO = 4 };

constexpr int MAX_PARTIALS = 16384;
// Rows of an operator's partial-sum array: the PCG slots, and up to seven
// rows for the initial-guess guard (one per extrapolation order).
constexpr int PARTIAL_ROWS = 7;
static_assert(PARTIAL_ROWS >= NUM_SLOTS, "partial rows");

// Launch plan of the single-launch preconditioner (pfused.hip) for one kind
// of launch: 0 standalone apply, 1 PCG iteration.
struct PfPlan {
    int state = 0;   // 0 not planned, 1 usable, -1 not usable (three launches)
    int G = 0, R = 0, L2 = 0;   // strips, rows per strip, modes per workgroup of the reduced phase
    size_t shm = 0;
    void *fn = nullptr;
};

struct Operator {
    int nr = 0, nz = 0, bc_z = 0;
    bool nodes = false;              // the paper's node grid (AXIPCG_GRID_NODES)
    double lr = 0, lz = 0, hr = 0, hz = 0;
    double kbar = 0, qbar = 0;
    double gamma1 = 0, gamma2 = 0;   // energy-equivalence bounds of B^{-1} A (eq. (10))
    int device = 0;
    int last_iters = 0;              // iterations of the previous solve (chunk sizing)
    hipStream_t create_stream = nullptr;

    // scheme coefficients (device, [nr][nz]):
    //   D   diagonal of A
    //   CR  coupling of cell (i,k) with (i+1,k)  (0 in the last row)
    //   CZ  coupling of cell (i,k) with (i,k+1)  (0 in the last column)
    //   W   r q
    double *D = nullptr, *CR = nullptr, *CZ = nullptr, *W = nullptr;

    // r-line and mode data of the preconditioner (device):
    //   cb[i]  = rho_{i+1/2} kbar / h_r^2 (i < nr-1), coupling of rows i, i+1
    //   db[i]  = r-part of the diagonal (cb[i] + cb[i-1], outer face doubled)
    //   rw[i]  = r_i
    //   lam[j] = kbar mu_j + qbar (mode j)
    double *cb64 = nullptr, *db64 = nullptr, *rw64 = nullptr, *lam64 = nullptr;
    float *cb32 = nullptr, *db32 = nullptr, *rw32 = nullptr, *lam32 = nullptr;
    // FFT tables for length nz: tw[k] = exp(-2 pi i k / nz), pt[m] = exp(-i pi m / (2 nz))
    double2 *tw64 = nullptr, *pt64 = nullptr;
    float2 *tw32 = nullptr, *pt32 = nullptr;

    // PCG workspace (device)
    double *r = nullptr, *z = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr;
    void *spec = nullptr;          // spectral buffer, nr*nz doubles (used as float or double)
    double *partials = nullptr;    // [PARTIAL_ROWS][MAX_PARTIALS] per-workgroup partial sums
    PcgState *state = nullptr;
    double *dscal = nullptr;         // 24 device scalars: residual norms [0..1], the guard [8..16]
    PcgState *state_host = nullptr;  // pinned copy of the state (read after the stream drains)
    HostMirror *mirror_host = nullptr;   // coherent pinned progress record (host address)
    HostMirror *mirror_dev = nullptr;    // the same, device address
    unsigned mirror_seq = 0;             // number of the current solve
    double *au_cache = nullptr;          // series_run's cache of A u for the guard (POLY_HISTORY arrays)
    double *scratch_host = nullptr;  // pinned host scalars (16)

    // strip-partitioned preconditioner (strip.hip): reduced data of the strips
    // (three [nr / R][nz] arrays, used as float or double); on unless disabled
    void *strip_red = nullptr;
    int strip_rows = 4;   // strip height (4 or 8), 0 = the per-mode r-solve instead

    // single-launch preconditioner (pfused.hip): plans [standalone, PCG]
    PfPlan pf[2];
    bool fused_enabled = false;      // axipcg_op_set_fused
    unsigned *pf_bar = nullptr;      // grid barrier numbers: completed, then one per strip
    int *pf_err = nullptr;           // set when a grid barrier gave up
    unsigned pf_epoch = 0;           // launches so far (barrier numbers 2 epoch + 1, + 2)

    // per-kernel timing (axipcg_profile_*)
    int prof_kernel = -1;
    int prof_every = 1;                   // time one launch in `every` of the class
    long long prof_seen = 0;              // launches of the class since select
    std::vector<hipEvent_t> prof_events;  // pairs (start, stop)
    std::vector<int> prof_iter;           // iteration of each pair
    size_t prof_used = 0;
    double prof_ms = 0.0;
    long long prof_count = 0;
    bool prof_error = false;              // a stop event failed to record (reported by profile_read)
};

// One problem of a batched solve, as the batched kernels see it.  Workgroup g
// of a row-indexed launch belongs to the problem whose [row_start, row_start +
// nr) range holds g; of the r-solve launch, [tri_start, tri_start + nz / M);
// of its transform launch, [tr_start, tr_start + n_tr); of the SpMV launch
// (one tile of BATCH_SPMV_RW rows by SPMV_CHUNK columns per workgroup),
// [sp_start, sp_start + n_sp).
struct ProbDesc {
    int nr, nz, bc_z;
    int row_start, tri_start;
    int tr_start, n_tr;
    int sp_start, n_sp;
    int tri_S, tri_L, tri_Lp, tri_pitch;
    double tau, rho2;   // Chebyshev form: 2 / (gamma1 + gamma2), ((1 - xi) / (1 + xi))^2, xi = gamma1 / gamma2
    const double *b;
    double *x;
    const double *D, *CR, *CZ;
    double *r, *z, *p0, *p1, *q;
    void *spec;
    double *partials;
    PcgState *state;
    const float *cb32, *db32, *rw32, *lam32;
    const double *cb64, *db64, *rw64, *lam64;
    const float2 *tw32, *pt32;
    const double2 *tw64, *pt64;
};

// Index of the problem owning global workgroup g (binary search on the
// starts of the launch's ranges: rows, r-solve mode groups, transform
// workgroups or SpMV tiles).
enum : int { RANGE_ROWS = 0, RANGE_TRI = 1, RANGE_TR = 2, RANGE_SP = 3 };
__device__ inline int find_problem(const ProbDesc *d, int n, int g, int range)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int st = range == RANGE_TRI ? d[mid].tri_start
                       : range == RANGE_TR ? d[mid].tr_start
                       : range == RANGE_SP ? d[mid].sp_start
                                           : d[mid].row_start;
        if (st <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Run an ABI body: translate exceptions into status codes and keep the
// message for axipcg_last_error().
template <typename F>
int guarded(F &&f)
{
    try {
        clear_last_error();
        return f();
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("out of host memory");
        return AXIPCG_ENOMEM;
    } catch (...) {
        set_last_error("unexpected exception");
        return AXIPCG_EDEVICE;
    }
}

inline bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
inline int ilog2(int n) { int l = 0; while ((1 << l) < n) ++l; return l; }

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Scratch doubles for block_sum / block_total in a workgroup of up to 1024
// threads (16 waves, plus the slot block_total publishes the total in).
constexpr int RED_SLOTS = 17;

// Block-wide sum in a fixed order; result valid in thread 0.  `sm` needs
// blockDim.x / 64 doubles.
__device__ inline double block_sum(double v, double *sm)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sm[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) s += sm[i];
    }
    return s;
}

// Sum of parts[0..n) in a fixed order (strided per thread, then the block
// tree), returned in every thread.  `sm` needs blockDim.x / 64 + 1 doubles.
// Each thread issues its (up to eight) loads before the first add, so the
// reads of one round are in flight together rather than one latency apiece.
// total_issue and total_finish split the same sum in two: the first
// round's loads issued early, the additions (in the same order) later.
struct TotalLoads {
    double v[8];
};

__device__ inline void total_issue(const double *__restrict__ parts, int n, TotalLoads &t)
{
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int i = (int)threadIdx.x + j * (int)blockDim.x;
        t.v[j] = (i < n) ? parts[i] : 0.0;
    }
}

__device__ inline double total_finish(const double *__restrict__ parts, int n, const TotalLoads &t, double *sm)
{
    const int nt = blockDim.x;
    double s = 0.0;
    s += ((t.v[0] + t.v[1]) + (t.v[2] + t.v[3])) + ((t.v[4] + t.v[5]) + (t.v[6] + t.v[7]));
    for (int base = 8 * nt; base < n; base += 8 * nt) {
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int i = base + (int)threadIdx.x + j * nt;
            v[j] = (i < n) ? parts[i] : 0.0;
        }
        s += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    }
    s = block_sum(s, sm);
    const int nw = (blockDim.x + 63) >> 6;
    if (threadIdx.x == 0) sm[nw] = s;
    __syncthreads();
    s = sm[nw];
    __syncthreads();
    return s;
}

__device__ inline double block_total(const double *__restrict__ parts, int n, double *sm)
{
    double s = 0.0;
    const int nt = blockDim.x;
    for (int base = 0; base < n; base += 8 * nt) {
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int i = base + (int)threadIdx.x + j * nt;
            v[j] = (i < n) ? parts[i] : 0.0;
        }
        s += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    }
    s = block_sum(s, sm);
    const int nw = (blockDim.x + 63) >> 6;
    if (threadIdx.x == 0) sm[nw] = s;
    __syncthreads();
    s = sm[nw];
    __syncthreads();
    return s;
}

// Map a block index to a logical tile so that each XCD (blocks are dealt to
// the 8 XCDs round-robin) works on one contiguous range of tiles.
__device__ inline int xcd_swizzle(int b, int nb)
{
    const int per = nb >> 3;
    if ((nb & 7) != 0 || per == 0) return b;
    return (b & 7) * per + (b >> 3);
}

}  // namespace axipcg
