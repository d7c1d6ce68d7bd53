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
// Device-side PCG scalars.  One instance per operator, written only by the
// "last block" of the kernel that completes a reduction.
// ---------------------------------------------------------------------------
struct PcgState {
    double rho;      // r . z of the current iterate
    double alpha;    // rho / (p . Ap)
    double beta;     // rho_new / rho_old
    double rr;       // ||r||^2
    double bb;       // ||b||^2
    double tol2;     // rtol^2 ||b||^2
    double rz_old;   // r_new . z_old (Polak-Ribiere)
    double pad0;
    int done;        // 0 running, 1 converged, 2 breakdown
    int iters;       // completed iterations
    int maxit;
    int flags;
};

// Reduction slots: each fused kernel owns one ticket counter and one
// partial-sum array in the operator's workspace.
enum Slot { SLOT_PQ = 0, SLOT_RR = 1, SLOT_RZ = 2, SLOT_MISC = 3, SLOT_RZOLD = 4, NUM_SLOTS = 5 };

constexpr int MAX_PARTIALS = 16384;

struct Operator {
    int nr = 0, nz = 0, bc_z = 0;
    double lr = 0, lz = 0, hr = 0, hz = 0;
    double kbar = 0, qbar = 0;
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
    double *partials = nullptr;    // [NUM_SLOTS][MAX_PARTIALS]
    unsigned *tickets = nullptr;   // [NUM_SLOTS] (64-byte strided)
    PcgState *state = nullptr;
    double *dscal = nullptr;         // 16 device scalars (residual norms)
    PcgState *state_host = nullptr;  // pinned mirror
    double *scratch_host = nullptr;  // pinned host scalars

    // per-kernel timing (axipcg_profile_*)
    int prof_kernel = -1;
    std::vector<hipEvent_t> prof_events;  // pairs (start, stop)
    std::vector<int> prof_iter;           // iteration of each pair
    size_t prof_used = 0;
    double prof_ms = 0.0;
    long long prof_count = 0;
};

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

__device__ inline double load_agent(const double *p)
{
    unsigned long long u = __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p),
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double(static_cast<long long>(u));
}

// Publish this block's partial sum; returns true in every thread of the block
// that finishes last.  That block then sees every partial through
// load_agent().  The ticket is reset by the last block.
__device__ inline bool publish_partial(double blocksum, double *partials, unsigned *ticket,
                                       unsigned nblocks, int bid)
{
    __shared__ int am_last;
    if (threadIdx.x == 0) {
        __hip_atomic_store(reinterpret_cast<unsigned long long *>(partials + bid),
                           static_cast<unsigned long long>(__double_as_longlong(blocksum)),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        am_last = (t == nblocks - 1);
        if (am_last) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return am_last != 0;
}

// Sum of partials[0..n) in a fixed order (strided per thread, then the block
// tree); valid in thread 0.
__device__ inline double sum_partials(const double *partials, unsigned n, double *sm)
{
    double s = 0.0;
    for (unsigned i = threadIdx.x; i < n; i += blockDim.x) s += load_agent(partials + i);
    return block_sum(s, sm);
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
