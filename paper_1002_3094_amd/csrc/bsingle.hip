// Batched PCG in one cooperative launch (§2.2 eq. (8) for every problem of the
// batch; the series setting of §1 eq. (1) with one operator per problem).
//
// The grid (every workgroup resident, as many as the occupancy allows) walks
// the phases of the multi-launch batch in order, with a grid barrier
// (gridbar.h) between phases:
//   start      r = b - A x, ||r||^2, ||b||^2          items: rows
//              forward z-transform of r              items: transform blocks
//              start test; r-solves                  items: mode groups
//              x = 0 where b = 0; inverse, r.z       items: rows; transform blocks
//   iteration  SpMV: beta, p update, q = A p, p.q   items: SpMV tiles
//              alpha; x, r update; forward           items: transform blocks
//              stop test; r-solves                   items: mode groups
//              inverse transform, r.z                items: transform blocks
// A phase deals its items to the workgroups round-robin.  An item is one
// workgroup of the multi-launch form (spmv.h, xform.h), so every problem
// goes through the operations of the multi-launch batch in the same order
// (partial sums and stop test included); only the compiler's choice of fused
// multiply-adds in this kernel's code can differ, by rounding.  After the stop test's barrier every workgroup reads all
// problems' flags (no phase writes them again before the next barrier), so
// the whole grid leaves the iteration loop together once no problem runs.
// Workgroup 0 then copies the states out for a single read-back.  A barrier
// that gives up sets the error word and the kernel returns.
#include "gridbar.h"
#include "spmv.h"
#include "xform.h"

namespace axipcg {
namespace {

constexpr int MAX_PLANS = 5;

struct SingleArgs {
    const ProbDesc *d;    // by problem (row_start, tri_start)
    const ProbDesc *dp;   // by transform plan (tr_start counted within the plan)
    int n, rows, tri, spt, nplan;
    int r2[MAX_PLANS], off[MAX_PLANS], np[MAX_PLANS], twl[MAX_PLANS];
    int base[MAX_PLANS + 1];   // first transform item of each plan
    TriGate g_start, g_step;
    int M, maxit;
    unsigned *bar;
    int *err;
    PcgState *out;
};

// PH 0: start forward (plain), 1: step forward (fused), 2: start inverse,
// 3: step inverse.
template <typename T, int PH, int R2>
__device__ __forceinline__ void wave_item(const ProbDesc *d, int n, int g, int parity, bool pr)
{
    static_assert(wave_rows<T, R2>() == 4, "one row per wave of a 256-thread workgroup");
    if constexpr (PH == 0) b_zfwd_w_item<T, false, R2, true>(d, n, g, parity);
    else if constexpr (PH == 1) b_zfwd_w_item<T, true, R2, true>(d, n, g, parity);
    else if constexpr (PH == 2) b_zinv_w_item<T, 2, R2>(d, n, g, false);
    else b_zinv_w_item<T, 1, R2>(d, n, g, pr);
}

template <typename T, int PH, bool TWLDS>
__device__ __forceinline__ void block_item(const ProbDesc *d, int n, int g, int parity, bool pr)
{
    if constexpr (PH == 0) b_zfwd_item<T, false, TWLDS, true>(d, n, g, parity);
    else if constexpr (PH == 1) b_zfwd_item<T, true, TWLDS, true>(d, n, g, parity);
    else if constexpr (PH == 2) b_zinv_item<T, 2, TWLDS>(d, n, g, false);
    else b_zinv_item<T, 1, TWLDS>(d, n, g, pr);
}

template <typename T, int RMAX, int PH>
__device__ __forceinline__ void tr_phase(const SingleArgs &A, int parity, bool pr)
{
    const int total = A.base[A.nplan];
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        int pl = 0;
        while (t >= A.base[pl + 1]) ++pl;
        const ProbDesc *d = A.dp + A.off[pl];
        const int n = A.np[pl], g = t - A.base[pl];
        switch (A.r2[pl]) {
        case 2: wave_item<T, PH, 2>(d, n, g, parity, pr); break;
        case 4: wave_item<T, PH, 4>(d, n, g, parity, pr); break;
        case 8:
            if constexpr (RMAX >= 8) wave_item<T, PH, 8>(d, n, g, parity, pr);
            break;
        case 16:
            if constexpr (RMAX >= 16) wave_item<T, PH, 16>(d, n, g, parity, pr);
            break;
        default:
            if (A.twl[pl]) block_item<T, PH, true>(d, n, g, parity, pr);
            else block_item<T, PH, false>(d, n, g, parity, pr);
        }
        __syncthreads();   // the item's LDS is free for the next one
    }
}

template <typename T>
__device__ __forceinline__ void tri_phase(const SingleArgs &A, const TriGate &g)
{
    for (int t = blockIdx.x; t < A.tri; t += gridDim.x) {
        b_tridiag_item<T>(A.d, A.n, g, A.M, t);
        __syncthreads();
    }
}

// Whether some problem still runs, as one value for the whole workgroup.
__device__ inline bool any_running(const SingleArgs &A)
{
    int run = 0;
    for (int p = threadIdx.x; p < A.n; p += blockDim.x) run |= (A.d[p].state->done == ST_RUN) ? 1 : 0;
    return __syncthreads_or(run) != 0;
}

template <typename T, int RMAX, bool PR>
__device__ __forceinline__ bool single_run(const SingleArgs &A, int *flag)
{
    const int G = gridDim.x;
    unsigned target = 0;
    auto sync = [&]() { return grid_sync(A.bar, G, ++target, flag); };

    for (int g = blockIdx.x; g < A.rows; g += G) {
        b_init_item(A.d, A.n, g);
        __syncthreads();
    }
    if (!sync()) return false;
    tr_phase<T, RMAX, 0>(A, 0, false);
    if (!sync()) return false;
    tri_phase<T>(A, A.g_start);
    if (!sync()) return false;
    for (int g = blockIdx.x; g < A.rows; g += G) {
        b_zero_item(A.d, A.n, g);
        __syncthreads();
    }
    tr_phase<T, RMAX, 2>(A, 0, false);
    if (!sync()) return false;

    int parity = 0;
    for (int it = 0; it < A.maxit && any_running(A); ++it) {
        for (int g = blockIdx.x; g < A.spt; g += G) {
            b_spmv_item<PR>(A.d, A.n, g, parity);
            __syncthreads();
        }
        if (!sync()) return false;
        tr_phase<T, RMAX, 1>(A, parity, PR);
        if (!sync()) return false;
        tri_phase<T>(A, A.g_step);
        if (!sync()) return false;
        if (!any_running(A)) break;
        tr_phase<T, RMAX, 3>(A, parity, PR);
        if (!sync()) return false;
        parity ^= 1;
    }
    return true;
}

// RMAX: the largest one-wave transform plan (R2) of the batch; the kernel
// holds no larger plan's code, whose registers would set its occupancy.
template <typename T, int RMAX, bool PR>
__global__ void __launch_bounds__(256) k_b_single(SingleArgs A)
{
    __shared__ int flag;
    if (!single_run<T, RMAX, PR>(A, &flag)) {
        if (threadIdx.x == 0) __hip_atomic_store(A.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    if (blockIdx.x == 0)
        for (int p = threadIdx.x; p < A.n; p += blockDim.x) A.out[p] = *A.d[p].state;
}

// Rows of up to 1024 points (R2 <= 8): the 2048-point one-wave plan alone
// needs about 500 registers, which the single kernel would spill.
const void *single_kernel(int prec, int rmax, bool pr)
{
    AXI_REQUIRE(rmax <= 8, "the single-launch batch takes rows of up to 1024 points");
    if (prec == AXIPCG_PREC_FP32)
        return pr ? (const void *)k_b_single<float, 8, true> : (const void *)k_b_single<float, 8, false>;
    return pr ? (const void *)k_b_single<double, 8, true> : (const void *)k_b_single<double, 8, false>;
}

}  // namespace

int batch_single_grid(int prec, int rmax, bool pr, size_t shm)
{
    const void *fn = single_kernel(prec, rmax, pr);
    int dev = 0, coop = 0, cus = 0, per_cu = 0;
    AXI_CHECK_HIP(hipGetDevice(&dev));
    AXI_CHECK_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    AXI_REQUIRE(coop, "the device does not support cooperative launches");
    AXI_CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    hipFuncAttributes attr;
    AXI_CHECK_HIP(hipFuncGetAttributes(&attr, fn));
    AXI_REQUIRE(attr.sharedSizeBytes + shm <= 160 * 1024, "the single-launch batch needs more LDS than a CU has");
    if (attr.sharedSizeBytes + shm > 65536)
        AXI_CHECK_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    AXI_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, shm));
    AXI_REQUIRE(per_cu >= 1, "the single-launch batch kernel does not fit on a compute unit");
    return per_cu * cus;
}

void launch_b_single(const BatchSingle &b, int prec, int rmax, bool pr, int grid, size_t shm, hipStream_t s)
{
    AXI_REQUIRE(b.nplan >= 1 && b.nplan <= MAX_PLANS, "bad transform plan count");
    SingleArgs a{};
    a.d = b.d;
    a.dp = b.dp;
    a.n = b.n;
    a.rows = b.rows;
    a.tri = b.tri;
    a.spt = b.spt;
    a.nplan = b.nplan;
    a.base[0] = 0;
    for (int i = 0; i < b.nplan; ++i) {
        a.r2[i] = b.plans[i].r2;
        a.off[i] = b.plans[i].off;
        a.np[i] = b.plans[i].n;
        a.twl[i] = b.twl[i] ? 1 : 0;
        a.base[i + 1] = a.base[i] + b.plans[i].blocks;
    }
    a.g_start = b.g_start;
    a.g_step = b.g_step;
    a.M = b.M;
    a.maxit = b.maxit;
    a.bar = b.bar;
    a.err = b.err;
    a.out = b.out;
    void *args[] = {&a};
    AXI_CHECK_HIP(hipLaunchCooperativeKernel(single_kernel(prec, rmax, pr), dim3(grid), dim3(256), args, (unsigned)shm, s));
}

}  // namespace axipcg
