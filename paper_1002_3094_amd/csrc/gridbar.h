// Grid barrier of a cooperative launch (every workgroup resident).
//
// bar[0] is the last completed barrier number and bar[1 + w] the last barrier
// number workgroup w has reached.  A launch passes numbers that only grow
// (from a counter kept across launches, or from zeroed flags), so a flag left
// behind by an earlier launch, even one whose barrier gave up, is always
// below the number a later barrier waits for and can never let it through
// early.  Each workgroup releases its stores at agent scope (the XCDs' L2s
// are not coherent with each other otherwise) and posts its flag; workgroup
// 0 waits for every flag, acquires, and publishes the number; the others wait
// for it and acquire.  Every wait is bounded: grid_sync returns false when a
// wait runs past the spin limit, and the caller then ends its work.
#pragma once

#include "common.h"

namespace axipcg {
namespace {

constexpr unsigned long long ONE_SPIN_LIMIT = 1ull << 20;

__device__ inline bool one_wait(const unsigned *w, unsigned target)
{
    unsigned long long n = 0;
    while ((int)(__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
        if (++n > ONE_SPIN_LIMIT) return false;
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// One release and one acquire per workgroup (thread 0), the workgroup's own
// ordering through its barriers: an agent-scope fence writes back / drops
// the XCD's L2, so one per wave would repeat that work many times over.
__device__ inline bool grid_sync(unsigned *bar, int nblk, unsigned target, int *flag_lds)
{
    // each wave's own global stores acknowledged by the L2 first: a
    // workgroup barrier does not wait for them, and thread 0's release only
    // waits for its own wave's, so a store still in flight could land in the
    // L2 after the write-back and stay invisible to the other XCDs
    __builtin_amdgcn_s_waitcnt(0x0F70);   // s_waitcnt vmcnt(0) (gfx9 encoding)
    __syncthreads();
    if (threadIdx.x == 0) {
        *flag_lds = 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&bar[1 + blockIdx.x], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (blockIdx.x == 0) {
        __syncthreads();
        bool ok = true;
        for (int t = threadIdx.x; t < nblk; t += blockDim.x)
            if (!one_wait(&bar[1 + t], target)) ok = false;
        if (!ok) *flag_lds = 0;
        __syncthreads();
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            __hip_atomic_store(&bar[0], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else if (threadIdx.x == 0) {
        if (!one_wait(&bar[0], target)) *flag_lds = 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return *flag_lds != 0;
}

}  // namespace
}  // namespace axipcg
