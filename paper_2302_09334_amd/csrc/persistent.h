// persistent.h -- one cooperative launch that runs K world steps for a batch
// of worlds, with grid-wide barriers between the phases instead of kernel
// boundaries.  All blocks are co-resident (cooperative launch), every wait is
// bounded by a wall-clock limit, and a timed-out barrier sets the first
// world's error word and makes every block leave the kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace eco {

struct PersistArgs {
    Batch bt;                   // descriptors + block prefixes (as the per-phase kernels)
    int K;
    uint32_t* barrier;          // arrival counter, zeroed before the launch
    int32_t* err;               // device error word (first world's scalars)
    uint64_t spin_ticks;        // wall-clock ticks a barrier may wait
};

__global__ void k_zero_barrier(uint32_t* bar) {
    if (threadIdx.x == 0) bar[0] = 0;
}

// Returns false when the barrier timed out (or an earlier one did).  The
// block's writes are ordered before thread 0's release by the workgroup
// barrier; thread 0 spins on relaxed loads (an acquire per poll would
// invalidate the L2 each time) and performs one acquire fence at the end,
// which makes the other blocks' writes visible to the whole block.
__device__ __forceinline__ bool grid_sync(const PersistArgs& a, uint32_t& target, int* s_ok) {
    __builtin_amdgcn_s_waitcnt(0);   // this thread's stores have reached the L2
    __syncthreads();
    target += gridDim.x;
    if (threadIdx.x == 0) {
        int ok = 1;
        __hip_atomic_fetch_add(a.barrier, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(a.barrier, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            if (wall_clock64() - t0 > a.spin_ticks) {
                __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
        }
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

__global__ __launch_bounds__(kBlock) void k_persistent(PersistArgs a) {
    __shared__ StepShared sh;
    __shared__ int s_ok;
    const Batch& bt = a.bt;
    const int np = bt.n + 1;
    const int n_act = bt.pre[kPreAct * np + bt.n];
    const int n_move = bt.pre[kPreMove * np + bt.n];
    const int n_claim = bt.pre[kPreClaim * np + bt.n];
    const int tid = threadIdx.x;
    uint32_t target = 0;
    for (int s = 0; s < a.K; ++s) {
        for (int vb = blockIdx.x; vb < n_act; vb += gridDim.x) act_body<16>(bt, vb, tid, sh);
        if (!grid_sync(a, target, &s_ok)) return;
        for (int vb = blockIdx.x; vb < n_move; vb += gridDim.x) move_body(bt, vb, tid, sh);
        if (!grid_sync(a, target, &s_ok)) return;
        for (int vb = blockIdx.x; vb < n_claim; vb += gridDim.x) claim_body(bt, vb, tid, sh);
        if (!grid_sync(a, target, &s_ok)) return;
    }
}

}  // namespace eco
