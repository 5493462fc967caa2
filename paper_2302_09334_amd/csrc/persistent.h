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
    const WorldDev* const* w;   // n descriptors
    const int* pre;             // 3 x (n + 1) item prefixes: act waves, agent threads (x64), tiles
    int n;
    int K;
    uint32_t* barrier;          // arrival counter, zeroed before the launch
    int32_t* err;               // device error word (first world's scalars)
    uint64_t spin_ticks;        // wall-clock ticks a barrier may wait
    int max_useful_blocks;      // host-side cap on the grid
};

__global__ void k_zero_barrier(uint32_t* bar) {
    if (threadIdx.x == 0) bar[0] = 0;
}

// Returns false when the barrier timed out (or an earlier one did).
__device__ __forceinline__ bool grid_sync(const PersistArgs& a, uint32_t& target, int* s_ok) {
    __threadfence();
    __syncthreads();
    target += gridDim.x;
    if (threadIdx.x == 0) {
        int ok = 1;
        __hip_atomic_fetch_add(a.barrier, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(a.barrier, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
            if (wall_clock64() - t0 > a.spin_ticks) {
                __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
        }
        *s_ok = ok;
    }
    __syncthreads();
    __threadfence();
    return *s_ok != 0;
}

__global__ __launch_bounds__(kBlock) void k_persistent(PersistArgs a) {
    __shared__ uint8_t tile[(kTile + 4) * (kTile + 4)];
    __shared__ int sm[3 * (kBlock / 64)];
    __shared__ int s_ok;
    const int n = a.n;
    const int* pa = a.pre;                 // waves (cap per world)
    const int* pg = a.pre + (n + 1);       // threads (cap rounded up to 64 per world)
    const int* pt = a.pre + 2 * (n + 1);   // regrowth tiles
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    constexpr int WPB = kBlock / 64;
    uint32_t target = 0;

    for (int s = 0; s < a.K; ++s) {
        // P1: act
        if (tid == 0)
            for (int wi = blockIdx.x; wi < n; wi += gridDim.x) step_open(*a.w[wi], a.w[wi]->scal->t);
        for (int gi = blockIdx.x * WPB + wave; gi < pa[n]; gi += gridDim.x * WPB) {
            const int wi = find_world(pa, n, gi);
            const WorldDev& d = *a.w[wi];
            const int li = gi - pa[wi];
            const WorldScal* S = d.scal;
            if (li < S->n_live) {
                const int slot = d.live[S->live_sel][li];
                if (d.hd == 32) act_agent<32>(d, slot, li, S->t, lane);
                else act_agent<16>(d, slot, li, S->t, lane);
            }
        }
        if (!grid_sync(a, target, &s_ok)) return;

        // P2: move
        for (int base = blockIdx.x * kBlock; base < pg[n]; base += gridDim.x * kBlock) {
            const int wbase = base + wave * 64;
            int ate = 0;
            int64_t t = 0;
            int wi = -1;
            if (wbase < pg[n]) {
                wi = find_world(pg, n, wbase);
                const WorldDev& d = *a.w[wi];
                const int i = wbase + lane - pg[wi];
                t = d.scal->t;
                if (i < d.scal->n_live) ate = move_agent(d, d.live[d.scal->live_sel][i], t);
            }
            const int cnt = __popcll(__ballot(ate != 0));
            if (lane == 0 && cnt && wi >= 0)
                atomicAdd(a.w[wi]->ring + (t % kRing) * kCtrWords + kCtrEaten, cnt);
        }
        if (!grid_sync(a, target, &s_ok)) return;

        // P3: birth claims, then regrowth tiles
        for (int base = blockIdx.x * kBlock; base < pg[n]; base += gridDim.x * kBlock) {
            const int wbase = base + wave * 64;
            if (wbase < pg[n]) {
                const int wi = find_world(pg, n, wbase);
                const WorldDev& d = *a.w[wi];
                const int i = wbase + lane - pg[wi];
                if (i < d.scal->n_live) claim_agent(d, d.live[d.scal->live_sel][i], d.scal->t);
            }
        }
        for (int ti = blockIdx.x; ti < pt[n]; ti += gridDim.x) {
            const int wi = find_world(pt, n, ti);
            const WorldDev& d = *a.w[wi];
            const int64_t t = d.scal->t;
            const int cnt = regrow_tile(d, ti - pt[wi], t, tid, tile);
            if (lane == 0 && cnt) atomicAdd(d.ring + (t % kRing) * kCtrWords + kCtrRes, cnt);
        }
        if (!grid_sync(a, target, &s_ok)) return;

        // P4: per-world scan
        for (int wi = blockIdx.x; wi < n; wi += gridDim.x) scan_world(*a.w[wi], tid, sm);
        if (!grid_sync(a, target, &s_ok)) return;

        // P5: children; items of consecutive worlds continue the block
        // rotation so small per-world counts still spread over the grid.
        {
            int acc = 0;
            const int G = gridDim.x;
            for (int wi = 0; wi < n; ++wi) {
                const WorldDev& d = *a.w[wi];
                const int nchunks = (d.nblk + kBlock - 1) / kBlock;
                const int items = d.scal->n_child * nchunks;
                int first = (int(blockIdx.x) - acc) % G;
                if (first < 0) first += G;
                for (int it = first; it < items; it += G) spawn_item(d, it, nchunks, tid);
                acc = (acc + items) % G;
            }
        }
        if (!grid_sync(a, target, &s_ok)) return;
    }
}

}  // namespace eco
