// kernels.h -- launches of the world-step phases over one or many worlds.
//
// A launch covers a batch of worlds: `pre` holds, for each kernel kind, the
// prefix of blocks per world (n + 1 entries each), and `w` the device
// addresses of the worlds' descriptors.  A block finds its world by binary
// search over the prefix, so worlds of any size mix in one launch and every
// agent is processed by exactly the same code as when its world runs alone.
#pragma once

#include <hip/hip_runtime.h>

#include "phases.h"

namespace eco {

enum : int { kPreAct = 0, kPreMove = 1, kPreClaim = 2, kPreKinds = 3 };
constexpr int kNewbornBlocks = 64;   // leading act blocks that create children

struct Batch {
    const WorldDev* const* w;   // n descriptors
    const int* pre;             // kPreKinds x (n + 1) block prefixes
    int n;
    int act_rows;               // act-kernel tuning: input rows per round trip (8, 16, 32)
};

template <int ROWS>
__device__ __forceinline__ void act_dispatch(const WorldDev& d, AgentRec* rec, int li, int64_t t, int lane) {
    if (d.hd == 32) act_agent<32, ROWS>(d, rec, li, t, lane);
    else act_agent<16, ROWS>(d, rec, li, t, lane);
}

__device__ __forceinline__ int find_world(const int* pre, int n, int b) {
    int lo = 0, hi = n;   // largest i with pre[i] <= b
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Block bodies, shared by the per-phase kernels and the persistent kernel.
// `vb` is the block's index in the batch-wide numbering of its phase.

// Act blocks of a world: kNewbornBlocks leading blocks create the children of
// the previous step (rank r, r + kNewbornBlocks, ...) and run their first
// controller step (they are the last n_child entries of the live list); the
// remaining blocks run the controller of the other agents, four per block.
template <int ROWS>
__device__ __forceinline__ void act_body(const Batch& bt, int vb, int tid, StepShared& sh) {
    const int* pre = bt.pre + kPreAct * (bt.n + 1);
    const int wi = find_world(pre, bt.n, vb);
    const WorldDev& d = *bt.w[wi];
    const int lb = vb - pre[wi];
    const WorldScal* S = d.scal;
    const int64_t t = S->t;
    const int n = S->n_live;
    const int nc = S->n_child;
    const int sel = S->live_sel;
    if (lb < kNewbornBlocks) {
        if (lb == 0) {
            if (tid == 0) step_open(d, t);
            close_counters_in_step(d, tid, sh);
        }
        for (int rk = lb; rk < nc; rk += kNewbornBlocks) {
            spawn_child(d, rk, tid);
            __syncthreads();
            spawn_proj(d, rk, tid);
            __syncthreads();
            if (tid < 64) {
                const int li = n - nc + rk;
                act_dispatch<ROWS>(d, d.rec[sel] + li, li, t, tid);
            }
            __syncthreads();
        }
        return;
    }
    const int li = (lb - kNewbornBlocks) * (kBlock / 64) + (tid >> 6);
    if (li >= n - nc) return;
    act_dispatch<ROWS>(d, d.rec[sel] + li, li, t, tid & 63);
}

__device__ __forceinline__ void move_body(const Batch& bt, int vb, int tid, StepShared& sh) {
    const int* pre = bt.pre + kPreMove * (bt.n + 1);
    const int wi = find_world(pre, bt.n, vb);
    move_block(*bt.w[wi], vb - pre[wi], tid, sh);
}

// Claim blocks of a world: the claim tiles (look-back order), the regrowth
// tiles, then one wave per survivor computing the recurrent projection for
// the next act phase (the survivors are the first entries of the next live
// list, whose count the move look-back has fixed).
__device__ __forceinline__ void claim_body(const Batch& bt, int vb, int tid, StepShared& sh) {
    const int* pre = bt.pre + kPreClaim * (bt.n + 1);
    const int wi = find_world(pre, bt.n, vb);
    const WorldDev& d = *bt.w[wi];
    const int lb = vb - pre[wi];
    const int ntile = (d.cap + kBlock - 1) / kBlock;
    if (lb < ntile) {
        claim_block(d, lb, tid, sh);
        return;
    }
    if (lb < ntile + d.ntiles) {
        regrow_tile(d, lb - ntile, tid, sh);
        return;
    }
    const int li = (lb - ntile - d.ntiles) * (kBlock / 64) + (tid >> 6);
    const int surv = int(unpack_a(lookback_total(d.lb_move, ntile)));
    if (li >= surv) return;
    const int slot = d.live[d.scal->live_sel ^ 1][li];
    if (d.hd == 32) proj_agent<32>(d, slot, tid & 63);
    else proj_agent<16>(d, slot, tid & 63);
}

#ifndef ECO_ACT_WAVES
#define ECO_ACT_WAVES 0   // waves per SIMD the act kernel is compiled for (0 = compiler's choice)
#endif
#if ECO_ACT_WAVES > 0
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(ECO_ACT_WAVES, ECO_ACT_WAVES)))
#else
__global__ __launch_bounds__(kBlock)
#endif
void k_act(Batch bt) {
    __shared__ StepShared sh;
    act_body<16>(bt, blockIdx.x, threadIdx.x, sh);
}

// Tuning variants of the act kernel (identical results, different numbers of
// loads in flight per wave).
template <int ROWS>
__global__ __launch_bounds__(kBlock) void k_act_rows(Batch bt) {
    __shared__ StepShared sh;
    act_body<ROWS>(bt, blockIdx.x, threadIdx.x, sh);
}

// Creates the pending children of a world's last step now (before its state
// is read by the host); k_clear_pending then marks them as created, so the
// next act phase treats them as ordinary agents.
__global__ __launch_bounds__(kBlock) void k_materialize(const WorldDev* dp) {
    const WorldDev& d = *dp;
    const int nc = d.scal->n_child;
    for (int rk = blockIdx.x; rk < nc; rk += gridDim.x) {
        spawn_child(d, rk, threadIdx.x);
        __syncthreads();
        spawn_proj(d, rk, threadIdx.x);
        __syncthreads();
    }
}

// Recurrent projections of every live agent of a world (after creation or a
// load, when no move phase has produced them).
__global__ __launch_bounds__(kBlock) void k_proj_all(const WorldDev* dp) {
    const WorldDev& d = *dp;
    const WorldScal* S = d.scal;
    const int li = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (li >= S->n_live) return;
    const int slot = d.live[S->live_sel][li];
    if (d.hd == 32) proj_agent<32>(d, slot, threadIdx.x & 63);
    else proj_agent<16>(d, slot, threadIdx.x & 63);
}

__global__ void k_clear_pending(const WorldDev* dp) {
    if (threadIdx.x == 0) dp->scal->n_child = 0;
}

// Sums the eaten / resource partials of a world's last step if still open.
__global__ __launch_bounds__(kBlock) void k_close_counters(const WorldDev* dp) {
    __shared__ StepShared sh;
    close_counters_in_step(*dp, threadIdx.x, sh);
}

__global__ __launch_bounds__(kBlock) void k_move(Batch bt) {
    __shared__ StepShared sh;
    move_body(bt, blockIdx.x, threadIdx.x, sh);
}

__global__ __launch_bounds__(kBlock) void k_claim(Batch bt) {
    __shared__ StepShared sh;
    claim_body(bt, blockIdx.x, threadIdx.x, sh);
}

// Initial genomes: agent slots [0, n_init) hold uids 0..n_init-1; parameter p
// of uid u is std(p) * z_p with z_p lane p % 4 of INIT_W draw (u, 0, p / 4).
__global__ __launch_bounds__(kBlock) void k_init_theta(const WorldDev* dp, int n_init, float std_ih,
                                                       float std_hd) {
    const WorldDev& d = *dp;
    const int64_t total = int64_t(n_init) * d.nblk;
    for (int64_t it = int64_t(blockIdx.x) * kBlock + threadIdx.x; it < total;
         it += int64_t(gridDim.x) * kBlock) {
        const int a = int(it / d.nblk);
        const int blk = int(it - int64_t(a) * d.nblk);
        const Draw4 dr = philox(uint32_t(a), 0u, kInitW, uint32_t(blk), d.seed_lo, d.seed_hi);
        float z[4];
        box_muller(dr.x, dr.y, z[0], z[1]);
        box_muller(dr.z, dr.w, z[2], z[3]);
        float o[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int p = 4 * blk + j;
            float sd = 0.f;
            if (p < d.off_hh) sd = std_ih;
            else if (p < d.off_bih) sd = std_hd;
            else if (p < d.off_wo) sd = 0.f;
            else if (p < d.off_bo) sd = std_hd;
            o[j] = (p < d.P && sd != 0.f) ? sd * z[j] : 0.f;
        }
        *reinterpret_cast<float4*>(d.theta + size_t(a) * size_t(d.Ppad) + 4 * blk) =
            make_float4(o[0], o[1], o[2], o[3]);
    }
}

__global__ __launch_bounds__(kBlock) void k_copy16(const int4* __restrict__ src, int4* __restrict__ dst, size_t n) {
    for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += size_t(gridDim.x) * kBlock) dst[i] = src[i];
}

__global__ void k_test_philox(const uint32_t* ctr, size_t n, uint32_t k0, uint32_t k1, uint32_t* out) {
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Draw4 r = philox(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
    out[4 * i] = r.x;
    out[4 * i + 1] = r.y;
    out[4 * i + 2] = r.z;
    out[4 * i + 3] = r.w;
}

__global__ void k_test_gauss(const uint32_t* a, const uint32_t* b, size_t n, float* z0, float* z1) {
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    box_muller(a[i], b[i], z0[i], z1[i]);
}

}  // namespace eco
