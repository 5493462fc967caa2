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

enum : int { kPreAct = 0, kPreAgent = 1, kPreTile = 2, kPreSpawn = 3, kPreKinds = 4 };
constexpr int kSpawnBlocksPerWorld = 32;

struct Batch {
    const WorldDev* const* w;   // n descriptors
    const int* pre;             // kPreKinds x (n + 1) block prefixes
    int n;
};

__device__ __forceinline__ int find_world(const int* pre, int n, int b) {
    int lo = 0, hi = n;   // largest i with pre[i] <= b
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_act(Batch bt) {
    const int* pre = bt.pre + kPreAct * (bt.n + 1);
    const int wi = find_world(pre, bt.n, blockIdx.x);
    const WorldDev& d = *bt.w[wi];
    const int lb = blockIdx.x - pre[wi];
    const int64_t t = d.scal->t;
    const int n = d.scal->n_live;
    if (lb == 0 && threadIdx.x == 0) step_open(d, t);
    const int li = lb * (kBlock / 64) + int(threadIdx.x >> 6);
    if (li >= n) return;
    const int slot = d.live[d.scal->live_sel][li];
    const int lane = threadIdx.x & 63;
    if (d.hd == 32) act_agent<32>(d, slot, li, t, lane);
    else act_agent<16>(d, slot, li, t, lane);
}

__global__ __launch_bounds__(kBlock) void k_move(Batch bt) {
    const int* pre = bt.pre + kPreAgent * (bt.n + 1);
    const int wi = find_world(pre, bt.n, blockIdx.x);
    const WorldDev& d = *bt.w[wi];
    const int i = (blockIdx.x - pre[wi]) * kBlock + threadIdx.x;
    const int64_t t = d.scal->t;
    int ate = 0;
    if (i < d.scal->n_live) ate = move_agent(d, d.live[d.scal->live_sel][i], t);
    const int cnt = __popcll(__ballot(ate != 0));
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(d.ring + (t % kRing) * kCtrWords + kCtrEaten, cnt);
}

__global__ __launch_bounds__(kBlock) void k_claim(Batch bt) {
    const int* pre = bt.pre + kPreAgent * (bt.n + 1);
    const int wi = find_world(pre, bt.n, blockIdx.x);
    const WorldDev& d = *bt.w[wi];
    const int i = (blockIdx.x - pre[wi]) * kBlock + threadIdx.x;
    if (i < d.scal->n_live) claim_agent(d, d.live[d.scal->live_sel][i], d.scal->t);
}

__global__ __launch_bounds__(kBlock) void k_regrow(Batch bt) {
    __shared__ uint8_t s[(kTile + 4) * (kTile + 4)];
    const int* pre = bt.pre + kPreTile * (bt.n + 1);
    const int wi = find_world(pre, bt.n, blockIdx.x);
    const WorldDev& d = *bt.w[wi];
    const int64_t t = d.scal->t;
    const int cnt = regrow_tile(d, blockIdx.x - pre[wi], t, threadIdx.x, s);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(d.ring + (t % kRing) * kCtrWords + kCtrRes, cnt);
}

__global__ __launch_bounds__(kBlock) void k_scan(Batch bt) {
    __shared__ int sm[3 * (kBlock / 64)];
    scan_world(*bt.w[blockIdx.x], threadIdx.x, sm);
}

__global__ __launch_bounds__(kBlock) void k_spawn(Batch bt) {
    const int* pre = bt.pre + kPreSpawn * (bt.n + 1);
    const int wi = find_world(pre, bt.n, blockIdx.x);
    const WorldDev& d = *bt.w[wi];
    const int nchunks = (d.nblk + kBlock - 1) / kBlock;
    const int items = d.scal->n_child * nchunks;
    const int nb = pre[wi + 1] - pre[wi];
    for (int it = blockIdx.x - pre[wi]; it < items; it += nb) spawn_item(d, it, nchunks, threadIdx.x);
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
