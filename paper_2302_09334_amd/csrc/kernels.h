// kernels.h -- launches of the world-step phases over one or many worlds.
//
// A launch covers a batch of worlds: `pre` holds, for each kernel kind, the
// prefix of blocks per world (n + 1 entries each), and `w` the device
// addresses of the worlds' descriptors.  A block finds its world by binary
// search over the prefix, so worlds of any size mix in one launch and every
// agent is processed by exactly the same code as when its world runs alone.
#pragma once

#include <hip/hip_runtime.h>

#include "net.h"
#include "phases.h"

namespace eco {

enum : int { kPreAct = 0, kPreMove = 1, kPreClaim = 2, kPreKinds = 3 };
#ifndef ECO_NEWBORN_BLOCKS
#define ECO_NEWBORN_BLOCKS 512
#endif
constexpr int kNewbornBlocks = ECO_NEWBORN_BLOCKS;  // leading act blocks that create children (idle ones exit at once)

#ifndef ECO_PROJ_PER
#define ECO_PROJ_PER 2   // live-list positions per recurrent-projection wave of the move phase
#endif
constexpr int kProjPer = ECO_PROJ_PER;
#ifndef ECO_PROJ_PER_CLAIM
#define ECO_PROJ_PER_CLAIM 1   // ... and of the claim phase
#endif
constexpr int kProjPerClaim = ECO_PROJ_PER_CLAIM;
#ifndef ECO_PROJ_MOVE_EIGHTHS
#define ECO_PROJ_MOVE_EIGHTHS 4   // eighths of the live list whose projection runs in the move phase
#endif
constexpr int kProjMove8 = ECO_PROJ_MOVE_EIGHTHS;

// Live-list positions [0, proj_split(n)) are projected in the move phase, the
// rest in the claim phase.
__host__ __device__ constexpr int proj_split(int n) { return n * kProjMove8 / 8; }
// Recurrent-projection waves of a GRU world with `cap` slots in the move and
// in the claim phase (n - proj_split(n) grows with n, so cap bounds both).
__host__ __device__ constexpr int proj_waves_move(int cap) { return (proj_split(cap) + kProjPer - 1) / kProjPer; }
__host__ __device__ constexpr int proj_waves(int cap) { return (cap - proj_split(cap) + kProjPerClaim - 1) / kProjPerClaim; }

// Newborn blocks of a world with `cap` slots (a world never has more children
// per step than slots).
__host__ __device__ constexpr int newborn_blocks(int cap) { return cap < kNewbornBlocks ? cap : kNewbornBlocks; }

struct Batch {
    const WorldDev* const* w;   // n descriptors
    const int* pre;             // kPreKinds x (n + 1) block prefixes
    int n;
    int act_rows;               // act-kernel tuning: input rows per round trip (8, 16, 32)
    const WorldDev* w0;         // n == 1: the descriptor itself (else null)
    int cap0;                   // n == 1: its agent capacity
    int ctrl;                   // controller of every world in the batch
    int dyn;                    // dynamics of every world in the batch
    int net_wide;               // host only: the network act kernel for five waves per SIMD
    int act_waves;              // host only: agents (waves) per block of the GRU act kernel (2, 4, 8)
    int tile;                   // host only: regrowth tile edge (8, 16, 32)
    int may_stream;             // host only: the GRU act kernel holding the streaming copy of the rows
};

// Live-genome bytes of a world above which its act phase streams the input
// rows (non-temporal loads): the last-level cache (Infinity Cache, 256 MiB).
// Measured at 4608 agents (genomes 233 MiB) plain loads are faster (30.9
// against 32.7 us per step: rows kept from earlier steps hit), at 15k agents
// streaming is (77.1 against 83.4 us per step).
#ifndef ECO_ROWS_STREAM_MIB
#define ECO_ROWS_STREAM_MIB 256
#endif
constexpr size_t kRowsStreamBytes = size_t(ECO_ROWS_STREAM_MIB) << 20;

// The streaming copy exists only in the act kernels compiled with
// STREAMABLE (launched for worlds whose genomes can exceed the cache), and
// there only for the wide (hd 32) agents of the act blocks: it costs code
// size, and the act kernel's code is close to the size of the instruction
// cache.  Children acting in their first step (a few per step) and hd 16
// worlds (whose genomes stay below the cache up to about 11k agents) load as
// usual.
template <int ROWS, bool STREAMABLE>
__device__ __forceinline__ void act_dispatch(DevRef d, AgentRec* rec, int4 rv, int li, int64_t t, int lane,
                                             bool stream) {
    if (d.hd == 32) {
        if (STREAMABLE && stream) act_agent<32, ROWS, STREAMABLE>(d, rec, rv, li, t, lane);
        else act_agent<32, ROWS, false>(d, rec, rv, li, t, lane);
    } else {
        act_agent<16, ROWS, false>(d, rec, rv, li, t, lane);
    }
}

// A block's world and its index among that world's blocks of one phase.  The
// launch tables and descriptors are written by the host only, so they are
// read through the scalar cache; the scalars and the per-position records
// sit at fixed offsets from the descriptor.
struct BlockWorld {
    kptr<WorldDev> d;
    WorldScal* S;
    PosRec* P;
    int lb;
    int cap;
};

__device__ __forceinline__ int find_world(kptr<int> pre, int n, int b) {
    int lo = 0, hi = n;   // largest i with pre[i] <= b
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ BlockWorld block_world(const Batch& bt, int kind, int vb) {
    const WorldDev* p = bt.w0;
    int lb = vb;
    int cap = bt.cap0;
    pin_s(cap);
    if (p == nullptr) {
        const kptr<int> pre = kconst(bt.pre) + kind * (bt.n + 1);
        const int wi = find_world(pre, bt.n, vb);
        p = kconst(bt.w)[wi];
        lb = vb - pre[wi];
        cap = kconst(p)->cap;
    }
    char* base = (char*)p;
    return {kconst(p), reinterpret_cast<WorldScal*>(base + kScalOff), reinterpret_cast<PosRec*>(base + kPosOff), lb,
            cap};
}

// The first controller step of a child with the paper's network.  Kept out
// of line: inlined a second time into the newborn path, the network raised
// the whole act kernel to 128 registers with 22 spilled (the compiler sizes
// the kernel for its worst path); out of line the kernel needs 120 and
// spills none, and the call's own cost falls on the rare newborn blocks.
// One instance per kernel (WIDE): an instance shared by the kernels for four
// and five waves per SIMD is allocated for the tighter budget of the two.
template <bool PAPER, bool WIDE>
__device__ __attribute__((noinline)) void net_child_act(DevRef d, AgentRec* recp, int4 rv, int4 rv2, int li,
                                                        int64_t t, int lane, net::WaveLds& L) {
    net::act_agent<PAPER>(d, recp, rv, rv2, li, t, lane, L);
}

// Block bodies.  `vb` is the block's index in the batch-wide numbering of its
// phase.

// Act blocks of a world: nb = newborn_blocks(cap) leading blocks create the
// children of the previous step (rank r, r + nb, ...) and run their first
// controller step (they are the last n_child entries of the live list); the
// remaining blocks run the controller of the other agents, NT / 64 per block.
// NET: the paper's network (with `lds`, one scratch per wave), else the GRU;
// WIDE: the kernel is compiled for five waves per SIMD.
template <int ROWS, bool NET, bool PAPER = false, bool WIDE = false, int NT = kBlock, bool STREAMABLE = false>
__device__ __forceinline__ void act_body(const Batch& bt, int vb, int tid, StepShared& sh, net::WaveLds* lds) {
    const BlockWorld bw = block_world(bt, kPreAct, vb);
    DevRef d = *bw.d;
    PosRec* P = bw.P;
    const int lb = bw.lb;
    // the agent's record words in both lists, read together with the
    // scalars (index clamped; the newborn blocks read theirs later)
    const int nb = newborn_blocks(bw.cap);
    const int li = (lb - nb) * (NT / 64) + (tid >> 6);
    const int lc = min(max(li, 0), bw.cap - 1);
    const int4 q0 = *reinterpret_cast<const int4*>(&P[lc].r[0]);
    const int4 q1 = *reinterpret_cast<const int4*>(&P[lc].r[1]);
    int4 q0b = make_int4(0, 0, 0, 0), q1b = make_int4(0, 0, 0, 0);
    if constexpr (NET) {   // the second half: previous action and ate bit
        q0b = *(reinterpret_cast<const int4*>(&P[lc].r[0]) + 1);
        q1b = *(reinterpret_cast<const int4*>(&P[lc].r[1]) + 1);
    }
    const StepScal ss = read_step(bw.S);
    pin(q0.x);
    pin(q1.x);
    if constexpr (NET) {
        pin(q0b.z);
        pin(q1b.z);
    }
    if (ss.err) return;   // the world failed: it no longer steps
    const int64_t t = ss.t;
    const int n = ss.n;
    const int nc = ss.nc;
    const int sel = ss.sel;
    // the same choice for every wave of the world in this step
    const bool stream = STREAMABLE && size_t(n) * size_t(d.Ppad) * sizeof(float) > kRowsStreamBytes;
    if (lb < nb) {
        if (lb == 0) {
            if (tid == 0) step_open(d, t);
            if (t % kMoveWin == 0 && tid <= kMoveBins)   // a movement window starts: clear its record
                d.mhist[((t / kMoveWin) % kMoveRing) * (kMoveBins + 1) + tid] = 0;
            close_counters_in_step<NT>(d, tid, sh);
        }
        for (int rk = lb; rk < nc; rk += nb) {
            spawn_child<NT>(d, rk, tid, NET ? net::kState : d.hd);
            __syncthreads();
            if constexpr (!NET) {
                spawn_proj<NT>(d, rk, tid);
                __syncthreads();
            }
            if (tid < 64) {
                const int lj = n - nc + rk;
                const int4 rv = *reinterpret_cast<const int4*>(&P[lj].r[sel]);
                if constexpr (NET) {
                    const int4 rv2 = *(reinterpret_cast<const int4*>(&P[lj].r[sel]) + 1);
                    net_child_act<PAPER, WIDE>(d, &P[lj].r[sel], rv, rv2, lj, t, tid, lds[0]);
                } else {
                    act_dispatch<ROWS, false>(d, &P[lj].r[sel], rv, lj, t, tid, false);
                }
            }
            __syncthreads();
        }
        return;
    }
    if (li >= n - nc) return;
    if constexpr (NET)
        net::act_agent<PAPER>(d, &P[li].r[sel], sel ? q1 : q0, sel ? q1b : q0b, li, t, tid & 63, lds[tid >> 6]);
    else act_dispatch<ROWS, STREAMABLE>(d, &P[li].r[sel], sel ? q1 : q0, li, t, tid & 63, stream);
}

// Move blocks of a world (one wave each): the move tiles, in look-back
// order, then (GRU worlds) proj_waves_move(cap) blocks computing the
// recurrent projection of live-list positions [0, proj_split(n)) (see
// claim_body; a dying agent is projected too, harmlessly: a child taking
// over its slot is projected when the next act phase creates it).  The first
// tile also records the step and its live count for the claim phase, whose
// regrowth and projection blocks must not read the scalars the last claim
// tile rewrites.
__device__ __forceinline__ void move_body(const Batch& bt, int vb, int lane) {
    const BlockWorld bw = block_world(bt, kPreMove, vb);
    DevRef d = *bw.d;
    PosRec* P = bw.P;
    const int lb = bw.lb;
    const int ntile = (bw.cap + kTileN - 1) / kTileN;
    if (kProjMove8 > 0 && lb >= ntile) {   // recurrent projections of positions [0, proj_split(n))
        const StepScal ss = read_step(bw.S);
        if (ss.err) return;
        const int nw = proj_waves_move(bw.cap);
        for (int li = lb - ntile; li < proj_split(ss.n); li += nw) {
            const int slot = P[li].r[ss.sel].slot;
            if (d.hd == 32) proj_agent<32>(d, slot, lane);
            else proj_agent<16>(d, slot, lane);
        }
        return;
    }
    const int ci = min(lb * kTileN + lane, bw.cap - 1);
    const AgentRec r0 = P[ci].r[0];
    const AgentRec r1 = P[ci].r[1];
    const StepScal ss = read_step(bw.S);
    pin(r0.slot);
    pin(r1.slot);
    if (ss.err) return;
    if (lb == 0 && lane == 0) {
        bw.S->t_grow = ss.t;
        bw.S->n_grow = ss.n;
    }
    move_block(d, P, lb, lane, ss, r0, r1);
}

// Claim blocks of a world (one wave each): the claim tiles (look-back
// order), the regrowth tiles, then (GRU worlds) proj_waves(cap) blocks that
// compute, position by position of the step's live list from proj_split(n)
// on, the recurrent projection W_hh h + b_hh of the hidden state its act phase
// wrote, for the next act phase.  Only survivors of the move phase are
// projected here: no kernel of this phase writes a hidden state or genome,
// and a child taking over a dead agent's slot is projected when the next act
// phase creates it.
//
// The projection (about half of a step's bytes) streams while the move and
// claim tiles, which are latency-bound, wait on their round trips; every tile
// load then queues behind the projection's loads, so it is split between the
// two phases.  Measured at 4608 agents, two positions per wave: half of the
// list in each phase 31.4 us per step, three eighths in the move phase 31.9
// (all of it here: 34.4 before the claim tiles skipped their gathers in steps
// without a free slot).  Here one position per wave: the chain of a wave that
// projects two agents in turn outlasts the claim tiles (31.6 -> 31.25 us per
// step; three per wave 32.2), while the move phase keeps two (one there was
// slower).
template <bool PAPER, int TILE>
__device__ __forceinline__ void claim_body(const Batch& bt, int vb, int lane, uint8_t* tile) {
    const BlockWorld bw = block_world(bt, kPreClaim, vb);
    DevRef d = *bw.d;
    const int lb = bw.lb;
    const int ntile = (bw.cap + kTileN - 1) / kTileN;
    if (lb < ntile) {
        const PostRec p = bw.P[min(lb * kTileN + lane, bw.cap - 1)].post;
        const StepScal ss = read_step(bw.S);
        pin(p.slot);
        if (ss.err) return;
        claim_block<PAPER>(d, bw.S, bw.P, lb, lane, ss, p);
        return;
    }
    const int ngrow = ((d.H + TILE - 1) / TILE) * ((d.W + TILE - 1) / TILE);
    if (lb < ntile + ngrow) {
        regrow_tile<TILE>(d, lb - ntile, lane, tile, kconst(bw.S)->t_grow, ngrow);
        return;
    }
    const int nw = proj_waves(bw.cap);
    const int n = kconst(bw.S)->n_grow;
    for (int li = proj_split(n) + lb - ntile - ngrow; li < n; li += nw) {
        const int4 q = *reinterpret_cast<const int4*>(&bw.P[li].post);   // slot, ..., alive
        if (!q.w) continue;
        if (d.hd == 32) proj_agent<32>(d, q.x, lane);
        else proj_agent<16>(d, q.x, lane);
    }
}

// Act kernels of GRU worlds: ROWS input rows per wave per round trip, WAVES
// agents (one wave each) per block.  Both are tuning knobs that change no
// result: an agent's summation order depends on its observation only, and
// the block-wide work (child genomes, window totals, counter sums) is
// elementwise or integer.
template <int ROWS, int WAVES, bool STREAMABLE>
__global__ __launch_bounds__(64 * WAVES) void k_act_gru(Batch bt) {
    __shared__ StepShared sh;
    act_body<ROWS, false, false, false, 64 * WAVES, STREAMABLE>(bt, blockIdx.x, threadIdx.x, sh, nullptr);
}

// Act kernels of worlds with the paper's network.  The compiler's own
// register choice (about 185, two waves per SIMD) leaves the load round trip
// of each wave exposed; four waves measured about 20% faster.  Four waves per
// SIMD hold 16 waves per CU, one agent each: a launch with more agents runs
// the rest as a second round, so such launches use the kernels compiled for
// five waves (96 registers, none spilled; 29.7 against 31.5 us per step with
// 4608 agents), while smaller ones keep four (five cost 0.1 to 0.3 us per step
// with 1000 agents).  A spill of a register that holds a load of the first
// round trip waits for that load and splits the round trip: six waves spill
// and are slower.
#ifndef ECO_NET_WAVES_WIDE
#define ECO_NET_WAVES_WIDE 5
#endif
#ifndef ECO_NET_WAVES
#define ECO_NET_WAVES 4   // waves per SIMD the network act kernel is compiled for (0 = compiler's choice)
#endif
#if ECO_NET_WAVES > 0
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(ECO_NET_WAVES, ECO_NET_WAVES)))
#else
__global__ __launch_bounds__(kBlock)
#endif
void k_act_net(Batch bt) {
    __shared__ StepShared sh;
    __shared__ net::WaveLds lds[kBlock / 64];
    act_body<16, true, false>(bt, blockIdx.x, threadIdx.x, sh, lds);
}

// The same for worlds with the paper's dynamics.
#if ECO_NET_WAVES > 0
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(ECO_NET_WAVES, ECO_NET_WAVES)))
#else
__global__ __launch_bounds__(kBlock)
#endif
void k_act_net_paper(Batch bt) {
    __shared__ StepShared sh;
    __shared__ net::WaveLds lds[kBlock / 64];
    act_body<16, true, true>(bt, blockIdx.x, threadIdx.x, sh, lds);
}

// The same two kernels for launches with more agents than four waves per
// SIMD hold.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(ECO_NET_WAVES_WIDE, ECO_NET_WAVES_WIDE)))
void k_act_net_wide(Batch bt) {
    __shared__ StepShared sh;
    __shared__ net::WaveLds lds[kBlock / 64];
    act_body<16, true, false, true>(bt, blockIdx.x, threadIdx.x, sh, lds);
}

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(ECO_NET_WAVES_WIDE, ECO_NET_WAVES_WIDE)))
void k_act_net_paper_wide(Batch bt) {
    __shared__ StepShared sh;
    __shared__ net::WaveLds lds[kBlock / 64];
    act_body<16, true, true, true>(bt, blockIdx.x, threadIdx.x, sh, lds);
}

// Creates the pending children of a world's last step now (before its state
// is read by the host); k_clear_pending then marks them as created, so the
// next act phase treats them as ordinary agents.
__global__ __launch_bounds__(kBlock) void k_materialize(const WorldDev* dp) {
    DevRef d = *kconst(dp);
    if (d.scal->err) return;
    const int nc = d.scal->n_child;
    for (int rk = blockIdx.x; rk < nc; rk += gridDim.x) {
        spawn_child<kBlock>(d, rk, threadIdx.x, d.ss);
        __syncthreads();
        if (d.ctrl == kCtrlGru) {
            spawn_proj<kBlock>(d, rk, threadIdx.x);
            __syncthreads();
        }
    }
}

// Recurrent projections of every live agent of a world (after creation or a
// load, when no claim phase has produced them).
__global__ __launch_bounds__(kBlock) void k_proj_all(const WorldDev* dp) {
    DevRef d = *kconst(dp);
    const WorldScal* S = d.scal;
    const int li = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (li >= S->n_live) return;
    const int slot = d.live[S->live_sel][li];
    if (d.hd == 32) proj_agent<32>(d, slot, threadIdx.x & 63);
    else proj_agent<16>(d, slot, threadIdx.x & 63);
}

// Window sums of the input weights of every live agent of a world (after
// creation or a load), one block per agent.
__global__ __launch_bounds__(kBlock) void k_rsum_all(const WorldDev* dp) {
    DevRef d = *kconst(dp);
    const WorldScal* S = d.scal;
    if (int(blockIdx.x) >= S->n_live) return;
    rsum_agent(d, d.live[S->live_sel][blockIdx.x], threadIdx.x, kBlock);
}

__global__ void k_clear_pending(const WorldDev* dp) {
    if (threadIdx.x == 0) dp->scal->n_child = 0;
}

// Sums the eaten / resource partials of a world's last step if still open.
__global__ __launch_bounds__(kBlock) void k_close_counters(const WorldDev* dp) {
    __shared__ StepShared sh;
    close_counters_in_step<kBlock>(*kconst(dp), threadIdx.x, sh);
}

__global__ __launch_bounds__(64) void k_move(Batch bt) { move_body(bt, blockIdx.x, threadIdx.x); }

// Claim kernels, one per regrowth tile edge TILE (a tuning knob).
template <int TILE>
__global__ __launch_bounds__(64) void k_claim(Batch bt) {
    __shared__ uint8_t tile[(TILE + 4) * (TILE + 4)];
    claim_body<false, TILE>(bt, blockIdx.x, threadIdx.x, tile);
}

// The claim phase of worlds with the paper's dynamics (births on the parent's
// cell, no neighbour scan).
template <int TILE>
__global__ __launch_bounds__(64) void k_claim_paper(Batch bt) {
    __shared__ uint8_t tile[(TILE + 4) * (TILE + 4)];
    claim_body<true, TILE>(bt, blockIdx.x, threadIdx.x, tile);
}

// Spread of the initial weights: parameter p takes sd[k] for the first k with
// p < end[k] (0 for biases).
struct InitSegs {
    int n;
    int end[12];
    float sd[12];
};

// Initial genomes: agent slots [0, n_init) hold uids 0..n_init-1; parameter p
// of uid u is std(p) * z_p with z_p lane p % 4 of INIT_W draw (u, 0, p / 4).
__global__ __launch_bounds__(kBlock) void k_init_theta(const WorldDev* dp, int n_init, InitSegs segs) {
    DevRef d = *kconst(dp);
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
            bool found = false;
            for (int k = 0; k < segs.n; ++k)
                if (!found && p < segs.end[k]) {
                    sd = segs.sd[k];
                    found = true;
                }
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

__global__ void k_test_gumbel(const uint32_t* w, size_t n, float* g) {
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    g[i] = gumbel_of_word(w[i]);
}

__global__ void k_test_gauss(const uint32_t* a, const uint32_t* b, size_t n, float* z0, float* z1) {
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    box_muller(a[i], b[i], z0[i], z1[i]);
}

}  // namespace eco
