// phases.h -- device code of one world step (gfx950, wave64).
//
// A step is three phases separated by device-wide ordering points (kernel
// boundaries or grid barriers):
//   P1 act     observe + GRU controller + arg-max, one wave per agent; the
//              children born in the previous step are first created (genome =
//              parent + sigma * N(0, 1), record, occB) by leading blocks,
//              which then run their first controller step
//   P2 move    move resolution, eating, energy, age, death, streak; a
//              decoupled look-back scan over the live list (uid order)
//              compacts the survivors and ranks the dead
//   P3 claim   birth claims and their resolution, ranked by a second
//              look-back scan (born = rank < cap - survivors, so every
//              winner knows its child slot at once); regrowth tiles; the
//              last claim block to finish closes the step's bookkeeping
// Every decision is a gather: an agent reads its neighbours' state and
// decides on its own; cross-block communication is limited to the look-back
// status words and one completion counter per world.
//
// Paper mapping: observation and controller App. B.2/B.5, moves and energy
// App. B.2, reproduction/mutation/death App. B.3, regrowth App. B.1 Eq. (1).
#pragma once

#include <hip/hip_runtime.h>

#include "rng.h"
#include "world_dev.h"

namespace eco {

// occB word of a live agent after P2: slot | eligible << 30 | birth dir << 28.
constexpr int kOccElig = 1 << 30;
constexpr int kOccDirShift = 28;
constexpr int kOccSlotMask = (1 << 28) - 1;

// Action deltas: 0 = N (row - 1), 1 = S (row + 1), 2 = E (col + 1),
// 3 = W (col - 1), 4 = stay.
__device__ __forceinline__ int act_dr(int a) { return a == 0 ? -1 : (a == 1 ? 1 : 0); }
__device__ __forceinline__ int act_dc(int a) { return a == 2 ? 1 : (a == 3 ? -1 : 0); }

__device__ __forceinline__ uint64_t claim_key(uint32_t draw_word, uint32_t u) {
    return (uint64_t(draw_word) << 32) | u;
}

__device__ __forceinline__ float sigmoidf_(float v) { return 1.0f / (1.0f + expf(-v)); }

// ---------------------------------------------------------------------------
// P1: observation + GRU + head + arg-max for the agent in `slot` (one wave).
//
// Lane layout: G = 64 / HD groups of HD lanes; lane (g, k) owns hidden unit k
// of group g.  Each input row of W_ih holds the 3 gate weights of every
// hidden unit contiguously (3 * HD floats), so a group reads one row with one
// 12-byte load per lane.  Inputs are binary except the energy, so the input
// projection is a sum of the rows whose input is 1: the set bits of two wave
// ballots are dealt round-robin to the groups, each group sums its rows in
// increasing input order, and the group partials are combined by a fixed xor
// tree.  The summation order therefore depends only on the agent's own
// observation, never on the launch shape or on other worlds in the launch.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Recurrent projection gh = W_hh h + b_hh of the agent in `slot` (one wave),
// written to gh[slot] (3 * HD floats, gate-interleaved per hidden unit).  It
// depends only on the hidden state left by the last act phase, so it is
// computed ahead of the next act phase, off its critical path.  Group g sums
// the recurrent rows j = jj * G + g in increasing jj, then the groups combine
// by a fixed xor tree: the order depends on nothing but the agent.
// ---------------------------------------------------------------------------
template <int HD>
__device__ __forceinline__ void proj_agent(const WorldDev& d, int slot, int lane) {
    constexpr int G = 64 / HD;
    constexpr int RW = 3 * HD;
    constexpr int JJ = HD / G;
    const int g = lane / HD;
    const int k = lane - g * HD;
    const float* th = d.theta + size_t(slot) * size_t(d.Ppad);
    const float hk = d.h[size_t(slot) * HD + k];
    float whr[JJ], whz[JJ], whn[JJ];
#pragma unroll
    for (int jj = 0; jj < JJ; ++jj) {
        const float* p = th + d.off_hh + (jj * G + g) * RW + 3 * k;
        whr[jj] = p[0];
        whz[jj] = p[1];
        whn[jj] = p[2];
    }
    const float* pbh = th + d.off_bhh + 3 * k;
    const float bhr = pbh[0], bhz = pbh[1], bhn = pbh[2];
    float hr = 0.f, hz = 0.f, hn = 0.f;
#pragma unroll
    for (int jj = 0; jj < JJ; ++jj) {
        const float hj = __shfl(hk, jj * G + g);
        hr = fmaf(hj, whr[jj], hr);
        hz = fmaf(hj, whz[jj], hz);
        hn = fmaf(hj, whn[jj], hn);
    }
#pragma unroll
    for (int off = HD; off < 64; off <<= 1) {
        hr += __shfl_xor(hr, off);
        hz += __shfl_xor(hz, off);
        hn += __shfl_xor(hn, off);
    }
    if (g == 0) {
        float* o = d.gh + size_t(slot) * RW + 3 * k;
        o[0] = hr + bhr;
        o[1] = hz + bhz;
        o[2] = hn + bhn;
    }
}

// A zero hidden state (new agents) projects to b_hh.
template <int HD>
__device__ __forceinline__ void proj_zero(const WorldDev& d, int slot, int lane) {
    constexpr int RW = 3 * HD;
    if (lane < HD) {
        const float* pbh = d.theta + size_t(slot) * size_t(d.Ppad) + d.off_bhh + 3 * lane;
        float* o = d.gh + size_t(slot) * RW + 3 * lane;
        // 0 * W_hh summed from +0 is +0, and +0 + b = b: the same bits as the
        // full projection of a zero hidden state.
        o[0] = 0.f + pbh[0];
        o[1] = 0.f + pbh[1];
        o[2] = 0.f + pbh[2];
    }
}

// ---------------------------------------------------------------------------
// P1: observation + GRU + head + arg-max for the agent in `slot` (one wave).
//
// Lane layout: G = 64 / HD groups of HD lanes; lane (g, k) owns hidden unit k
// of group g.  Each input row of W_ih holds the 3 gate weights of every
// hidden unit contiguously (3 * HD floats), so a group reads one row with one
// 12-byte load per lane.  Inputs are binary except the energy, so the input
// projection is a sum of the rows whose input is 1: the set bits of two wave
// ballots are dealt round-robin to the groups, each group sums its rows in
// increasing input order, and the group partials are combined by a fixed xor
// tree.  The summation order therefore depends only on the agent's own
// observation, never on the launch shape or on other worlds in the launch:
// ROWS (input rows fetched per wave per round trip) only changes how many
// loads are in flight, since row q of the enumeration always goes to group
// q % G and each group adds its rows in increasing q.
// The recurrent projection comes precomputed from gh[slot].
// ---------------------------------------------------------------------------
template <int HD, int ROWS>
__device__ __forceinline__ void act_agent(const WorldDev& d, AgentRec* recp, int li, int64_t t, int lane) {
    constexpr int G = 64 / HD;
    constexpr int RW = 3 * HD;   // floats per input row
    constexpr int B = ROWS / G;  // input rows per group per round trip
    const int g = lane / HD;
    const int k = lane - g * HD;
    const int H = d.H, W = d.W;
    const int4 rv = *reinterpret_cast<const int4*>(recp);   // slot, cell, energy, uid
    const int slot = rv.x;
    const int cell = rv.y;
    const int r = cell / W;
    const int c = cell - r * W;
    const int e = rv.z;
    const uint32_t u = uint32_t(rv.w);
    const float* th = d.theta + size_t(slot) * size_t(d.Ppad);
    const int rho = d.rho;
    const int win = 2 * rho + 1;
    const int w2 = win * win;
    const int erow = 2 * w2;   // energy input row

    // Round trip 1: everything that does not depend on the observation (the
    // hidden state, the recurrent projection, the input biases, the energy
    // row, the head) together with the observation window itself.
    const float hk = d.h[size_t(slot) * HD + k];
    const float* pg = d.gh + size_t(slot) * RW + 3 * k;
    const float ghr = pg[0], ghz = pg[1], ghn = pg[2];
    const float* pe = th + erow * RW + 3 * k;
    const float* pbi = th + d.off_bih + 3 * k;
    const float er = pe[0], ez = pe[1], en = pe[2];
    const float bir = pbi[0], biz = pbi[1], bin = pbi[2];
    float wo[5], bo[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        wo[a] = th[d.off_wo + a * HD + k];
        bo[a] = th[d.off_bo + a];
    }
    const uint8_t* R = d.R[t & 1];
    bool rb = false, ob = false;
    if (lane < w2) {
        const int dy = lane / win - rho;
        const int dx = lane - (lane / win) * win - rho;
        const int rr = r + dy, cc = c + dx;
        if (rr >= 0 && rr < H && cc >= 0 && cc < W) {
            const int q = rr * W + cc;
            rb = R[q] != 0;
            ob = d.occA[q] != -1;
        } else {
            ob = true;   // outside the grid reads as occupied, no resource
        }
    }
    uint64_t mR = __ballot(rb);
    uint64_t mO = __ballot(ob);
    const uint64_t occ_bits = mO;

    // Round trip 2 (usually the last): every input row whose input is 1.
    float ar = 0.f, az = 0.f, an = 0.f;
    while (mR | mO) {
        int rows[G * B];
#pragma unroll
        for (int q = 0; q < G * B; ++q) {
            int row = -1;
            if (mR) {
                row = __builtin_ctzll(mR);
                mR &= mR - 1;
            } else if (mO) {
                row = w2 + __builtin_ctzll(mO);
                mO &= mO - 1;
            }
            rows[q] = row;
        }
        float vr[B], vz[B], vn[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            int row = rows[b * G];
#pragma unroll
            for (int gg = 1; gg < G; ++gg)
                if (g == gg) row = rows[b * G + gg];
            const bool ok = row >= 0;
            const float* p = th + (ok ? row : erow) * RW + 3 * k;
            const float x0 = p[0], x1 = p[1], x2 = p[2];
            vr[b] = ok ? x0 : 0.f;
            vz[b] = ok ? x1 : 0.f;
            vn[b] = ok ? x2 : 0.f;
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            ar += vr[b];
            az += vz[b];
            an += vn[b];
        }
    }
#pragma unroll
    for (int off = HD; off < 64; off <<= 1) {
        ar += __shfl_xor(ar, off);
        az += __shfl_xor(az, off);
        an += __shfl_xor(an, off);
    }

    const float xe = float(e) / float(d.E0);
    const float gir = fmaf(xe, er, ar) + bir;
    const float giz = fmaf(xe, ez, az) + biz;
    const float gin = fmaf(xe, en, an) + bin;
    const float rg = sigmoidf_(gir + ghr);
    const float zg = sigmoidf_(giz + ghz);
    const float ng = tanhf(fmaf(rg, ghn, gin));
    const float hnew = fmaf(zg, hk - ng, ng);

    float lg[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        float v = hnew * wo[a];
#pragma unroll
        for (int off = HD / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
        lg[a] = v + bo[a];
    }
    int best = 0;
#pragma unroll
    for (int a = 1; a < 5; ++a)
        if (lg[a] > lg[best]) best = a;
    if (d.forced >= 0) best = d.forced;

    if (g == 0) d.h[size_t(slot) * HD + k] = hnew;
    if (lane == 0) {
        d.action[slot] = uint8_t(best);
        recp->action = best;
        // Move claim (resolved by the next phase): a move targets the window
        // cell one step away, which must be inside the grid and empty at the
        // step start (its occupancy bit, outside cells reading occupied, is 0).
        // The smallest (MOVE draw, uid) among a cell's claimants wins; an
        // atomic minimum is independent of the order of the claims.
        if (best < 4) {
            const int q = (rho + act_dr(best)) * win + (rho + act_dc(best));
            if (!((occ_bits >> q) & 1ull)) {
                const uint64_t key = claim_key(philox(u, uint32_t(t), kMove, 0, d.seed_lo, d.seed_hi).x, u);
                const int Y = (r + act_dr(best)) * W + (c + act_dc(best));
                atomicMin(reinterpret_cast<unsigned long long*>(d.mclaim + Y), (unsigned long long)key);
            }
        }
    }
    if (d.log_steps > 0) {
        const size_t row = size_t(t % d.log_steps) * size_t(d.cap) + size_t(li);
        if (lane == 0) {
            d.log_uid[row] = u;
            d.log_act[row] = uint8_t(best);
        }
        if (lane < 5) {
            float v = lg[0];
#pragma unroll
            for (int a = 1; a < 5; ++a)
                if (lane == a) v = lg[a];
            d.log_logits[row * 5 + lane] = v;
        }
    }
}

// Step-start bookkeeping done once per world per step by one thread.
__device__ __forceinline__ void step_open(const WorldDev& d, int64_t t) {
    if (d.log_steps > 0) d.log_n[t % d.log_steps] = d.scal->n_live;
}

// ---------------------------------------------------------------------------
// Decoupled look-back prefix sum over the tiles of one phase (tile = one
// block of kBlock live-list entries).  A status word packs
//   [epoch 20 | flag 2 | a 21 | b 21]   flag 1 = tile total, 2 = inclusive
// where epoch = step mod 2^20, so words from earlier steps are ignored and the
// arrays never need clearing between steps.  Returns the exclusive prefix of
// the packed (a, b) pair; waits are bounded (2 s) and a time-out sets the
// world's error word.
// ---------------------------------------------------------------------------
constexpr int kCntBits = 21;
constexpr uint64_t kCntMask = (uint64_t(1) << kCntBits) - 1;
constexpr uint64_t kValMask = (uint64_t(1) << (2 * kCntBits)) - 1;

__device__ __forceinline__ uint64_t pack2(uint32_t a, uint32_t b) { return (uint64_t(a) << kCntBits) | b; }
__device__ __forceinline__ uint32_t unpack_a(uint64_t v) { return uint32_t((v >> kCntBits) & kCntMask); }
__device__ __forceinline__ uint32_t unpack_b(uint64_t v) { return uint32_t(v & kCntMask); }

__device__ __forceinline__ uint64_t lookback(const WorldDev& d, uint64_t* st, int tile, uint32_t epoch,
                                             uint64_t local, int tid, uint64_t* s_bcast) {
    // Wave 0 publishes this tile's total, then examines the predecessors 64 at
    // a time (one status word per lane) until the nearest one holding an
    // inclusive prefix: the prefix is that word plus the totals in between.
    if (tid < 64) {
        const int lane = tid;
        const uint64_t tag = uint64_t(epoch & 0xFFFFFu);
        if (lane == 0)
            __hip_atomic_store(st + tile, (tag << 44) | (uint64_t(tile == 0 ? 2 : 1) << 42) | local,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint64_t excl = 0;
        int end = tile;
        const uint64_t t0 = wall_clock64();
        bool timed_out = false;
        while (end > 0) {
            const int k = end - 1 - lane;   // lane 0 = nearest predecessor
            uint64_t v = 0;
            uint32_t flag = 2;              // lanes past tile 0 act as an empty inclusive
            if (k >= 0) {
                while (true) {
                    v = __hip_atomic_load(st + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    flag = uint32_t(v >> 42) & 3u;
                    if ((v >> 44) == tag && flag != 0) break;
                    if (wall_clock64() - t0 > 200000000ull) {   // 2 s at the 100 MHz wall clock
                        timed_out = true;
                        v = 0;
                        flag = 2;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            const uint64_t val = (k >= 0) ? (v & kValMask) : 0;
            const uint64_t incl = __ballot(flag == 2);
            const int first = incl ? __builtin_ctzll(incl) : 64;   // nearest inclusive lane
            uint64_t part = (lane <= first) ? val : 0;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
            excl += part;
            if (incl) break;
            end -= 64;
        }
        if (__ballot(timed_out) && lane == 0)
            __hip_atomic_store(&d.scal->err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (lane == 0) {
            if (tile != 0)
                __hip_atomic_store(st + tile, (tag << 44) | (uint64_t(2) << 42) | (excl + local), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            *s_bcast = excl;
        }
    }
    __syncthreads();
    const uint64_t r = *s_bcast;
    __syncthreads();
    return r;
}

// Inclusive total of the last tile of a completed look-back.
__device__ __forceinline__ uint64_t lookback_total(const uint64_t* st, int ntile) {
    return __hip_atomic_load(st + ntile - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kValMask;
}

// Block-local exclusive ranks of two predicates and the block totals.
struct BlockRank {
    int ra, rb;   // this thread's exclusive rank among the block's a / b
    int ta, tb;   // block totals
};

__device__ __forceinline__ BlockRank block_rank2(bool a, bool b, int tid, int* sw) {
    const int lane = tid & 63, wv = tid >> 6;
    constexpr int NW = kBlock / 64;
    const uint64_t ma = __ballot(a), mb = __ballot(b);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (lane == 0) {
        sw[wv] = __popcll(ma);
        sw[NW + wv] = __popcll(mb);
    }
    __syncthreads();
    BlockRank r;
    r.ra = __popcll(ma & lt);
    r.rb = __popcll(mb & lt);
    r.ta = r.tb = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        if (w < wv) {
            r.ra += sw[w];
            r.rb += sw[NW + w];
        }
        r.ta += sw[w];
        r.tb += sw[NW + w];
    }
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// P2: moves (one thread per live agent).  A move was claimed in P1 only into
// an in-grid cell empty at the step start, and the cell's claim word holds
// the smallest (MOVE draw, uid) of its claimants: the agent moves iff that is
// its own key.  Then: eat the
// resource of the final cell, energy += gain * ate - decay, age += 1, death
// at energy <= 0 or age >= L_max, streak of survivors.  occB receives the
// moves and deaths; occA (read by every agent in this phase) is untouched.
// Returns bit 0 = ate, bit 1 = died.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int move_agent(const WorldDev& d, const AgentRec& a, int64_t t, PostRec* post,
                                          AgentRec* next_rec_src) {
    const int W = d.W, H = d.H;
    const int slot = a.slot;
    const int X = a.cell;
    const int act = a.action;
    const uint32_t u = a.uid;
    const int r = X / W, c = X - (X / W) * W;
    uint8_t* Rc = d.R[t & 1];
    // the claim word of the target and both possible resource bytes together
    int Y = -1;
    if (act < 4) {
        const int tr = r + act_dr(act), tc = c + act_dc(act);
        if (tr >= 0 && tr < H && tc >= 0 && tc < W) Y = tr * W + tc;
    }
    const uint64_t cw = (Y >= 0) ? d.mclaim[Y] : ~0ull;
    const int rX = Rc[X];
    const int rY = (Y >= 0) ? Rc[Y] : 0;
    int newX = X;
    if (Y >= 0) {
        const uint64_t key = claim_key(philox(u, uint32_t(t), kMove, 0, d.seed_lo, d.seed_hi).x, u);
        if (cw == key) newX = Y;
    }
    const int ate = (newX == X ? rX : rY) != 0;
    if (ate) Rc[newX] = 0;
    const int en = a.energy - d.decay + d.gain * ate;
    const int ag = a.age + 1;
    const bool dead = en <= 0 || ag >= d.L_max;
    int st = a.streak;
    if (!dead) st = (en >= d.E_repr) ? st + 1 : 0;
    d.energy[slot] = en;
    d.age[slot] = ag;
    d.streak[slot] = st;
    d.cell[slot] = newX;
    d.prev_cell[slot] = X;
    d.alive[slot] = dead ? 0 : 1;
    // Both occupancy grids take the moves and deaths (neither is read in this
    // phase): occA is the next step's start state, occB is read by P3.  A
    // survivor's occB word also says whether it is eligible to reproduce and
    // from which direction its birth scan starts; its birth key is stored per
    // slot, so P3 learns a neighbour's claim from occupancy reads alone.
    int word = -1;
    if (!dead) {
        word = slot;
        if (st >= d.T_repr) {
            const Draw4 b = philox(u, uint32_t(t), kBirth, 0, d.seed_lo, d.seed_hi);
            word |= kOccElig | int((b.x & 3u) << kOccDirShift);
            d.bkey[slot] = claim_key(b.y, u);
        }
    }
    if (newX != X) {
        d.occA[X] = -1;
        d.occB[X] = -1;
        if (!dead) d.occA[newX] = slot;
    } else if (dead) {
        d.occA[X] = -1;
    }
    d.occB[newX] = word;
    PostRec p;
    p.slot = slot;
    p.prev_cell = X;
    p.cell = newX;
    p.alive = dead ? 0 : 1;
    p.streak = st;
    p.action = act;
    p.uid = u;
    p.next_pos = -1;
    *post = p;
    AgentRec nr;
    nr.slot = slot;
    nr.cell = newX;
    nr.energy = en;
    nr.uid = u;
    nr.age = ag;
    nr.streak = st;
    nr.action = 4;
    nr.pad = 0;
    *next_rec_src = nr;
    return ate | (dead ? 2 : 0);
}

struct StepShared {
    uint8_t tile[(kTile + 4) * (kTile + 4)];
    int sw[2 * (kBlock / 64)];
    uint64_t bcast;
    int flag;
};

// P2 for tile `j` (kBlock live-list entries) of one world.  Survivors keep
// their uid order in the next live list; dead slots are listed in uid order.
__device__ __forceinline__ void move_block(const WorldDev& d, int j, int tid, StepShared& sh) {
    const WorldScal* S = d.scal;
    const int n = S->n_live;
    const int sel = S->live_sel;
    const int64_t t = S->t;
    const int i = j * kBlock + tid;
    int res = 0;
    AgentRec nr;
    nr.slot = -1;
    if (i < n) res = move_agent(d, d.rec[sel][i], t, d.post + i, &nr);
    const bool alive = i < n && !(res & 2);
    const bool dead = i < n && (res & 2);
    const int cnt = __popcll(__ballot((res & 1) != 0));
    if ((tid & 63) == 0) d.eat_part[i >> 6] = cnt;
    const BlockRank br = block_rank2(alive, dead, tid, sh.sw);
    const uint64_t ex = lookback(d, d.lb_move, j, uint32_t(t), pack2(br.ta, br.tb), tid, &sh.bcast);
    if (alive) {
        const int pos = int(unpack_a(ex)) + br.ra;
        d.live[sel ^ 1][pos] = nr.slot;
        d.rec[sel ^ 1][pos] = nr;
        d.post[i].next_pos = pos;
    }
    if (dead) d.deadlist[unpack_b(ex) + br.rb] = nr.slot;
}

// First free in-grid 4-neighbour of `cell` (order N, S, E, W cyclically from
// `d0`) in the post-move, post-death occupancy; -1 if none.  The four
// occupancy words are loaded together.
__device__ __forceinline__ int birth_target(const WorldDev& d, int cell, int d0) {
    const int W = d.W, H = d.H;
    const int r = cell / W, c = cell - (cell / W) * W;
    int nb[4];
    bool freec[4];
#pragma unroll
    for (int dd = 0; dd < 4; ++dd) {
        const int nr = r + act_dr(dd), nc = c + act_dc(dd);
        const bool in = nr >= 0 && nr < H && nc >= 0 && nc < W;
        nb[dd] = nr * W + nc;
        freec[dd] = in && d.occB[in ? nb[dd] : cell] == -1;
    }
    int C = -1;
#pragma unroll
    for (int k = 3; k >= 0; --k) {
        const int dd = (d0 + k) & 3;
        if (freec[dd]) C = nb[dd];
    }
    return C;
}

// ---------------------------------------------------------------------------
// P3a: clear this agent's move-claim word, then, for an eligible survivor,
// compute its birth claim and resolve it against the other eligible agents
// next to the claimed cell: their occB words give eligibility and scan start,
// their claims are recomputed from occB, their keys come from bkey.
// Returns the claimed cell of a claim winner, -1 otherwise.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int claim_agent(const WorldDev& d, const PostRec& p, int64_t t) {
    const int X = p.prev_cell;
    const int X2 = p.cell;
    const bool alive = p.alive != 0;
    {
        // clear the move-claim word this agent may have written in P1
        const int a = p.action;
        if (a < 4) {
            const int tr = X / d.W + act_dr(a), tc = X - (X / d.W) * d.W + act_dc(a);
            if (tr >= 0 && tr < d.H && tc >= 0 && tc < d.W) d.mclaim[tr * d.W + tc] = ~0ull;
        }
    }
    int C = -1;
    bool won = false;
    if (alive && p.streak >= d.T_repr) {
        const uint32_t u = p.uid;
        const Draw4 b = philox(u, uint32_t(t), kBirth, 0, d.seed_lo, d.seed_hi);
        C = birth_target(d, X2, int(b.x & 3u));
        if (C >= 0) {
            const uint64_t key = claim_key(b.y, u);
            won = true;
            const int W = d.W, H = d.H;
            const int cr = C / W, cc = C - (C / W) * W;
            int M[4], v[4];
#pragma unroll
            for (int dd = 0; dd < 4; ++dd) {
                const int mr = cr + act_dr(dd), mc = cc + act_dc(dd);
                const bool in = mr >= 0 && mr < H && mc >= 0 && mc < W;
                M[dd] = mr * W + mc;
                v[dd] = (in && M[dd] != X2) ? d.occB[M[dd]] : -1;
            }
#pragma unroll
            for (int dd = 0; dd < 4; ++dd) {
                if (v[dd] < 0 || !(v[dd] & kOccElig)) continue;
                const int o = v[dd] & kOccSlotMask;
                const uint64_t ko = d.bkey[o];
                if (birth_target(d, M[dd], (v[dd] >> kOccDirShift) & 3) != C) continue;
                if (ko < key) won = false;
            }
        }
    }
    d.claim[p.slot] = C;
    return won ? C : -1;
}

// P3a for tile `j` of one world.  The winner of global rank r (uid order) is
// born iff r < cap - survivors; its child takes free slot r of the ring if the
// ring holds more than r slots, else the (r - free)-th slot freed this step.
// The last claim tile to finish closes the step (counts, free ring, scalars).
__device__ __forceinline__ void claim_block(const WorldDev& d, int j, int tid, StepShared& sh) {
    WorldScal* S = d.scal;
    const int n = S->n_live;
    const int sel = S->live_sel;
    const int64_t t = S->t;
    const int cap = d.cap;
    const int ntile = (cap + kBlock - 1) / kBlock;
    const int i = j * kBlock + tid;
    int slot = -1, cell = -1, pos = -1;
    bool win = false;
    if (i < n) {
        const PostRec p = d.post[i];
        slot = p.slot;
        pos = p.next_pos;
        cell = claim_agent(d, p, t);
        win = cell >= 0;
    }
    const BlockRank br = block_rank2(win, false, tid, sh.sw);
    const uint64_t ex = lookback(d, d.lb_claim, j, uint32_t(t), pack2(br.ta, 0), tid, &sh.bcast);
    const int surv = int(unpack_a(lookback_total(d.lb_move, ntile)));
    const int nfree = cap - n;
    if (win) {
        const int rk = int(unpack_a(ex)) + br.ra;
        if (rk < cap - surv) {
            int cs;
            if (rk < nfree) {
                int q = S->free_head + rk;
                if (q >= cap) q -= cap;
                cs = d.freeq[q];
            } else {
                cs = d.deadlist[rk - nfree];
            }
            const uint32_t cu = S->next_uid + uint32_t(rk);
            d.child[rk] = make_int4(cs, slot, cell, int(cu));
            d.live[sel ^ 1][surv + rk] = cs;
            AgentRec cr;
            cr.slot = cs;
            cr.cell = cell;
            cr.energy = d.E0;
            cr.uid = cu;
            cr.age = 0;
            cr.streak = 0;
            cr.action = 4;
            cr.pad = 0;
            d.rec[sel ^ 1][surv + rk] = cr;
            d.occA[cell] = cs;   // occA is neither read nor written by others in this phase
            // the parent's streak restarts (no phase reads these in P3)
            d.rec[sel ^ 1][pos].streak = 0;
            d.streak[slot] = 0;
        }
    }
    // completion: the last tile to get here closes the step
    __syncthreads();
    if (tid == 0) {
        // Relaxed: the closing block reads only look-back words (atomics) and
        // data of earlier phases; the counter orders its writes of the
        // scalars after every tile's reads of them.
        const uint32_t prev = __hip_atomic_fetch_add(d.done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sh.flag = (prev == uint32_t(ntile - 1)) ? 1 : 0;
    }
    __syncthreads();
    if (!sh.flag) return;
    const int wins = int(unpack_a(lookback_total(d.lb_claim, ntile)));
    const int dead = n - surv;
    const int nb = min(wins, cap - surv);
    const int consumed = max(0, nb - nfree);
    const int ft = S->free_tail;
    for (int q = consumed + tid; q < dead; q += kBlock) {
        int pos = ft + q - consumed;
        if (pos >= cap) pos -= cap;
        d.freeq[pos] = d.deadlist[q];
    }
    __syncthreads();
    if (tid == 0) {
        __hip_atomic_store(d.done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int nfh = S->free_head + min(nb, nfree);
        if (nfh >= cap) nfh -= cap;
        int nft = ft + (dead - consumed);
        if (nft >= cap) nft -= cap;
        int32_t* rec = d.ring + (t % kRing) * kCtrWords;
        rec[kCtrLive] = surv + nb;
        rec[kCtrBirths] = nb;
        rec[kCtrDeaths] = dead;
        rec[kCtrWins] = wins;
        S->n_prev = n;
        S->free_head = nfh;
        S->free_tail = nft;
        S->n_live = surv + nb;
        S->next_uid = S->next_uid + uint32_t(nb);
        S->live_sel = sel ^ 1;
        S->n_child = nb;
        S->spawn_t = t;
        S->ctr_open = 1;
        S->t = t + 1;
    }
}

// ---------------------------------------------------------------------------
// P3b: regrowth of one kTile x kTile tile (one block).  The tile plus a
// 2-cell halo of the post-eating grid is staged in LDS; an empty cell counts
// the resources among its 24 neighbours and grows iff its REGROW draw is
// below thr[row][count].  Writes the other grid buffer (synchronous update)
// and the tile's resource count.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void regrow_tile(const WorldDev& d, int tile, int tid, StepShared& sh) {
    constexpr int E = kTile + 4;
    const int64_t t = d.scal->t;
    uint8_t* s = sh.tile;
    const int ntx = (d.W + kTile - 1) / kTile;
    const int ty0 = (tile / ntx) * kTile;
    const int tx0 = (tile - (tile / ntx) * ntx) * kTile;
    const uint8_t* Rc = d.R[t & 1];
    uint8_t* Rn = d.R[(t + 1) & 1];
    for (int idx = tid; idx < E * E; idx += kBlock) {
        const int ly = idx / E, lx = idx - (idx / E) * E;
        const int gy = ty0 + ly - 2, gx = tx0 + lx - 2;
        s[idx] = (gy >= 0 && gy < d.H && gx >= 0 && gx < d.W) ? Rc[gy * d.W + gx] : uint8_t(0);
    }
    __syncthreads();
    const int ly = tid / kTile, lx = tid - (tid / kTile) * kTile;
    const int gy = ty0 + ly, gx = tx0 + lx;
    int v = 0;
    if (gy < d.H && gx < d.W) {
        const int q = gy * d.W + gx;
        v = s[(ly + 2) * E + lx + 2];
        if (!v) {
            int cnt = 0;
#pragma unroll
            for (int dy = 0; dy < 5; ++dy)
#pragma unroll
                for (int dx = 0; dx < 5; ++dx) cnt += s[(ly + dy) * E + lx + dx];
            const Draw4 dr = philox(uint32_t(q), uint32_t(t), kRegrow, 0, d.seed_lo, d.seed_hi);
            v = uint64_t(dr.x) < d.thr[gy * 25 + cnt] ? 1 : 0;
        }
        Rn[q] = uint8_t(v);
    }
    const BlockRank br = block_rank2(v != 0, false, tid, sh.sw);
    if (tid == 0) d.res_part[tile] = br.ta;
}

// ---------------------------------------------------------------------------
// Child creation (start of P1, one block per child): the genome is
// theta_child[p] = fmaf(sigma, z_p, theta_parent[p]) with z_p lane p % 4 of
// the MUTATE draw (child uid, birth step, block p / 4); the record gets
// energy E0, age 0, streak 0 and a zero hidden state; the child enters occB
// (occA received it when it was born; the parent's streak restarted then).
// Every store is complete when this returns, so the same block can run the
// child's controller right after a block barrier.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void spawn_child(const WorldDev& d, int rk, int tid) {
    const int4 rec = d.child[rk];   // child slot, parent slot, cell, uid
    const uint32_t ts = uint32_t(d.scal->spawn_t);
    const float* par = d.theta + size_t(rec.y) * size_t(d.Ppad);
    float* out = d.theta + size_t(rec.x) * size_t(d.Ppad);
    for (int blk = tid; blk < d.nblk; blk += kBlock) {
        const int p0 = 4 * blk;
        const float4 pv = *reinterpret_cast<const float4*>(par + p0);
        const Draw4 dr = philox(uint32_t(rec.w), ts, kMutate, uint32_t(blk), d.seed_lo, d.seed_hi);
        float z0, z1, z2, z3;
        box_muller(dr.x, dr.y, z0, z1);
        box_muller(dr.z, dr.w, z2, z3);
        float4 o;
        o.x = fmaf(d.sigma, z0, pv.x);
        o.y = p0 + 1 < d.P ? fmaf(d.sigma, z1, pv.y) : 0.f;
        o.z = p0 + 2 < d.P ? fmaf(d.sigma, z2, pv.z) : 0.f;
        o.w = p0 + 3 < d.P ? fmaf(d.sigma, z3, pv.w) : 0.f;
        *reinterpret_cast<float4*>(out + p0) = o;
    }
    const int cs = rec.x;
    if (tid == 0) {
        d.uid[cs] = uint32_t(rec.w);
        d.cell[cs] = rec.z;
        d.prev_cell[cs] = rec.z;
        d.energy[cs] = d.E0;
        d.age[cs] = 0;
        d.streak[cs] = 0;
        d.alive[cs] = 1;
        d.claim[cs] = -1;
        d.action[cs] = 4;
        d.occB[rec.z] = cs;
    }
    if (tid < d.hd) d.h[size_t(cs) * d.hd + tid] = 0.f;
    __builtin_amdgcn_s_waitcnt(0);   // this thread's stores have completed
}

// Recurrent projection of a new agent (after spawn_child and a barrier).
__device__ __forceinline__ void spawn_proj(const WorldDev& d, int rk, int tid) {
    if (tid < 64) {
        const int cs = d.child[rk].x;
        if (d.hd == 32) proj_zero<32>(d, cs, tid);
        else proj_zero<16>(d, cs, tid);
    }
    __builtin_amdgcn_s_waitcnt(0);
}

// Eaten and resource totals of the step just closed (one block per world).
__device__ __forceinline__ void close_counters(const WorldDev& d, int tid, StepShared& sh) {
    WorldScal* S = d.scal;
    if (!S->ctr_open) return;
    const int nwv = (S->n_prev + 63) / 64;
    int pe = 0, pr = 0;
    for (int i = tid; i < nwv; i += kBlock) pe += d.eat_part[i];
    for (int i = tid; i < d.ntiles; i += kBlock) pr += d.res_part[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        pe += __shfl_xor(pe, off);
        pr += __shfl_xor(pr, off);
    }
    if ((tid & 63) == 0) {
        sh.sw[tid >> 6] = pe;
        sh.sw[(kBlock / 64) + (tid >> 6)] = pr;
    }
    __syncthreads();
    if (tid == 0) {
        int te = 0, tr = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            te += sh.sw[w];
            tr += sh.sw[(kBlock / 64) + w];
        }
        int32_t* rec = d.ring + (S->spawn_t % kRing) * kCtrWords;
        rec[kCtrEaten] = te;
        rec[kCtrRes] = tr;
    }
    __syncthreads();
}

// P1 bookkeeping by the first block of a world: sum the eaten / resource
// partials of the previous step (written by its P2 and P3).
__device__ __forceinline__ void close_counters_in_step(const WorldDev& d, int tid, StepShared& sh) {
    close_counters(d, tid, sh);
    if (tid == 0) d.scal->ctr_open = 0;
}

}  // namespace eco
