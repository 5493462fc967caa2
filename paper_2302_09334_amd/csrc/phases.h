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
//              last claim tile closes the step's bookkeeping
// Every decision is a gather: an agent reads its neighbours' state and
// decides on its own; cross-block communication is limited to the look-back
// status words.
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

// Test hook (scripted policies): the action forced on the agent with uid
// `u` -- its entry of the by-uid table if it has one >= 0, else the world's
// default -- or the controller's choice `best` when neither forces one.
__device__ __forceinline__ int forced_of(DevRef d, uint32_t u, int best) {
    int fa = d.forced;
    if (u < uint32_t(d.n_forced)) {
        const int v = d.forced_tab[u];
        if (v >= 0) fa = v;
    }
    return fa >= 0 ? fa : best;
}

// The act phase's claim on the cell the chosen action leads to (one lane per
// agent).  Benchmark rules: a move claims its target when it lies inside the
// grid and is empty at the step start; the smallest (MOVE draw, uid) moves.
// Paper rules: the agent claims the resource of the cell it will stand on
// (its target, or its own cell when it stays) when that cell lies inside the
// grid and holds a resource at the step start; the smallest (EAT draw, uid)
// eats it.  `t_free` / `t_res`: the target's occupancy and resource as
// observed; an atomic minimum does not depend on the order of the claims.
__device__ __forceinline__ void act_claim(DevRef d, int best, int r, int c, uint32_t u, int64_t t, bool t_free,
                                          bool t_res) {
    const int tr = r + act_dr(best), tc = c + act_dc(best);
    const bool in = tr >= 0 && tr < d.H && tc >= 0 && tc < d.W;
    bool claim;
    uint32_t stream;
    if (d.dyn == kDynPaper) {
        claim = in && t_res;
        stream = kEat;
    } else {
        claim = best < 4 && in && t_free;
        stream = kMove;
    }
    if (claim) {
        const uint64_t key = claim_key(philox(u, uint32_t(t), stream, 0, d.seed_lo, d.seed_hi).x, u);
        atomicMin(reinterpret_cast<unsigned long long*>(d.mclaim + tr * d.W + tc), (unsigned long long)key);
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
__device__ __forceinline__ void proj_agent(DevRef d, int slot, int lane) {
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

// Column totals of the agent's input weights over each binary window, kept
// after its genome (theta rows tot_row and tot_row + 1, same column layout as
// the input rows): row tot_row holds the sum of the resource-window rows of
// W_ih, row tot_row + 1 the sum of the occupancy-window rows, each added in
// increasing row order.  The act phase sums a window that holds more ones
// than zeros as this total minus the rows of its zeros.
__device__ __forceinline__ void rsum_agent(DevRef d, int slot, int tid, int nthreads) {
    const int RW = 3 * d.hd;
    const int w2 = (2 * d.rho + 1) * (2 * d.rho + 1);
    float* th = d.theta + size_t(slot) * size_t(d.Ppad);
    constexpr int kMaxW2 = 49;   // window of radius 3
    for (int j = tid; j < 2 * RW; j += nthreads) {
        const int win = j / RW, c = j - win * RW;
        const float* col = th + size_t(win) * w2 * RW + c;
        float v[kMaxW2];
#pragma unroll
        for (int i = 0; i < kMaxW2; ++i) v[i] = i < w2 ? col[i * RW] : 0.f;   // all loads in flight together
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < kMaxW2; ++i)
            if (i < w2) acc += v[i];
        th[size_t(d.tot_row) * RW + j] = acc;
    }
}

// A zero hidden state (new agents) projects to b_hh.
template <int HD>
__device__ __forceinline__ void proj_zero(DevRef d, int slot, int lane) {
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
// projection is a sum of the rows whose input is 1 (or, for a window with
// more ones than zeros, the window's precomputed column total minus the rows
// of its zeros): the items are dealt round-robin to the groups, each group
// sums its items in enumeration order, and the group partials are combined by
// a fixed xor tree.  The summation order therefore depends only on the
// agent's own observation, never on the launch shape or on other worlds in
// the launch: ROWS (input rows fetched per wave per round trip) only changes
// how many loads are in flight, since item q of the enumeration always goes
// to group q % G and each group adds its items in increasing q.
// The recurrent projection comes precomputed from gh[slot].
// STREAM: the input rows are read with non-temporal loads (chosen per world
// and step by the caller when the live genomes exceed the last-level cache:
// then they cannot be held there from one step to the next, and streaming
// them leaves the cache to the data the step's later phases read again).
// ---------------------------------------------------------------------------
template <int HD, int ROWS, bool STREAM>
__device__ __forceinline__ void act_agent(DevRef d, AgentRec* recp, int4 rv, int li, int64_t t, int lane) {
    constexpr int G = 64 / HD;
    constexpr int RW = 3 * HD;   // floats per input row
    constexpr int B = ROWS / G;  // input rows per group per round trip
    const int g = lane / HD;
    const int k = lane - g * HD;
    const int H = d.H, W = d.W;
    const int slot = rv.x;   // record words: slot, cell, energy, uid
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
    const bool seen = mR != 0;   // a resource in the field of view
    const uint64_t res_bits = mR;

    // Round trips 2..: the input rows.  A window with more ones than zeros is
    // summed as its precomputed column total minus the rows of its zeros
    // (fewer rows to read); the items are dealt to the groups in the order
    // [total R], R rows, [total O], O rows, each with its sign.
    const uint64_t wmask = ~0ull >> (64 - w2);
    const bool cR = 2 * __popcll(mR) > w2;
    const bool cO = 2 * __popcll(mO) > w2;
    if (cR) mR = ~mR & wmask;
    if (cO) mO = ~mO & wmask;
    int pend = (cR ? 1 : 0) | (cO ? 2 : 0);   // window totals still to add
    const int nrows = __popcll(mR) + __popcll(mO) + (cR ? 1 : 0) + (cO ? 1 : 0);   // input rows read
    constexpr int kNeg = 1 << 16;
    const int tot_row = d.tot_row;
    float ar = 0.f, az = 0.f, an = 0.f;
    while (mR | mO | uint64_t(pend)) {
        int items[G * B];
#pragma unroll
        for (int q = 0; q < G * B; ++q) {
            int it = tot_row + 2;   // the zero row: nothing left to add
            // (every lane loads unconditionally, so the loads of a round trip
            // stay together)
            if (pend & 1) {
                it = tot_row;
                pend &= ~1;
            } else if (mR) {
                it = __builtin_ctzll(mR) | (cR ? kNeg : 0);
                mR &= mR - 1;
            } else if (pend & 2) {
                it = tot_row + 1;
                pend &= ~2;
            } else if (mO) {
                it = (w2 + __builtin_ctzll(mO)) | (cO ? kNeg : 0);
                mO &= mO - 1;
            }
            items[q] = it;
        }
        float vr[B], vz[B], vn[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            int it = items[b * G];
#pragma unroll
            for (int gg = 1; gg < G; ++gg)
                if (g == gg) it = items[b * G + gg];
            const float* p = th + (it & (kNeg - 1)) * RW + 3 * k;
            float x0, x1, x2;
            if constexpr (STREAM) {
                x0 = __builtin_nontemporal_load(p);
                x1 = __builtin_nontemporal_load(p + 1);
                x2 = __builtin_nontemporal_load(p + 2);
            } else {
                x0 = p[0];
                x1 = p[1];
                x2 = p[2];
            }
            const bool neg = (it & kNeg) != 0;
            vr[b] = neg ? -x0 : x0;
            vz[b] = neg ? -x1 : x1;
            vn[b] = neg ? -x2 : x2;
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
    if (d.forced_on) best = forced_of(d, u, best);

    if (g == 0) d.h[size_t(slot) * HD + k] = hnew;
    if (lane == 0 && t % kMoveWin == 0) {   // a movement window starts with this step
        d.wcell[slot] = cell;
        d.wuid[slot] = u;
    }
    if (lane == 0) {
        d.action[slot] = uint8_t(best);
        recp->action = best | (seen ? kSeenBit : 0) | (nrows << kRowsShift);
        // the claim on the target cell (resolved by the next phase); the
        // target's window bits (outside cells read occupied, no resource)
        const int q = (rho + act_dr(best)) * win + (rho + act_dc(best));
        act_claim(d, best, r, c, u, t, !((occ_bits >> q) & 1ull), ((res_bits >> q) & 1ull) != 0);
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
__device__ __forceinline__ void step_open(DevRef d, int64_t t) {
    if (d.log_steps > 0) d.log_n[t % d.log_steps] = d.scal->n_live;
}

// ---------------------------------------------------------------------------
// Decoupled look-back prefix sum over the tiles of one phase (tile = one wave
// of kTileN live-list entries, one block).  A status word packs
//   [epoch 20 | flag 2 | a 21 | b 21]   flag 1 = tile total, 2 = inclusive
// where epoch = step mod 2^20, so words from earlier steps are ignored and the
// arrays never need clearing between steps.  Every lane returns the
// exclusive prefix of the packed (a, b) pair; waits are bounded (d.spin_ticks,
// 2 s unless a test shortens it) and a time-out sets the world's error word,
// after which every phase kernel of the world exits at once (the prefixes of
// a timed-out scan are partial sums: every index they yield stays in range,
// but the step's state is not valid).  `withhold`: publish nothing (a test
// hook that makes the next tile's wait time out).
// ---------------------------------------------------------------------------
constexpr int kTileN = 64;   // live-list entries per move / claim tile
constexpr int kCntBits = 21;
constexpr uint64_t kCntMask = (uint64_t(1) << kCntBits) - 1;
constexpr uint64_t kValMask = (uint64_t(1) << (2 * kCntBits)) - 1;

__device__ __forceinline__ uint64_t pack2(uint32_t a, uint32_t b) { return (uint64_t(a) << kCntBits) | b; }
__device__ __forceinline__ uint32_t unpack_a(uint64_t v) { return uint32_t((v >> kCntBits) & kCntMask); }
__device__ __forceinline__ uint32_t unpack_b(uint64_t v) { return uint32_t(v & kCntMask); }

__device__ __forceinline__ uint64_t lookback(DevRef d, uint64_t* st, int tile, uint32_t epoch, uint64_t local,
                                             int lane, bool withhold = false) {
    // Publish this tile's total, then examine the predecessors 64 at a time
    // (one status word per lane) until the nearest one holding an inclusive
    // prefix: the prefix is that word plus the totals in between.
    const uint64_t tag = uint64_t(epoch & 0xFFFFFu);
    if (lane == 0 && !withhold)
        __hip_atomic_store(st + tile, (tag << 44) | (uint64_t(tile == 0 ? 2 : 1) << 42) | local, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    uint64_t excl = 0;
    int end = tile;
    const uint64_t t0 = wall_clock64();
    const uint64_t limit = d.spin_ticks;
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
                if (wall_clock64() - t0 > limit) {
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
    if (lane == 0 && tile != 0 && !withhold)
        __hip_atomic_store(st + tile, (tag << 44) | (uint64_t(2) << 42) | (excl + local), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

// Exclusive ranks of two predicates within the wave and the wave totals.
struct WaveRank {
    int ra, rb;   // this lane's exclusive rank among the wave's a / b
    int ta, tb;   // wave totals
};

__device__ __forceinline__ WaveRank wave_rank2(bool a, bool b, int lane) {
    const uint64_t ma = __ballot(a), mb = __ballot(b);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    return {int(__popcll(ma & lt)), int(__popcll(mb & lt)), int(__popcll(ma)), int(__popcll(mb))};
}

// ---------------------------------------------------------------------------
// P2: moves (one thread per live agent).  A move was claimed in P1 only into
// an in-grid cell empty at the step start, and the cell's claim word holds
// the smallest (MOVE draw, uid) of its claimants: the agent moves iff that is
// its own key.  Then: eat the
// resource of the final cell, energy += gain * ate - decay, age += 1, death
// at energy <= 0 or age >= L_max, streak of survivors.  occB receives the
// moves and deaths; occA (read by every agent in this phase) is untouched.
// Returns bit 0 = ate, bit 1 = died, bit 2 = had a resource in view, bits
// 3.. = input rows its act phase read.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int move_agent(DevRef d, const AgentRec& a, int64_t t, PostRec* post,
                                          AgentRec* next_rec_src) {
    const int W = d.W, H = d.H;
    const int slot = a.slot;
    const int X = a.cell;
    const int act = a.action & kActMask;
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
    d.ate[slot] = uint8_t(ate);
    // Both occupancy grids take the moves and deaths (neither is read in this
    // phase): occA is the next step's start state, occB is read by P3.  A
    // survivor's occB word also says whether it is eligible to reproduce and
    // from which direction its birth scan starts; its birth key is stored at
    // its cell, so P3 learns a neighbour's claim from reads by cell alone.
    int word = -1;
    if (!dead) {
        word = slot;
        if (st >= d.T_repr) {
            const Draw4 b = philox(u, uint32_t(t), kBirth, 0, d.seed_lo, d.seed_hi);
            word |= kOccElig | int((b.x & 3u) << kOccDirShift);
            d.bkey[newX] = claim_key(b.y, u);
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
    nr.action = act;   // the previous action and ate bit of the next step
    nr.ate = ate;
    *next_rec_src = nr;
    return ate | (dead ? 2 : 0) | ((a.action & kSeenBit) ? 4 : 0) | (((a.action >> kRowsShift) & kRowsMask) << 3);
}

// P2 under the paper's dynamics (App. B.2, B.3): the move always happens,
// except into a wall (outside the grid), which kills; the agent eats the
// resource of its final cell iff its act-phase claim on that cell is the
// smallest; e <- min(e - decay + gain * ate, E_max); the signed streak counts
// consecutive steps above (+) or below (-) E_repr; death at -T_death, past
// L_max or at a wall.  occA (agents minus one per cell) takes the moves and
// deaths by atomic steps.  Same record outputs and return bits as move_agent.
__device__ __forceinline__ int move_agent_paper(DevRef d, const AgentRec& a, int64_t t, PostRec* post,
                                                AgentRec* next_rec_src) {
    const int W = d.W, H = d.H;
    const int slot = a.slot;
    const int X = a.cell;
    const int act = a.action & kActMask;
    const uint32_t u = a.uid;
    const int r = X / W, c = X - (X / W) * W;
    uint8_t* Rc = d.R[t & 1];
    const int tr = r + act_dr(act), tc = c + act_dc(act);
    const bool wall = !(tr >= 0 && tr < H && tc >= 0 && tc < W);
    const int newX = wall ? X : tr * W + tc;
    const uint64_t cw = d.mclaim[newX];
    const int rY = Rc[newX];
    int ate = 0;
    if (!wall && rY) {
        const uint64_t key = claim_key(philox(u, uint32_t(t), kEat, 0, d.seed_lo, d.seed_hi).x, u);
        ate = cw == key;
    }
    if (ate) Rc[newX] = 0;
    int en = a.energy - d.decay + d.gain * ate;
    if (en > d.E_max) en = d.E_max;
    const int ag = a.age + 1;
    int st = a.streak;
    if (en > d.E_repr) st = (st > 0 ? st : 0) + 1;
    else if (en < d.E_repr) st = (st < 0 ? st : 0) - 1;
    else st = 0;
    const bool dead = wall || -st >= d.T_death || ag > d.L_max;
    d.energy[slot] = en;
    d.age[slot] = ag;
    d.streak[slot] = st;
    d.cell[slot] = newX;
    d.prev_cell[slot] = X;
    d.alive[slot] = dead ? 0 : 1;
    d.ate[slot] = uint8_t(ate);
    if (dead || newX != X) atomicAdd(d.occA + X, -1);
    if (!dead && newX != X) atomicAdd(d.occA + newX, 1);
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
    nr.action = act;
    nr.ate = ate;
    *next_rec_src = nr;
    return ate | (dead ? 2 : 0) | ((a.action & kSeenBit) ? 4 : 0) | (((a.action >> kRowsShift) & kRowsMask) << 3);
}

// The world scalars a block works with, read once at its start.
struct StepScal {
    int64_t t;
    int n, sel, nc;
    int n_surv;   // survivors of this step's move phase (valid in its claim phase)
    int err;   // nonzero after a device failure: the world no longer steps
    uint32_t next_uid;
    int free_head, free_tail;
};

template <class P>
__device__ __forceinline__ StepScal read_step_from(P S) {
    StepScal s;
    s.t = S->t;
    s.n = S->n_live;
    s.n_surv = S->n_surv;
    s.sel = S->live_sel;
    s.nc = S->n_child;
    s.next_uid = S->next_uid;
    s.free_head = S->free_head;
    s.free_tail = S->free_tail;
    s.err = S->err;
    return s;
}

// Completes a load at this point, so that it stays among the loads issued
// together at a block's start instead of being moved into the branch that
// uses it (which would add a dependent round trip).  pin: per-lane values,
// pin_s: uniform values.
__device__ __forceinline__ void pin(int v) { asm volatile("" ::"v"(v)); }
__device__ __forceinline__ void pin_s(int v) { asm volatile("" ::"s"(v)); }
__device__ __forceinline__ void pin64(uint64_t v) { asm volatile("" ::"v"(v)); }

// The scalars through the scalar cache: no block writes them before every
// block of the same kernel that reads them has done so (the last claim tile
// rewrites them once its look-back has seen every other claim tile publish,
// which each does after reading them; the regrowth tiles read t_grow, which
// it does not write; the last move tile writes n_surv, which only the next
// kernel, the claim phase, uses).
__device__ __forceinline__ StepScal read_step(const WorldScal* S) {
    const StepScal s = read_step_from(kconst(S));
    pin_s(int(s.t));
    pin_s(s.n);
    pin_s(s.sel);
    pin_s(s.nc);
    return s;
}

constexpr int kMaxBlockWaves = 8;   // waves per block of the act kernels (2, 4 or 8)
struct StepShared {
    int sw[4 * kMaxBlockWaves];
    long long sw64[kMaxBlockWaves];
};

// P2 for tile `j` (kTileN live-list entries, one wave) of one world.
// Survivors keep their uid order in the next live list; dead slots are
// listed in uid order.  `r0` / `r1`: this lane's entry of both record lists,
// read before the scalars arrived.
__device__ __forceinline__ void move_block(DevRef d, PosRec* P, int j, int lane, const StepScal& ss,
                                           const AgentRec& r0, const AgentRec& r1) {
    const int i = j * kTileN + lane;
    const int n = ss.n;
    const int sel = ss.sel;
    const int64_t t = ss.t;
    int res = 0;
    AgentRec nr;
    nr.slot = -1;
    if (i < n)
        res = d.dyn == kDynPaper ? move_agent_paper(d, sel ? r1 : r0, t, &P[i].post, &nr)
                                 : move_agent(d, sel ? r1 : r0, t, &P[i].post, &nr);
    const bool alive = i < n && !(res & 2);
    const bool dead = i < n && (res & 2);
    const int cnt = __popcll(__ballot((res & 1) != 0));
    const int cnt_seen = __popcll(__ballot((res & 4) != 0));
    int rows = res >> 3;   // input rows read by the act phase
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) rows += __shfl_xor(rows, off);
    int dage = dead ? nr.age : 0;   // age at death (life expectancy, App. C)
    if (__ballot(dead)) {            // deaths are rare: most tiles skip the sum
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) dage += __shfl_xor(dage, off);
    }
    if (lane == 0) {
        d.eat_part[j] = cnt | (cnt_seen << 16);
        d.dage_part[j] = dage;
        d.rows_part[j] = rows;
    }
    // Movement metric (App. C): the window ends with this step; every
    // survivor whose slot recorded it at the window start counts, in bin
    // (Manhattan distance from that cell) / 3.
    if ((t + 1) % kMoveWin == 0) {
        bool counted = false;
        int bin = 0;
        if (alive && d.wuid[nr.slot] == nr.uid) {
            const int c0 = d.wcell[nr.slot];
            const int r0 = c0 / d.W, q0 = c0 - r0 * d.W;
            const int r1 = nr.cell / d.W, q1 = nr.cell - r1 * d.W;
            const int dist = abs(r1 - r0) + abs(q1 - q0);
            bin = dist / 3;
            counted = true;
        }
        int32_t* hist = d.mhist + ((t / kMoveWin) % kMoveRing) * (kMoveBins + 1);
        const int total = __popcll(__ballot(counted));
        if (total) {
            for (int b = 0; b < kMoveBins; ++b) {
                const int c = __popcll(__ballot(counted && bin == b));
                if (lane == 0 && c) __hip_atomic_fetch_add(hist + b, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (lane == 0) __hip_atomic_fetch_add(hist + kMoveBins, total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    const WaveRank wr = wave_rank2(alive, dead, lane);
    const uint64_t ex = lookback(d, d.lb_move, j, uint32_t(t), pack2(wr.ta, wr.tb), lane, j == d.stall_tile);
    // the last tile's inclusive prefix is the step's survivor count, which the
    // claim phase reads with its other scalars
    if (lane == 0 && j == (d.cap + kTileN - 1) / kTileN - 1) d.scal->n_surv = int(unpack_a(ex)) + wr.ta;
    if (alive) {
        const int pos = int(unpack_a(ex)) + wr.ra;
        d.live[sel ^ 1][pos] = nr.slot;
        P[pos].r[sel ^ 1] = nr;
        P[i].post.next_pos = pos;
    }
    if (dead) d.deadlist[unpack_b(ex) + wr.rb] = nr.slot;
}

// Direction of the first free cell among the four neighbours of the cell at
// offset (OY, OX), scanned N, S, E, W cyclically from `d0`; -1 if none.  `fr`
// is the free map of the radius-3 neighbourhood of the claiming agent.
template <int OY, int OX>
__device__ __forceinline__ int first_free_dir(const bool (&fr)[7][7], int d0) {
    int dir = -1;
#pragma unroll
    for (int k = 3; k >= 0; --k) {
#pragma unroll
        for (int dd = 0; dd < 4; ++dd) {
            const bool f = fr[OY + 3 + (dd == 0 ? -1 : (dd == 1 ? 1 : 0))][OX + 3 + (dd == 2 ? 1 : (dd == 3 ? -1 : 0))];
            if (((d0 + k) & 3) == dd && f) dir = dd;
        }
    }
    return dir;
}

// Does the agent whose post-move occB word is `v`, at offset (MY, MX) of the
// claimant, claim its neighbour in direction BACK?  Only an eligible agent
// claims; its claim is the first free neighbour from its own scan start,
// recomputed from the same free map.
template <int MY, int MX, int BACK>
__device__ __forceinline__ bool rival_claims(const bool (&fr)[7][7], int v) {
    if (v < 0 || !(v & kOccElig)) return false;
    return first_free_dir<MY, MX>(fr, (v >> kOccDirShift) & 3) == BACK;
}

// ---------------------------------------------------------------------------
// P3a: clear this agent's move-claim word, then, for an eligible survivor,
// compute its birth claim and resolve it against the other eligible agents
// next to the claimed cell.  A birth claim is the first free in-grid
// 4-neighbour (post-move, post-death occupancy) from the agent's scan start;
// a rival claiming the same cell sits two steps away and its own claim
// depends on cells up to three steps away, so the occB words of the whole
// radius-3 diamond (24 cells) and the birth keys of the 8 cells at distance
// 2 are loaded together, and the resolution is computed from them.  With
// no free slot (`room` false: the survivors fill the cap) no birth can
// follow, and no claim is made.
// Returns the claimed cell of a claim winner, -1 otherwise.
// ---------------------------------------------------------------------------
template <bool PAPER>
__device__ __forceinline__ int claim_agent(DevRef d, const PostRec& p, int64_t t, bool room) {
    const int X = p.prev_cell;
    const int X2 = p.cell;
    const bool alive = p.alive != 0 && room;
    constexpr bool paper = PAPER;
    {
        // clear the claim word this agent may have written in P1 (its move
        // target; under the paper's rules also its own cell when it stayed)
        const int a = p.action;
        if (a < 4 || paper) {
            const int tr = X / d.W + act_dr(a), tc = X - (X / d.W) * d.W + act_dc(a);
            if (tr >= 0 && tr < d.H && tc >= 0 && tc < d.W) d.mclaim[tr * d.W + tc] = ~0ull;
        }
    }
    int C = -1;
    bool won = false;
    if constexpr (PAPER) {
        // the paper's rules: the offspring appears on the parent's cell
        if (alive && p.streak >= d.T_repr) {
            won = true;
            C = X2;
        }
    } else if (alive && p.streak >= d.T_repr) {
        const int W = d.W, H = d.H;
        const int r = X2 / W, c = X2 - (X2 / W) * W;
        // occB words of the diamond (-2 outside the grid; the agent's own
        // cell is occupied by itself) and the keys at distance 2
        int occ[7][7];
        uint64_t kc[7][7];
#pragma unroll
        for (int dy = -3; dy <= 3; ++dy) {
#pragma unroll
            for (int dx = -3; dx <= 3; ++dx) {
                const int m = (dy < 0 ? -dy : dy) + (dx < 0 ? -dx : dx);
                occ[dy + 3][dx + 3] = 0;
                kc[dy + 3][dx + 3] = 0;
                if (m == 0 || m > 3) continue;
                const int rr = r + dy, cc = c + dx;
                const bool in = rr >= 0 && rr < H && cc >= 0 && cc < W;
                const int q = in ? rr * W + cc : X2;
                const int v = d.occB[q];
                occ[dy + 3][dx + 3] = in ? v : -2;
                if (m == 2) kc[dy + 3][dx + 3] = d.bkey[q];
            }
        }
        // one round trip for the whole neighbourhood
#pragma unroll
        for (int y = 0; y < 7; ++y)
#pragma unroll
            for (int x = 0; x < 7; ++x) {
                const int m = (y < 3 ? 3 - y : y - 3) + (x < 3 ? 3 - x : x - 3);
                if (m == 0 || m > 3) continue;
                pin(occ[y][x]);
                if (m == 2) pin64(kc[y][x]);
            }
        bool fr[7][7];
#pragma unroll
        for (int y = 0; y < 7; ++y)
#pragma unroll
            for (int x = 0; x < 7; ++x) fr[y][x] = occ[y][x] == -1;
        const uint32_t u = p.uid;
        const Draw4 b = philox(u, uint32_t(t), kBirth, 0, d.seed_lo, d.seed_hi);
        const int cdir = first_free_dir<0, 0>(fr, int(b.x & 3u));
        if (cdir >= 0) {
            const uint64_t key = claim_key(b.y, u);
            won = true;
            // rivals around C = own cell + e1: at e1 + e2 for the three e2
            // that do not lead back to the own cell; each claims C iff its
            // first free neighbour lies in direction -e2
#define ECO_RIVAL(E1, DY1, DX1, E2, DY2, DX2, BACK)                                                  \
    if (cdir == E1) {                                                                                \
        const int v_ = occ[DY1 + DY2 + 3][DX1 + DX2 + 3];                                           \
        if (rival_claims<DY1 + DY2, DX1 + DX2, BACK>(fr, v_) && kc[DY1 + DY2 + 3][DX1 + DX2 + 3] < key) \
            won = false;                                                                             \
    }
            // directions: 0 = N (-1, 0), 1 = S (+1, 0), 2 = E (0, +1), 3 = W (0, -1)
            ECO_RIVAL(0, -1, 0, 0, -1, 0, 1)
            ECO_RIVAL(0, -1, 0, 2, 0, 1, 3)
            ECO_RIVAL(0, -1, 0, 3, 0, -1, 2)
            ECO_RIVAL(1, 1, 0, 1, 1, 0, 0)
            ECO_RIVAL(1, 1, 0, 2, 0, 1, 3)
            ECO_RIVAL(1, 1, 0, 3, 0, -1, 2)
            ECO_RIVAL(2, 0, 1, 2, 0, 1, 3)
            ECO_RIVAL(2, 0, 1, 0, -1, 0, 1)
            ECO_RIVAL(2, 0, 1, 1, 1, 0, 0)
            ECO_RIVAL(3, 0, -1, 3, 0, -1, 2)
            ECO_RIVAL(3, 0, -1, 0, -1, 0, 1)
            ECO_RIVAL(3, 0, -1, 1, 1, 0, 0)
#undef ECO_RIVAL
            C = (r + act_dr(cdir)) * W + (c + act_dc(cdir));
        }
    }
    d.claim[p.slot] = C;
    return won ? C : -1;
}

// P3a for tile `j` (kTileN live-list entries, one wave) of one world.  The
// winner of global rank r (uid order) is born iff r < cap - survivors; its
// child takes free slot r of the ring if the ring holds more than r slots,
// else the (r - free)-th slot freed this step.  The last claim tile closes
// the step (counts, free ring, scalars) as soon as its look-back returns.  `p`: this lane's post-move
// record, read before the scalars arrived.
template <bool PAPER>
__device__ __forceinline__ void claim_block(DevRef d, WorldScal* S, PosRec* P, int j, int lane, const StepScal& ss,
                                            const PostRec& p) {
    const int cap = d.cap;
    const int i = j * kTileN + lane;
    const int n = ss.n;
    const int sel = ss.sel;
    const int64_t t = ss.t;
    const int surv = ss.n_surv;
    const int ntile = (cap + kTileN - 1) / kTileN;
    int slot = -1, cell = -1, pos = -1;
    bool win = false;
    if (i < n) {
        slot = p.slot;
        pos = p.next_pos;
        cell = claim_agent<PAPER>(d, p, t, surv < cap);
        win = cell >= 0;
    }
    const WaveRank wr = wave_rank2(win, false, lane);
    const uint64_t ex = lookback(d, d.lb_claim, j, uint32_t(t), pack2(wr.ta, 0), lane);
    const int nfree = cap - n;
    if (win) {
        const int rk = int(unpack_a(ex)) + wr.ra;
        if (rk < cap - surv) {
            int cs;
            if (rk < nfree) {
                int q = ss.free_head + rk;
                if (q >= cap) q -= cap;
                cs = d.freeq[q];
            } else {
                cs = d.deadlist[rk - nfree];
            }
            const uint32_t cu = ss.next_uid + uint32_t(rk);
            d.child[rk] = make_int4(cs, slot, cell, int(cu));
            d.live[sel ^ 1][surv + rk] = cs;
            AgentRec cr;
            cr.slot = cs;
            cr.cell = cell;
            cr.energy = d.E0;
            cr.uid = cu;
            cr.age = 0;
            cr.streak = 0;
            cr.action = kNoAction;
            cr.ate = 0;
            P[surv + rk].r[sel ^ 1] = cr;
            // occA is not read in this phase; under the paper's rules it
            // counts the agents per cell (several children may share one)
            if constexpr (PAPER) atomicAdd(d.occA + cell, 1);
            else d.occA[cell] = cs;
            // the parent's streak restarts (no phase reads these in P3)
            P[pos].r[sel ^ 1].streak = 0;
            d.streak[slot] = 0;
        }
    }
    // The last tile closes the step: its look-back prefix covers every other
    // tile, so all of them have read the scalars (they do so before
    // publishing their look-back word) and the totals are known.
    if (j != ntile - 1) return;
    const int wins = int(unpack_a(ex)) + wr.ta;
    const int dead = n - surv;
    const int nb = min(wins, cap - surv);
    const int consumed = max(0, nb - nfree);
    const int ft = ss.free_tail;
    for (int q = consumed + lane; q < dead; q += kTileN) {
        int fpos = ft + q - consumed;
        if (fpos >= cap) fpos -= cap;
        d.freeq[fpos] = d.deadlist[q];
    }
    if (lane == 0) {
        int nfh = ss.free_head + min(nb, nfree);
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
        S->next_uid = ss.next_uid + uint32_t(nb);
        S->live_sel = sel ^ 1;
        S->n_child = nb;
        S->spawn_t = t;
        S->ctr_open = 1;
        S->t = t + 1;
    }
}

// ---------------------------------------------------------------------------
// P3b: regrowth of one TILE x TILE tile (one wave, TILE * TILE / 64 cells per lane).
// The tile plus a 2-cell halo of the post-eating grid is staged in LDS; an
// empty cell counts the resources among its 24 neighbours and grows iff its
// REGROW draw is below thr[row][count].  Writes the other grid buffer
// (synchronous update) and the tile's resource count.
// ---------------------------------------------------------------------------
// Regrowth tile edges a launch may use (a tuning knob: every cell's result
// depends on its own draw and its 5 x 5 neighbourhood only, so the tiling
// changes nothing but the per-tile resource partials, which are integers).
constexpr int kTileMin = 8;
constexpr int kTileMax = 32;

template <int TILE>
__device__ __forceinline__ void regrow_tile(DevRef d, int tile, int lane, uint8_t* s, int64_t t, int ntiles) {
    constexpr int E = TILE + 4;
    const int ntx = (d.W + TILE - 1) / TILE;
    const int ty0 = (tile / ntx) * TILE;
    const int tx0 = (tile - (tile / ntx) * ntx) * TILE;
    const uint8_t* Rc = d.R[t & 1];
    uint8_t* Rn = d.R[(t + 1) & 1];
    for (int idx = lane; idx < E * E; idx += 64) {
        const int ly = idx / E, lx = idx - (idx / E) * E;
        const int gy = ty0 + ly - 2, gx = tx0 + lx - 2;
        s[idx] = (gy >= 0 && gy < d.H && gx >= 0 && gx < d.W) ? Rc[gy * d.W + gx] : uint8_t(0);
    }
    __syncthreads();
    int total = 0;
#pragma unroll
    for (int part = 0; part < TILE * TILE / 64; ++part) {
        const int c = part * 64 + lane;
        const int ly = c / TILE, lx = c - (c / TILE) * TILE;
        const int gy = ty0 + ly, gx = tx0 + lx;
        int v = 0;
        if (gy < d.H && gx < d.W) {
            const int q = gy * d.W + gx;
            v = s[(ly + 2) * E + lx + 2];
            if (!v) {
                int cnt = 0;
                if (d.dyn == kDynPaper) {   // the four direct neighbours (App. B.1)
                    cnt = s[(ly + 1) * E + lx + 2] + s[(ly + 3) * E + lx + 2] + s[(ly + 2) * E + lx + 1] +
                          s[(ly + 2) * E + lx + 3];
                } else {
#pragma unroll
                    for (int dy = 0; dy < 5; ++dy)
#pragma unroll
                        for (int dx = 0; dx < 5; ++dx) cnt += s[(ly + dy) * E + lx + dx];
                }
                const Draw4 dr = philox(uint32_t(q), uint32_t(t), kRegrow, 0, d.seed_lo, d.seed_hi);
                v = uint64_t(dr.x) < d.thr[gy * 25 + cnt] ? 1 : 0;
            }
            Rn[q] = uint8_t(v);
        }
        total += __popcll(__ballot(v != 0));
    }
    if (lane == 0) {
        d.res_part[tile] = total;
        if (tile == 0) *d.res_ntiles = ntiles;   // how many partials the counter close sums
    }
}

// ---------------------------------------------------------------------------
// Child creation (start of P1, one block per child): the genome is
// theta_child[p] = fmaf(sigma, z_p, theta_parent[p]) with z_p lane p % 4 of
// the MUTATE draw (child uid, birth step, block p / 4); the record gets
// energy E0, age 0, streak 0, no previous action, a zero recurrent state;
// the child enters occB
// (occA received it when it was born; the parent's streak restarted then).
// Every store is complete when this returns, so the same block can run the
// child's controller right after a block barrier.  `ss`: recurrent state
// floats per slot (the caller's, so that the GRU act kernel sizes it by the
// descriptor field its controller already reads).
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ void spawn_child(DevRef d, int rk, int tid, int ss) {
    const int4 rec = d.child[rk];   // child slot, parent slot, cell, uid
    const uint32_t ts = uint32_t(d.scal->spawn_t);
    const float* par = d.theta + size_t(rec.y) * size_t(d.Ppad);
    float* out = d.theta + size_t(rec.x) * size_t(d.Ppad);
    for (int blk = tid; blk < d.nblk; blk += NT) {
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
        d.action[cs] = kNoAction;
        d.ate[cs] = 0;
        d.occB[rec.z] = cs;
    }
    if (tid < ss) d.h[size_t(cs) * ss + tid] = 0.f;
    __builtin_amdgcn_s_waitcnt(0);   // this thread's stores have completed
}

// Recurrent projection and window sums of a new agent of a GRU world (after
// spawn_child and a barrier).
template <int NT>
__device__ __forceinline__ void spawn_proj(DevRef d, int rk, int tid) {
    const int cs = d.child[rk].x;
    if (tid < 64) {
        if (d.hd == 32) proj_zero<32>(d, cs, tid);
        else proj_zero<16>(d, cs, tid);
    }
    rsum_agent(d, cs, tid, NT);
    __builtin_amdgcn_s_waitcnt(0);
}

// Eaten, resource and age-at-death totals of the step just closed (one block
// per world).
template <int NT>
__device__ __forceinline__ void close_counters(DevRef d, int tid, StepShared& sh) {
    WorldScal* S = d.scal;
    if (!S->ctr_open) return;
    const int nwv = (S->n_prev + 63) / 64;
    int pe = 0, pr = 0, ps = 0, pw = 0;
    long long pa = 0;
    for (int i = tid; i < nwv; i += NT) {
        const int ep = d.eat_part[i];
        pe += ep & 0xFFFF;
        ps += ep >> 16;
        pa += d.dage_part[i];
        pw += d.rows_part[i];
    }
    const int ntiles = *d.res_ntiles;
    for (int i = tid; i < ntiles; i += NT) pr += d.res_part[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        pe += __shfl_xor(pe, off);
        pr += __shfl_xor(pr, off);
        ps += __shfl_xor(ps, off);
        pa += __shfl_xor(pa, off);
        pw += __shfl_xor(pw, off);
    }
    constexpr int NW = NT / 64;
    if ((tid & 63) == 0) {
        sh.sw[tid >> 6] = pe;
        sh.sw[NW + (tid >> 6)] = pr;
        sh.sw[2 * NW + (tid >> 6)] = ps;
        sh.sw[3 * NW + (tid >> 6)] = pw;
        sh.sw64[tid >> 6] = pa;
    }
    __syncthreads();
    if (tid == 0) {
        int te = 0, tr = 0, ts = 0, tw = 0;
        long long ta = 0;
        for (int w = 0; w < NW; ++w) {
            te += sh.sw[w];
            tr += sh.sw[NW + w];
            ts += sh.sw[2 * NW + w];
            tw += sh.sw[3 * NW + w];
            ta += sh.sw64[w];
        }
        int32_t* rec = d.ring + (S->spawn_t % kRing) * kCtrWords;
        rec[kCtrEaten] = te;
        rec[kCtrRes] = tr;
        rec[kCtrDeadAgeLo] = int32_t(uint64_t(ta) & 0xFFFFFFFFu);
        rec[kCtrDeadAgeHi] = int32_t(uint64_t(ta) >> 32);
        rec[kCtrSeen] = ts;
        rec[kCtrRows] = tw;
    }
    __syncthreads();
}

// P1 bookkeeping by the first block of a world: sum the eaten / resource
// partials of the previous step (written by its P2 and P3).
template <int NT>
__device__ __forceinline__ void close_counters_in_step(DevRef d, int tid, StepShared& sh) {
    close_counters<NT>(d, tid, sh);
    if (tid == 0) d.scal->ctr_open = 0;
}

}  // namespace eco
