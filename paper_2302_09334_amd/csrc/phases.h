// phases.h -- device code of one world step (gfx950, wave64).
//
// A step is split into five phases separated by device-wide ordering points
// (kernel boundaries or grid barriers):
//   P1 act     observe + GRU controller + arg-max, one wave per agent
//   P2 move    move resolution, eating, energy, age, death, streak
//   P3 claim   birth claims and their resolution; regrowth of the grid
//   P4 scan    one block per world: survivors, deaths and winners in uid
//              order, slot allocation for children, live-list compaction
//   P5 spawn   child genomes (parent + sigma * N(0, 1)) and child records
// Every decision is a gather: an agent reads its neighbours' state and
// decides on its own, so no phase needs atomics except the integer counters.
//
// Paper mapping: observation and controller App. B.2/B.5, moves and energy
// App. B.2, reproduction/mutation/death App. B.3, regrowth App. B.1 Eq. (1).
#pragma once

#include <hip/hip_runtime.h>

#include "rng.h"
#include "world_dev.h"

namespace eco {

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
template <int HD>
__device__ __forceinline__ void act_agent(const WorldDev& d, int slot, int li, int64_t t, int lane) {
    constexpr int G = 64 / HD;
    constexpr int RW = 3 * HD;   // floats per input row
    constexpr int JJ = HD / G;   // recurrent rows per group
    constexpr int B = 8;         // input rows per group per batch
    const int g = lane / HD;
    const int k = lane - g * HD;
    const int H = d.H, W = d.W;
    const int cell = d.cell[slot];
    const int r = cell / W;
    const int c = cell - r * W;
    const int e = d.energy[slot];
    const float* th = d.theta + size_t(slot) * size_t(d.Ppad);

    // A child created in the previous step is entered into occB here, where
    // no phase reads occB.
    if (lane == 0 && d.age[slot] == 0) d.occB[cell] = slot;

    // Recurrent weights and hidden state do not depend on the observation:
    // issue them first.
    const float hk = d.h[size_t(slot) * HD + k];
    float whr[JJ], whz[JJ], whn[JJ];
#pragma unroll
    for (int jj = 0; jj < JJ; ++jj) {
        const float* p = th + d.off_hh + (jj * G + g) * RW + 3 * k;
        whr[jj] = p[0];
        whz[jj] = p[1];
        whn[jj] = p[2];
    }

    // Observation: lane q < w^2 looks at window cell (q / w - rho, q % w - rho).
    const int rho = d.rho;
    const int win = 2 * rho + 1;
    const int w2 = win * win;
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

    const int erow = 2 * w2;   // energy input row
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
        ar += __shfl_xor(ar, off);
        az += __shfl_xor(az, off);
        an += __shfl_xor(an, off);
        hr += __shfl_xor(hr, off);
        hz += __shfl_xor(hz, off);
        hn += __shfl_xor(hn, off);
    }

    const float xe = float(e) / float(d.E0);
    const float* pe = th + erow * RW + 3 * k;
    const float* pbi = th + d.off_bih + 3 * k;
    const float* pbh = th + d.off_bhh + 3 * k;
    const float gir = fmaf(xe, pe[0], ar) + pbi[0];
    const float giz = fmaf(xe, pe[1], az) + pbi[1];
    const float gin = fmaf(xe, pe[2], an) + pbi[2];
    const float ghr = hr + pbh[0];
    const float ghz = hz + pbh[1];
    const float ghn = hn + pbh[2];
    const float rg = sigmoidf_(gir + ghr);
    const float zg = sigmoidf_(giz + ghz);
    const float ng = tanhf(fmaf(rg, ghn, gin));
    const float hnew = fmaf(zg, hk - ng, ng);

    float lg[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        float v = hnew * th[d.off_wo + a * HD + k];
#pragma unroll
        for (int off = HD / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
        lg[a] = v + th[d.off_bo + a];
    }
    int best = 0;
#pragma unroll
    for (int a = 1; a < 5; ++a)
        if (lg[a] > lg[best]) best = a;
    if (d.forced >= 0) best = d.forced;

    if (g == 0) d.h[size_t(slot) * HD + k] = hnew;
    if (lane == 0) d.action[slot] = uint8_t(best);
    if (d.log_steps > 0) {
        const size_t row = size_t(t % d.log_steps) * size_t(d.cap) + size_t(li);
        if (lane == 0) {
            d.log_uid[row] = d.uid[slot];
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
    int32_t* rec = d.ring + (t % kRing) * kCtrWords;
    rec[kCtrEaten] = 0;
    rec[kCtrRes] = 0;
    if (d.log_steps > 0) d.log_n[t % d.log_steps] = d.scal->n_live;
}

// ---------------------------------------------------------------------------
// P2: moves (one thread per live agent).  A move is claimed only into an
// in-grid cell empty at the step start; the neighbours N of the target that
// claim it are exactly those whose action points from N to the target, and
// the smallest (MOVE draw, uid) among them wins.  Each agent evaluates the
// competition for its own target, so no claim grid is needed.  Then: eat the
// resource of the final cell, energy += gain * ate - decay, age += 1, death
// at energy <= 0 or age >= L_max, streak of survivors.  occB receives the
// moves and deaths; occA (read by every agent in this phase) is untouched.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int move_agent(const WorldDev& d, int slot, int64_t t) {
    const int W = d.W, H = d.H;
    const int X = d.cell[slot];
    const int a = d.action[slot];
    const uint32_t u = d.uid[slot];
    const int r = X / W, c = X - (X / W) * W;
    int newX = X;
    if (a < 4) {
        const int tr = r + act_dr(a), tc = c + act_dc(a);
        if (tr >= 0 && tr < H && tc >= 0 && tc < W) {
            const int Y = tr * W + tc;
            if (d.occA[Y] == -1) {
                const uint64_t key = claim_key(philox(u, uint32_t(t), kMove, 0, d.seed_lo, d.seed_hi).x, u);
                bool won = true;
                for (int d2 = 0; d2 < 4; ++d2) {
                    const int nr = tr - act_dr(d2), nc = tc - act_dc(d2);
                    if ((nr == r && nc == c) || nr < 0 || nr >= H || nc < 0 || nc >= W) continue;
                    const int o = d.occA[nr * W + nc];
                    if (o < 0 || d.action[o] != d2) continue;
                    const uint32_t uo = d.uid[o];
                    const uint64_t ko = claim_key(philox(uo, uint32_t(t), kMove, 0, d.seed_lo, d.seed_hi).x, uo);
                    if (ko < key) won = false;
                }
                if (won) newX = Y;
            }
        }
    }
    uint8_t* Rc = d.R[t & 1];
    const int ate = Rc[newX] != 0;
    if (ate) Rc[newX] = 0;
    const int en = d.energy[slot] - d.decay + d.gain * ate;
    const int ag = d.age[slot] + 1;
    const bool dead = en <= 0 || ag >= d.L_max;
    int st = d.streak[slot];
    if (!dead) st = (en >= d.E_repr) ? st + 1 : 0;
    d.energy[slot] = en;
    d.age[slot] = ag;
    d.streak[slot] = st;
    d.cell[slot] = newX;
    d.prev_cell[slot] = X;
    d.alive[slot] = dead ? 0 : 1;
    if (newX != X) {
        d.occB[X] = -1;
        if (!dead) d.occB[newX] = slot;
    } else if (dead) {
        d.occB[X] = -1;
    }
    return ate;
}

// First free in-grid 4-neighbour of `cell` (order N, S, E, W cyclically from
// `d0`) in the post-move, post-death occupancy; -1 if none.
__device__ __forceinline__ int birth_target(const WorldDev& d, int cell, int d0) {
    const int W = d.W, H = d.H;
    const int r = cell / W, c = cell - (cell / W) * W;
    for (int k = 0; k < 4; ++k) {
        const int dd = (d0 + k) & 3;
        const int nr = r + act_dr(dd), nc = c + act_dc(dd);
        if (nr >= 0 && nr < H && nc >= 0 && nc < W && d.occB[nr * W + nc] == -1) return nr * W + nc;
    }
    return -1;
}

// ---------------------------------------------------------------------------
// P3a: mirror this agent's move/death into occA, then, for an eligible
// survivor, compute its birth claim and resolve it against the other eligible
// agents next to the claimed cell (their claims are recomputed from occB).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void claim_agent(const WorldDev& d, int slot, int64_t t) {
    const int X = d.prev_cell[slot];
    const int X2 = d.cell[slot];
    const bool alive = d.alive[slot] != 0;
    if (!alive) {
        d.occA[X] = -1;
    } else if (X2 != X) {
        d.occA[X] = -1;
        d.occA[X2] = slot;
    }
    int C = -1;
    bool won = false;
    if (alive && d.streak[slot] >= d.T_repr) {
        const uint32_t u = d.uid[slot];
        const Draw4 b = philox(u, uint32_t(t), kBirth, 0, d.seed_lo, d.seed_hi);
        C = birth_target(d, X2, int(b.x & 3u));
        if (C >= 0) {
            const uint64_t key = claim_key(b.y, u);
            won = true;
            const int W = d.W, H = d.H;
            const int cr = C / W, cc = C - (C / W) * W;
            for (int dd = 0; dd < 4; ++dd) {
                const int mr = cr + act_dr(dd), mc = cc + act_dc(dd);
                if (mr < 0 || mr >= H || mc < 0 || mc >= W) continue;
                const int M = mr * W + mc;
                if (M == X2) continue;
                const int o = d.occB[M];
                if (o < 0 || d.streak[o] < d.T_repr) continue;
                const uint32_t uo = d.uid[o];
                const Draw4 bo = philox(uo, uint32_t(t), kBirth, 0, d.seed_lo, d.seed_hi);
                if (birth_target(d, M, int(bo.x & 3u)) != C) continue;
                if (claim_key(bo.y, uo) < key) won = false;
            }
        }
    }
    d.claim[slot] = C;
    d.win[slot] = won ? 1 : 0;
}

// ---------------------------------------------------------------------------
// P3b: regrowth of one kTile x kTile tile (one block).  The tile plus a
// 2-cell halo of the post-eating grid is staged in LDS; an empty cell counts
// the resources among its 24 neighbours and grows iff its REGROW draw is
// below thr[row][count].  Writes the other grid buffer (synchronous update).
// Returns the number of resources in the tile after regrowth (lane 0 of each
// wave holds its wave's count).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int regrow_tile(const WorldDev& d, int tile, int64_t t, int tid, uint8_t* s) {
    constexpr int E = kTile + 4;
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
            int n = 0;
#pragma unroll
            for (int dy = 0; dy < 5; ++dy)
#pragma unroll
                for (int dx = 0; dx < 5; ++dx) n += s[(ly + dy) * E + lx + dx];
            const Draw4 dr = philox(uint32_t(q), uint32_t(t), kRegrow, 0, d.seed_lo, d.seed_hi);
            v = uint64_t(dr.x) < d.thr[gy * 25 + n] ? 1 : 0;
        }
        Rn[q] = uint8_t(v);
    }
    const int cnt = __popcll(__ballot(v != 0));
    __syncthreads();   // the tile buffer is reused by the next tile
    return cnt;
}

// Exclusive prefix sums of three per-thread counts over a block of kBlock
// threads; also returns the block totals.  `sm` holds 3 * (kBlock / 64) ints.
__device__ __forceinline__ void block_scan3(int a, int b, int c, int& ea, int& eb, int& ec, int& ta,
                                            int& tb, int& tc, int tid, int* sm) {
    const int lane = tid & 63, wv = tid >> 6;
    int ia = a, ib = b, ic = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int xa = __shfl_up(ia, off), xb = __shfl_up(ib, off), xc = __shfl_up(ic, off);
        if (lane >= off) {
            ia += xa;
            ib += xb;
            ic += xc;
        }
    }
    constexpr int NW = kBlock / 64;
    if (lane == 63) {
        sm[wv] = ia;
        sm[NW + wv] = ib;
        sm[2 * NW + wv] = ic;
    }
    __syncthreads();
    int pa = 0, pb = 0, pc = 0;
    ta = tb = tc = 0;
    for (int w = 0; w < NW; ++w) {
        if (w < wv) {
            pa += sm[w];
            pb += sm[NW + w];
            pc += sm[2 * NW + w];
        }
        ta += sm[w];
        tb += sm[NW + w];
        tc += sm[2 * NW + w];
    }
    ea = pa + ia - a;
    eb = pb + ib - b;
    ec = pc + ic - c;
    __syncthreads();
}

// ---------------------------------------------------------------------------
// P4: one block per world.  In uid order (the live list): survivors are
// compacted into the other live buffer, dead slots are appended to the free
// ring, and birth-claim winners are ranked; the first min(winners, cap -
// survivors) are born, taking free slots from the head of the ring (pushes
// happen before pops, so a slot freed by a death this step can be reused).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void scan_world(const WorldDev& d, int tid, int* sm) {
    WorldScal* S = d.scal;
    const int n = S->n_live;
    const int sel = S->live_sel;
    const int64_t t = S->t;
    const uint32_t next_uid = S->next_uid;
    const int fh = S->free_head, ft = S->free_tail;
    const int cap = d.cap;
    const int* L = d.live[sel];
    int* Ln = d.live[sel ^ 1];
    const int per = (n + kBlock - 1) / kBlock;
    const int beg = min(n, tid * per);
    const int end = min(n, beg + per);
    int cs = 0, cd = 0, cw = 0;
    for (int i = beg; i < end; ++i) {
        const int s = L[i];
        if (d.alive[s]) {
            ++cs;
            cw += d.win[s];
        } else {
            ++cd;
        }
    }
    int os, od, ow, ns, nd, nw;
    block_scan3(cs, cd, cw, os, od, ow, ns, nd, nw, tid, sm);
    const int nb = min(nw, cap - ns);
    for (int i = beg; i < end; ++i) {
        const int s = L[i];
        if (d.alive[s]) {
            Ln[os++] = s;
        } else {
            int q = ft + od++;
            if (q >= cap) q -= cap;
            d.freeq[q] = s;
        }
    }
    __syncthreads();
    for (int i = beg; i < end; ++i) {
        const int s = L[i];
        if (d.alive[s] && d.win[s]) {
            const int rk = ow++;
            if (rk < nb) {
                int q = fh + rk;
                if (q >= cap) q -= cap;
                const int cslot = d.freeq[q];
                Ln[ns + rk] = cslot;
                d.child[rk] = make_int4(cslot, s, d.claim[s], int(next_uid + uint32_t(rk)));
                d.streak[s] = 0;
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        int nfh = fh + nb;
        if (nfh >= cap) nfh -= cap;
        int nft = ft + nd;
        if (nft >= cap) nft -= cap;
        S->free_head = nfh;
        S->free_tail = nft;
        S->n_live = ns + nb;
        S->next_uid = next_uid + uint32_t(nb);
        S->live_sel = sel ^ 1;
        S->n_child = nb;
        S->spawn_t = t;
        S->t = t + 1;
        int32_t* rec = d.ring + (t % kRing) * kCtrWords;
        rec[kCtrLive] = ns + nb;
        rec[kCtrBirths] = nb;
        rec[kCtrDeaths] = nd;
        rec[kCtrWins] = nw;
    }
}

// ---------------------------------------------------------------------------
// P5: one (child, chunk) item; a chunk is kBlock float4 blocks of the genome.
// theta_child[p] = fmaf(sigma, z_p, theta_parent[p]) with z_p lane p % 4 of
// the MUTATE draw (child uid, step, block p / 4).  Chunk 0 also writes the
// child's record (energy E0, age 0, streak 0, zero hidden state) and its occA
// cell; occB receives it in the next P1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void spawn_item(const WorldDev& d, int item, int nchunks, int tid) {
    const int rk = item / nchunks;
    const int q = item - rk * nchunks;
    const int4 rec = d.child[rk];   // child slot, parent slot, cell, uid
    const uint32_t ts = uint32_t(d.scal->spawn_t);
    const int blk = q * kBlock + tid;
    if (blk < d.nblk) {
        const int p0 = 4 * blk;
        const float4 par = *reinterpret_cast<const float4*>(d.theta + size_t(rec.y) * size_t(d.Ppad) + p0);
        const Draw4 dr = philox(uint32_t(rec.w), ts, kMutate, uint32_t(blk), d.seed_lo, d.seed_hi);
        float z0, z1, z2, z3;
        box_muller(dr.x, dr.y, z0, z1);
        box_muller(dr.z, dr.w, z2, z3);
        float4 o;
        o.x = fmaf(d.sigma, z0, par.x);
        o.y = p0 + 1 < d.P ? fmaf(d.sigma, z1, par.y) : 0.f;
        o.z = p0 + 2 < d.P ? fmaf(d.sigma, z2, par.z) : 0.f;
        o.w = p0 + 3 < d.P ? fmaf(d.sigma, z3, par.w) : 0.f;
        *reinterpret_cast<float4*>(d.theta + size_t(rec.x) * size_t(d.Ppad) + p0) = o;
    }
    if (q == 0) {
        const int cs = rec.x;
        if (tid == 0) {
            d.uid[cs] = uint32_t(rec.w);
            d.cell[cs] = rec.z;
            d.prev_cell[cs] = rec.z;
            d.energy[cs] = d.E0;
            d.age[cs] = 0;
            d.streak[cs] = 0;
            d.alive[cs] = 1;
            d.win[cs] = 0;
            d.claim[cs] = -1;
            d.action[cs] = 4;
            d.occA[rec.z] = cs;
        }
        if (tid < d.hd) d.h[size_t(cs) * d.hd + tid] = 0.f;
    }
}

}  // namespace eco
