// net.h -- act phase with the paper's controller (App. B.5), one wave per
// agent (gfx950, wave64).
//
// The network: the 15 x 15 x 3 observation (resource, agents, wall; App.
// B.2), conv 3x3 stride 2 with 4 features (zero padding 1), average pool 2x2
// stride 1, conv 3x3 stride 2 with 8 features (zero padding 1), average pool
// 2x2 stride 1, flattened (row, column, channel) to 72 features; the
// embedding appends the one-hot previous action (zero before the first) and
// the ate bit (78 values); an LSTM cell of 4 units (gates i, f, g, o, input
// kernel without bias, hidden kernel with bias); a dense layer of 8 with tanh
// over [embedding, new h] (82 values); 5 logits.  The action is sampled from
// the softmax at temperature 1/50 as arg max (50 l + Gumbel), the Gumbel
// terms from the ACT draws of the agent.  2445 parameters in the genome order
// conv1 K[ky][kx][ci][co], b; conv2 K[ky][kx][ci][co], b; LSTM Wi[i][gate]
// [unit], Wh[j][gate][unit], b[gate][unit]; dense W[i][o], b; dense W[o][a], b.
//
// Mapping.  Every weight load and the observation gather are issued at the
// start (one round trip from HBM); the layers then pass activations through
// the wave's own LDS:
//   conv1  lane = output pixel (8 x 8).  The inputs are bits and a wall pixel
//          holds nothing else, so each tap's contribution is one of five
//          weight sums (none, R, A, R + A, wall), tabulated per agent in LDS:
//          nine float4 lookups per lane instead of 108 multiply-adds.
//   pool1  lane = pooled pixel (7 x 7), four channels as a float4.
//   conv2  lane = (output channel, pixel pair): the 36 weights of its
//          channel in registers, the pooled inputs read as float4 (4 ci).
//   pool2  lane = feature (72, two per lane for the last eight).
//   LSTM   lane = (input group of 16, gate): float4 rows of the input kernel
//          (each load instruction covers 1 KB of the genome contiguously),
//          reduced over the input groups by an xor tree.
//   dense  lane = (input group of 32, half of the 8 outputs), same scheme.
//   head   lane = action (5 lanes), then the sampling draw on the same lanes.
// The summation order of every value depends only on the agent, never on the
// launch shape.
#pragma once

#include "phases.h"

namespace eco {
namespace net {

constexpr int kRho = 7;
constexpr int kWin = 2 * kRho + 1;      // 15
constexpr int kPix = kWin * kWin;       // 225
constexpr int kO1 = 8;                  // conv1 output edge: ceil(15 / 2)
constexpr int kP1 = kO1 - 1;            // 7
constexpr int kO2 = 4;                  // conv2 output edge: ceil(7 / 2)
constexpr int kP2 = kO2 - 1;            // 3
constexpr int kF1 = 4, kF2 = 8;
constexpr int kFlat = kP2 * kP2 * kF2;  // 72
constexpr int kEmb = kFlat + 5 + 1;     // 78
constexpr int kHd = 4;
constexpr int kCat = kEmb + kHd;        // 82
constexpr int kD = 8, kNA = 5;
constexpr int kState = 2 * kHd;         // h then c

// genome offsets (floats)
constexpr int kC1w = 0;
constexpr int kC1b = kC1w + 9 * 3 * kF1;       // 108
constexpr int kC2w = kC1b + kF1;               // 112
constexpr int kC2b = kC2w + 9 * kF1 * kF2;     // 400
constexpr int kLwi = kC2b + kF2;               // 408
constexpr int kLwh = kLwi + kEmb * 4 * kHd;    // 1656
constexpr int kLb = kLwh + kHd * 4 * kHd;      // 1720
constexpr int kD8w = kLb + 4 * kHd;            // 1736
constexpr int kD8b = kD8w + kCat * kD;         // 2392
constexpr int kD5w = kD8b + kD;                // 2400
constexpr int kD5b = kD5w + kD * kNA;          // 2440
constexpr int kP = kD5b + kNA;                 // 2445
static_assert(kP == 2445, "parameter count of the paper's network");
static_assert(kC1b % 4 == 0 && kLwi % 4 == 0 && kLwh % 4 == 0 && kLb % 4 == 0 && kD8w % 4 == 0 && kD8b % 4 == 0,
              "float4 rows");

// One wave's scratch.
struct alignas(16) WaveLds {
    float tab[9][5][4];   // conv1: weight sum of each channel combination per tap
    float a1[kO1 * kO1][kF1];
    float p1[kP1 * kP1][kF1];
    float a2[kO2 * kO2][kF2];
    float emb[84];        // embedding (78), then the new h (4)
    float z[16];          // LSTM pre-activations [gate][unit]
    float y8[kD];
    uint8_t obs[kPix + 7];   // pixel bits: 1 resource, 2 agent, 4 wall
};

// LDS written by some lanes of the wave is read by others below: complete
// the writes and keep the compiler from moving LDS accesses across.
__device__ __forceinline__ void wave_lds_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ float4 add4(float4 a, float4 b) {
    return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}

__device__ __forceinline__ float4 fma4(float s, float4 w, float4 acc) {
    return make_float4(fmaf(s, w.x, acc.x), fmaf(s, w.y, acc.y), fmaf(s, w.z, acc.z), fmaf(s, w.w, acc.w));
}

__device__ __forceinline__ float4 xor_sum4(float4 v, int off) {
    return make_float4(v.x + __shfl_xor(v.x, off), v.y + __shfl_xor(v.y, off), v.z + __shfl_xor(v.z, off),
                       v.w + __shfl_xor(v.w, off));
}

__device__ __forceinline__ float sigm(float v) { return 1.0f / (1.0f + expf(-v)); }

__device__ __forceinline__ void pin4(float4 v) {
    asm volatile("" ::"v"(v.x), "v"(v.y), "v"(v.z), "v"(v.w));
}
__device__ __forceinline__ void pinf(float v) { asm volatile("" ::"v"(v)); }

// `rv`, `rv2`: the agent's record (slot, cell, energy, uid / age, streak,
// previous action, ate).
__device__ __forceinline__ void act_agent(DevRef d, AgentRec* recp, int4 rv, int4 rv2, int li, int64_t t, int lane,
                                          WaveLds& L) {
    const int H = d.H, W = d.W;
    const int slot = rv.x;
    const int cell = rv.y;
    const uint32_t u = uint32_t(rv.w);
    const int prev = rv2.z;
    const int ate = rv2.w;
    const int r = cell / W;
    const int c = cell - r * W;
    const float* th = d.theta + size_t(slot) * size_t(d.Ppad);
    const float* hs = d.h + size_t(slot) * kState;
    const uint8_t* R = d.R[t & 1];

    // ---- one round trip: observation, state and every weight --------------
    int pb[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int q = lane + 64 * m;
        const int iy = q / kWin, ix = q - (q / kWin) * kWin;
        const int rr = r + iy - kRho, cc = c + ix - kRho;
        const bool in = q < kPix && rr >= 0 && rr < H && cc >= 0 && cc < W;
        const int qc = in ? rr * W + cc : cell;   // every lane loads (clamped)
        const int rb = R[qc];
        const int ob = d.occA[qc];
        pb[m] = in ? ((rb != 0 ? 1 : 0) | (ob != -1 ? 2 : 0)) : 4;
    }
    const float4 hv = *reinterpret_cast<const float4*>(hs);   // h (uniform)
    const float ck = hs[kHd + (lane & 3)];                       // c of unit lane % 4
    // conv1 weights of tap lane / 4, output channel lane % 4 (lanes < 36)
    const int l36 = min(lane, 35);
    const float w1r = th[kC1w + ((l36 >> 2) * 3 + 0) * kF1 + (l36 & 3)];
    const float w1a = th[kC1w + ((l36 >> 2) * 3 + 1) * kF1 + (l36 & 3)];
    const float w1w = th[kC1w + ((l36 >> 2) * 3 + 2) * kF1 + (l36 & 3)];
    const float4 b1 = *reinterpret_cast<const float4*>(th + kC1b);
    // conv2: the 36 weights of output channel lane % 8
    const int co2 = lane & 7;
    float w2[36];
#pragma unroll
    for (int k = 0; k < 36; ++k) w2[k] = th[kC2w + k * kF2 + co2];
    const float b2 = th[kC2b + co2];
    // LSTM: rows ig + 16 m of the input kernel, gate q = lane % 4
    const int ig = lane >> 2, gq = lane & 3;
    float4 wi[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        const int i = min(ig + 16 * m, kEmb - 1);
        wi[m] = *reinterpret_cast<const float4*>(th + kLwi + i * 16 + gq * 4);
    }
    float4 wh[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) wh[j] = *reinterpret_cast<const float4*>(th + kLwh + j * 16 + gq * 4);
    const float4 lb = *reinterpret_cast<const float4*>(th + kLb + gq * 4);
    // dense 8: rows ig8 + 32 m, outputs 4 hf .. 4 hf + 3
    const int ig8 = lane >> 1, hf = lane & 1;
    float4 w8[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const int i = min(ig8 + 32 * m, kCat - 1);
        w8[m] = *reinterpret_cast<const float4*>(th + kD8w + i * kD + hf * 4);
    }
    const float4 b8 = *reinterpret_cast<const float4*>(th + kD8b + hf * 4);
    // head: column a = lane (lanes < 5)
    const int a5 = min(lane, kNA - 1);
    float w5[kD];
#pragma unroll
    for (int o = 0; o < kD; ++o) w5[o] = th[kD5w + o * kNA + a5];
    const float b5 = th[kD5b + a5];
    // complete the loads here, so that none is moved into a branch that uses
    // it (which would add a dependent round trip)
#pragma unroll
    for (int m = 0; m < 4; ++m) pin(pb[m]);
    pinf(w1r);
    pinf(w1a);
    pinf(w1w);
    pin4(b8);

    // ---- observation bits and the conv1 table into LDS ---------------------
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int q = lane + 64 * m;
        if (q < kPix) L.obs[q] = uint8_t(pb[m]);
    }
    if (lane < 36) {
        float* tp = &L.tab[lane >> 2][0][lane & 3];
        tp[0 * 4] = 0.f;
        tp[1 * 4] = w1r;
        tp[2 * 4] = w1a;
        tp[3 * 4] = w1r + w1a;
        tp[4 * 4] = w1w;
    }
    wave_lds_sync();

    // ---- conv1: lane = output pixel ------------------------------------------
    {
        const int oy = lane >> 3, ox = lane & 7;
        float4 acc = b1;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int iy = 2 * oy - 1 + ky, ix = 2 * ox - 1 + kx;
                const bool ok = iy >= 0 && iy < kWin && ix >= 0 && ix < kWin;
                const int bits = ok ? L.obs[iy * kWin + ix] : 0;   // zero padding
                const float4 v = *reinterpret_cast<const float4*>(&L.tab[ky * 3 + kx][bits][0]);
                acc = add4(acc, v);
            }
        *reinterpret_cast<float4*>(&L.a1[lane][0]) = acc;
    }
    wave_lds_sync();

    // ---- pool1: lane = pooled pixel ------------------------------------------
    if (lane < kP1 * kP1) {
        const int y = lane / kP1, x = lane - (lane / kP1) * kP1;
        const float4 v00 = *reinterpret_cast<const float4*>(&L.a1[y * kO1 + x][0]);
        const float4 v01 = *reinterpret_cast<const float4*>(&L.a1[y * kO1 + x + 1][0]);
        const float4 v10 = *reinterpret_cast<const float4*>(&L.a1[(y + 1) * kO1 + x][0]);
        const float4 v11 = *reinterpret_cast<const float4*>(&L.a1[(y + 1) * kO1 + x + 1][0]);
        const float4 s = add4(add4(add4(v00, v01), v10), v11);
        *reinterpret_cast<float4*>(&L.p1[lane][0]) =
            make_float4(s.x * 0.25f, s.y * 0.25f, s.z * 0.25f, s.w * 0.25f);
    }
    wave_lds_sync();

    // ---- conv2: lane = (channel lane % 8, pixels lane / 8 and lane / 8 + 8) --
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const int p = (lane >> 3) + 8 * half;
        const int oy = p >> 2, ox = p & 3;
        float acc = 0.f;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int iy = 2 * oy - 1 + ky, ix = 2 * ox - 1 + kx;
                const bool ok = iy >= 0 && iy < kP1 && ix >= 0 && ix < kP1;
                const int q = ok ? iy * kP1 + ix : 0;
                float4 v = *reinterpret_cast<const float4*>(&L.p1[q][0]);
                if (!ok) v = make_float4(0.f, 0.f, 0.f, 0.f);   // zero padding
                const int k = (ky * 3 + kx) * kF1;
                acc = fmaf(v.x, w2[k + 0], acc);
                acc = fmaf(v.y, w2[k + 1], acc);
                acc = fmaf(v.z, w2[k + 2], acc);
                acc = fmaf(v.w, w2[k + 3], acc);
            }
        L.a2[p][co2] = acc + b2;
    }
    wave_lds_sync();

    // ---- pool2 into the embedding, then the previous action and ate bit -----
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int f = lane + 64 * m;   // (y, x, channel) = (f / 24, f / 8 % 3, f % 8)
        if (f < kFlat) {
            const int y = f / 24, x = (f >> 3) % 3, ch = f & 7;
            const float s = ((L.a2[y * kO2 + x][ch] + L.a2[y * kO2 + x + 1][ch]) + L.a2[(y + 1) * kO2 + x][ch]) +
                            L.a2[(y + 1) * kO2 + x + 1][ch];
            L.emb[f] = s * 0.25f;
        }
    }
    if (lane < kNA) L.emb[kFlat + lane] = (prev == lane) ? 1.f : 0.f;
    if (lane == kNA) L.emb[kFlat + kNA] = ate ? 1.f : 0.f;
    wave_lds_sync();

    // ---- LSTM: lane = (input group, gate) ------------------------------------
    {
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            const int i = ig + 16 * m;
            const float e = i < kEmb ? L.emb[min(i, kEmb - 1)] : 0.f;
            acc = fma4(e, wi[m], acc);
        }
#pragma unroll
        for (int off = 4; off < 64; off <<= 1) acc = xor_sum4(acc, off);
        float4 rec = make_float4(0.f, 0.f, 0.f, 0.f);
        rec = fma4(hv.x, wh[0], rec);
        rec = fma4(hv.y, wh[1], rec);
        rec = fma4(hv.z, wh[2], rec);
        rec = fma4(hv.w, wh[3], rec);
        const float4 z = add4(add4(acc, rec), lb);
        if (lane < 4) *reinterpret_cast<float4*>(&L.z[gq * 4]) = z;
    }
    wave_lds_sync();
    float hnew, cnew;
    {
        const int k = lane & 3;   // unit
        const float zi = L.z[0 * 4 + k], zf = L.z[1 * 4 + k], zg = L.z[2 * 4 + k], zo = L.z[3 * 4 + k];
        cnew = fmaf(sigm(zf), ck, sigm(zi) * tanhf(zg));
        hnew = sigm(zo) * tanhf(cnew);
        if (lane < 4) L.emb[kEmb + k] = hnew;
    }
    wave_lds_sync();

    // ---- dense 8 with tanh: lane = (input group, half of the outputs) ------
    {
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int i = ig8 + 32 * m;
            const float e = i < kCat ? L.emb[min(i, kCat - 1)] : 0.f;
            acc = fma4(e, w8[m], acc);
        }
#pragma unroll
        for (int off = 2; off < 64; off <<= 1) acc = xor_sum4(acc, off);
        if (lane < 2) {
            L.y8[hf * 4 + 0] = tanhf(acc.x + b8.x);
            L.y8[hf * 4 + 1] = tanhf(acc.y + b8.y);
            L.y8[hf * 4 + 2] = tanhf(acc.z + b8.z);
            L.y8[hf * 4 + 3] = tanhf(acc.w + b8.w);
        }
    }
    wave_lds_sync();

    // ---- logits (lane a < 5) and the sampled action -----------------------------
    float lg = 0.f;
#pragma unroll
    for (int o = 0; o < kD; ++o) lg = fmaf(L.y8[o], w5[o], lg);
    lg = lg + b5;
    // sampling score 50 l + g, g from word a % 4 of ACT block a / 4
    const Draw4 dr = philox(u, uint32_t(t), kAct, lane < 4 ? 0u : 1u, d.seed_lo, d.seed_hi);
    const int wsel = lane & 3;
    const uint32_t word = lane >= 4 ? dr.x : (wsel == 0 ? dr.x : (wsel == 1 ? dr.y : (wsel == 2 ? dr.z : dr.w)));
    const float sc = 50.0f * lg + gumbel_of_word(word);
    int best = 0;
    float top = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sc), 0));
#pragma unroll
    for (int a = 1; a < kNA; ++a) {
        const float v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sc), a));
        if (v > top) {
            top = v;
            best = a;
        }
    }
    if (d.forced >= 0) best = d.forced;

    // ---- outputs ----------------------------------------------------------------
    if (lane < kHd) {
        d.h[size_t(slot) * kState + lane] = hnew;
        d.h[size_t(slot) * kState + kHd + lane] = cnew;
    }
    if (lane == 0 && t % kMoveWin == 0) {   // a movement window starts with this step
        d.wcell[slot] = cell;
        d.wuid[slot] = u;
    }
    if (lane == 0) {
        d.action[slot] = uint8_t(best);
        recp->action = best;
        // Move claim: the target must be inside the grid and empty at the
        // step start (no agent, no wall in the observation).
        if (best < 4) {
            const int q = (kRho + act_dr(best)) * kWin + (kRho + act_dc(best));
            if ((L.obs[q] & 6) == 0) {
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
        if (lane < kNA) d.log_logits[row * 5 + lane] = lg;
    }
}

}  // namespace net
}  // namespace eco
