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
//   conv2  lane = (output channel, pixel pair): per tap the 4 weights of
//          its channel and the pooled inputs as float4 reads (4 ci) from LDS.
//   pool2  lane = feature (72, two per lane for the last eight).
//   LSTM   lane = (input group of 16, gate): float4 rows of the input kernel
//          (each load instruction covers 1 KB of the genome contiguously),
//          reduced over the input groups by an xor tree; the recurrent term
//          h_j Wh[j][gate][unit] on the four lanes of a (gate, unit), one j
//          each, summed by two exchanges.
//   dense  lane = (input group of 32, half of the 8 outputs), same scheme.
//   head   lane = (action, input) for 40 lanes, one weight each, summed over
//          the 8 inputs by an xor tree; then lane = action (5 lanes) for the
//          sampling draw.
// Each lane holds only the weights it multiplies (no copies across lanes),
// which keeps the kernel within 96 registers: five waves per SIMD.
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

// One wave's scratch.  The observation and the first pooled map carry a
// border of zeros (the convolutions' padding), so every tap reads at a fixed
// offset from the lane's base with no bounds test.
constexpr int kOb = kWin + 2;    // 17: bordered observation edge
constexpr int kPb = kP1 + 2;     // 9: bordered pool1 edge
constexpr int kW2N = kLwi - kC2w;   // conv2 kernel and bias: 296 floats
struct alignas(16) WaveLds {
    float w2s[kW2N + 24];        // conv2 kernel [tap][co][ci] and bias, staged for the channel-per-lane reads
    float tab[9][5][4];          // conv1: weight sum of each channel combination per tap
    float p1[kPb * kPb][kF1];
    union {
        float a1[kO1 * kO1][kF1];   // conv1 output, dead after pool1
        struct {
            float a2[kO2 * kO2][kF2];
            float emb[84];          // embedding (78), then the new h (4)
            float y8[kD];
        } late;
    } u;
    uint8_t obs[kOb * kOb + 3];  // pixel bits: 1 resource, 2 agent, 4 wall (0 on the border)
    uint8_t extra[kOb * kOb + 3];   // agents on the pixel beyond the first (paper dynamics; 0 on the border)
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

// Logistic function and tanh from the hardware exp2 and reciprocal (about one
// ulp each; absolute error near 1e-7).
__device__ __forceinline__ float sigm(float v) {
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(v * -1.44269504f));
}
__device__ __forceinline__ float tanh_(float v) { return fmaf(2.0f, sigm(2.0f * v), -1.0f); }

__device__ __forceinline__ void pinf(float v) { asm volatile("" ::"v"(v)); }
__device__ __forceinline__ void pin4(float4 v) {
    asm volatile("" ::"v"(v.x), "v"(v.y), "v"(v.z), "v"(v.w));
}

// Sum over the lanes that differ in lane bits lo..5 of a 4-vector, spread
// over those lanes: after the call each lane holds one component, component
// (2 bit_lo + bit_lo+1) of the total.  Two exchanges split the vector, the
// remaining bits are summed with one exchange each.
template <int LO>
__device__ __forceinline__ float reduce_scatter4(float4 v, int lane) {
    const bool b0 = (lane >> LO) & 1;
    float k0 = b0 ? v.z : v.x, k1 = b0 ? v.w : v.y;       // kept: components 2 b0, 2 b0 + 1
    const float s0 = b0 ? v.x : v.z, s1 = b0 ? v.y : v.w;  // sent to the partner
    k0 += __shfl_xor(s0, 1 << LO);
    k1 += __shfl_xor(s1, 1 << LO);
    const bool b1 = (lane >> (LO + 1)) & 1;
    float k = b1 ? k1 : k0;
    k += __shfl_xor(b1 ? k0 : k1, 1 << (LO + 1));
#pragma unroll
    for (int off = 1 << (LO + 2); off < 64; off <<= 1) k += __shfl_xor(k, off);
    return k;
}

// `rv`, `rv2`: the agent's record (slot, cell, energy, uid / age, streak,
// previous action, ate); every field is the same in all lanes.  PAPER: the
// world runs the paper's dynamics (agents stack: the agent channel counts
// them); a compile-time choice, so the other rules pay nothing for it.
template <bool PAPER>
__device__ __forceinline__ void act_agent(DevRef d, AgentRec* recp, int4 rv, int4 rv2, int li, int64_t t, int lane,
                                          WaveLds& L) {
    const int H = d.H, W = d.W;
    const int slot = __builtin_amdgcn_readfirstlane(rv.x);
    const int cell = __builtin_amdgcn_readfirstlane(rv.y);
    const uint32_t u = uint32_t(__builtin_amdgcn_readfirstlane(rv.w));
    const int prev = __builtin_amdgcn_readfirstlane(rv2.z);
    const int ate = __builtin_amdgcn_readfirstlane(rv2.w);
    const int r = cell / W;
    const int c = cell - r * W;
    const float* th = d.theta + size_t(slot) * size_t(d.Ppad);
    const float* hs = d.h + size_t(slot) * kState;
    const uint8_t* R = d.R[t & 1];

    // ---- one round trip: observation, state and every weight --------------
    // (the bounds test with bitwise ands and the raw words kept until the
    // loads complete below: a short-circuit test let the compiler put each
    // pixel's loads in a branch of its own, which waited for them there, four
    // round trips instead of one)
    int rbv[4], obv[4];
    bool inm[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int q = lane + 64 * m;
        const int iy = q / kWin, ix = q - (q / kWin) * kWin;
        const int rr = r + iy - kRho, cc = c + ix - kRho;
        const bool in = (q < kPix) & (rr >= 0) & (rr < H) & (cc >= 0) & (cc < W);
        const uint32_t qc = uint32_t(in ? rr * W + cc : cell);   // every lane loads (clamped)
        rbv[m] = R[qc];
        obv[m] = d.occA[qc];
        inm[m] = in;
    }
    // conv1 weights of tap lane / 4, output channel lane % 4 (lanes < 36)
    const int l36 = min(lane, 35);
    const uint32_t o1 = uint32_t(kC1w + (l36 >> 2) * 3 * kF1 + (l36 & 3));
    const float w1r = th[o1];
    const float w1a = th[o1 + kF1];
    const float w1w = th[o1 + 2 * kF1];
    const float4 b1 = *reinterpret_cast<const float4*>(th + kC1b);
    // conv2 kernel and bias: five coalesced words per lane, staged in LDS
    // (each lane later needs the 36 weights of one channel, strided)
    const int co2 = lane & 7;
    float w2raw[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) w2raw[j] = th[uint32_t(kC2w + min(j * 64 + lane, kW2N - 1))];
    // LSTM: rows ig + 16 m of the input kernel, gate gq = lane % 4; after the
    // reduction this lane owns unit uk of gate gq
    const int ig = lane >> 2, gq = lane & 3;
    const int uk = 2 * ((lane >> 2) & 1) + ((lane >> 3) & 1);
    float4 wi[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        const int i = min(ig + 16 * m, kEmb - 1);
        wi[m] = *reinterpret_cast<const float4*>(th + uint32_t(kLwi + i * 16 + gq * 4));
    }
    // recurrent term: lane takes unit j = lane / 16 of h and its weight to
    // (gate gq, unit uk); the four lanes of one (gq, uk) differ in j
    const int jr = lane >> 4;
    const float hj = hs[uint32_t(jr)];
    const float whj = th[uint32_t(kLwh + jr * 16 + gq * 4 + uk)];
    const float lbk = th[uint32_t(kLb + gq * 4 + uk)];
    const float ck = hs[uint32_t(kHd + uk)];                      // c of unit uk
    // dense 8: rows ig8 + 32 m, outputs 4 hf .. 4 hf + 3; after the reduction
    // this lane owns output o8
    const int ig8 = lane >> 1, hf = lane & 1;
    const int o8 = 4 * hf + 2 * ((lane >> 1) & 1) + ((lane >> 2) & 1);
    float4 w8[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const int i = min(ig8 + 32 * m, kCat - 1);
        w8[m] = *reinterpret_cast<const float4*>(th + uint32_t(kD8w + i * kD + hf * 4));
    }
    const float b8 = th[uint32_t(kD8b + o8)];
    // head: lane = (action lane / 8, input lane % 8) for lanes < 40, one
    // weight each; bias of action `lane` on lanes < 5
    const int o5 = lane & 7;
    const float w5j = th[uint32_t(kD5w + o5 * kNA + min(lane >> 3, kNA - 1))];
    const float b5 = th[uint32_t(kD5b + min(lane, kNA - 1))];
    // complete the loads here, so that none is moved into a branch that uses
    // it (which would add a dependent round trip)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        pin(rbv[m]);
        pin(obv[m]);
    }
    int pb[4], px[4];
    constexpr bool paper = PAPER;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        pb[m] = inm[m] ? ((rbv[m] != 0 ? 1 : 0) | (obv[m] != -1 ? 2 : 0)) : 4;
        // under the paper's dynamics occA holds the agents on the cell minus one
        px[m] = (paper && inm[m] && obv[m] > 0) ? min(obv[m], 255) : 0;
    }
    pinf(w1r);
    pinf(w1a);
    pinf(w1w);
    pinf(ck);

    // ---- observation bits (bordered) and the conv1 table into LDS ----------
    // (pixels past the window carry only the wall bit)
    const bool seen = __ballot(((pb[0] | pb[1] | pb[2] | pb[3]) & 1) != 0) != 0;   // a resource in view
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int q = lane + 64 * m;
        if (q < kPix) {
            const int o = (q / kWin + 1) * kOb + (q - (q / kWin) * kWin) + 1;
            L.obs[o] = uint8_t(pb[m]);
            if constexpr (PAPER) L.extra[o] = uint8_t(px[m]);
        }
    }
    {
        // the 64 border pixels, one per lane: top row, bottom row, left and
        // right columns
        int by, bx;
        if (lane < kOb) { by = 0; bx = lane; }
        else if (lane < 2 * kOb) { by = kOb - 1; bx = lane - kOb; }
        else if (lane < 2 * kOb + kWin) { by = lane - 2 * kOb + 1; bx = 0; }
        else { by = lane - 2 * kOb - kWin + 1; bx = kOb - 1; }
        L.obs[by * kOb + bx] = 0;
        if constexpr (PAPER) L.extra[by * kOb + bx] = 0;
    }
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        // kernel word (tap, ci, co) to [tap][co][ci]: one float4 per tap and
        // output channel; the bias stays behind the kernel
        const int gi = j * 64 + lane;
        const int tap = gi >> 5, ci = (gi >> 3) & 3, co = gi & 7;
        if (gi < kC2b - kC2w) L.w2s[tap * 32 + co * 4 + ci] = w2raw[j];
        else if (gi < kW2N) L.w2s[gi] = w2raw[j];
    }
    if (lane < 36) {
        float* tp = &L.tab[lane >> 2][0][lane & 3];
        tp[0 * 4] = 0.f;
        tp[1 * 4] = w1r;
        tp[2 * 4] = w1a;
        tp[3 * 4] = w1r + w1a;
        tp[4 * 4] = w1w;
    }
    if (lane < 4 * kPb - 4) {   // zero border of the pooled map
        int by, bx;
        if (lane < kPb) { by = 0; bx = lane; }
        else if (lane < 2 * kPb) { by = kPb - 1; bx = lane - kPb; }
        else if (lane < 2 * kPb + kP1) { by = lane - 2 * kPb + 1; bx = 0; }
        else { by = lane - 2 * kPb - kP1 + 1; bx = kPb - 1; }
        *reinterpret_cast<float4*>(&L.p1[by * kPb + bx][0]) = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    wave_lds_sync();

    // ---- conv1: lane = output pixel ------------------------------------------
    {
        const int oy = lane >> 3, ox = lane & 7;
        const uint8_t* ob = &L.obs[(2 * oy) * kOb + 2 * ox];
        float4 acc = b1;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int bits = ob[ky * kOb + kx];
                acc = add4(acc, *reinterpret_cast<const float4*>(&L.tab[ky * 3 + kx][bits][0]));
            }
        if constexpr (PAPER) {   // stacked agents: the agent channel holds their number
            const uint8_t* ex = &L.extra[(2 * oy) * kOb + 2 * ox];
#pragma unroll
            for (int ky = 0; ky < 3; ++ky)
#pragma unroll
                for (int kx = 0; kx < 3; ++kx)
                    acc = fma4(float(ex[ky * kOb + kx]), *reinterpret_cast<const float4*>(&L.tab[ky * 3 + kx][2][0]),
                               acc);
        }
        *reinterpret_cast<float4*>(&L.u.a1[lane][0]) = acc;
    }
    wave_lds_sync();

    // ---- pool1: lane = pooled pixel ------------------------------------------
    if (lane < kP1 * kP1) {
        const int y = lane / kP1, x = lane - (lane / kP1) * kP1;
        const float4 v00 = *reinterpret_cast<const float4*>(&L.u.a1[y * kO1 + x][0]);
        const float4 v01 = *reinterpret_cast<const float4*>(&L.u.a1[y * kO1 + x + 1][0]);
        const float4 v10 = *reinterpret_cast<const float4*>(&L.u.a1[(y + 1) * kO1 + x][0]);
        const float4 v11 = *reinterpret_cast<const float4*>(&L.u.a1[(y + 1) * kO1 + x + 1][0]);
        const float4 s = add4(add4(add4(v00, v01), v10), v11);
        *reinterpret_cast<float4*>(&L.p1[(y + 1) * kPb + x + 1][0]) =
            make_float4(s.x * 0.25f, s.y * 0.25f, s.z * 0.25f, s.w * 0.25f);
    }
    wave_lds_sync();

    // ---- conv2: lane = (channel lane % 8, pixels lane / 8 and lane / 8 + 8) --
    // the 4 weights of a tap and the lane's channel are one float4 read from
    // LDS, shared by the lane's two pixels
    {
        const float b2 = L.w2s[kC2b - kC2w + co2];
        const int p0 = lane >> 3, p1 = p0 + 8;
        const float4* pp0 = reinterpret_cast<const float4*>(&L.p1[(2 * (p0 >> 2)) * kPb + 2 * (p0 & 3)][0]);
        const float4* pp1 = reinterpret_cast<const float4*>(&L.p1[(2 * (p1 >> 2)) * kPb + 2 * (p1 & 3)][0]);
        const float4* wt = reinterpret_cast<const float4*>(&L.w2s[co2 * 4]);
        float acc0 = 0.f, acc1 = 0.f;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const float4 w = wt[(ky * 3 + kx) * kF2];
                const float4 v0 = pp0[ky * kPb + kx];
                const float4 v1 = pp1[ky * kPb + kx];
                acc0 = fmaf(v0.x, w.x, acc0);
                acc0 = fmaf(v0.y, w.y, acc0);
                acc0 = fmaf(v0.z, w.z, acc0);
                acc0 = fmaf(v0.w, w.w, acc0);
                acc1 = fmaf(v1.x, w.x, acc1);
                acc1 = fmaf(v1.y, w.y, acc1);
                acc1 = fmaf(v1.z, w.z, acc1);
                acc1 = fmaf(v1.w, w.w, acc1);
            }
        L.u.late.a2[p0][co2] = acc0 + b2;
        L.u.late.a2[p1][co2] = acc1 + b2;
    }
    wave_lds_sync();

    // ---- pool2 into the embedding, then the previous action and ate bit -----
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int f = lane + 64 * m;   // (y, x, channel) = (f / 24, f / 8 % 3, f % 8)
        if (f < kFlat) {
            const int y = f / 24, x = (f >> 3) % 3, ch = f & 7;
            const float(*a2)[kF2] = L.u.late.a2;
            const float s = ((a2[y * kO2 + x][ch] + a2[y * kO2 + x + 1][ch]) + a2[(y + 1) * kO2 + x][ch]) +
                            a2[(y + 1) * kO2 + x + 1][ch];
            L.u.late.emb[f] = s * 0.25f;
        }
    }
    if (lane < kNA) L.u.late.emb[kFlat + lane] = (prev == lane) ? 1.f : 0.f;
    if (lane == kNA) L.u.late.emb[kFlat + kNA] = ate ? 1.f : 0.f;
    wave_lds_sync();

    // ---- LSTM: lane = (input group, gate), then (unit uk, gate gq) ----------
    float hnew, cnew;
    {
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            const int i = ig + 16 * m;
            const float e = i < kEmb ? L.u.late.emb[min(i, kEmb - 1)] : 0.f;
            acc = fma4(e, wi[m], acc);
        }
        float z = reduce_scatter4<2>(acc, lane);
        float rec = hj * whj;
        rec += __shfl_xor(rec, 16);
        rec += __shfl_xor(rec, 32);
        z = (z + rec) + lbk;
        // the four gates of unit uk sit in the lane's quad (gq = 0..3)
        const int q0 = lane & ~3;
        const float zi = __shfl(z, q0 + 0), zf = __shfl(z, q0 + 1), zg = __shfl(z, q0 + 2), zo = __shfl(z, q0 + 3);
        cnew = fmaf(sigm(zf), ck, sigm(zi) * tanh_(zg));
        hnew = sigm(zo) * tanh_(cnew);
        if (lane < 16 && gq == 0) L.u.late.emb[kEmb + uk] = hnew;
    }
    wave_lds_sync();

    // ---- dense 8 with tanh: lane = (input group, half of the outputs) ------
    {
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int i = ig8 + 32 * m;
            const float e = i < kCat ? L.u.late.emb[min(i, kCat - 1)] : 0.f;
            acc = fma4(e, w8[m], acc);
        }
        const float y = tanh_(reduce_scatter4<1>(acc, lane) + b8);
        if (lane < 8) L.u.late.y8[o8] = y;
    }
    wave_lds_sync();

    // ---- logits (lane a < 5) and the sampled action -----------------------------
    float pl = L.u.late.y8[o5] * w5j;
    pl += __shfl_xor(pl, 1);
    pl += __shfl_xor(pl, 2);
    pl += __shfl_xor(pl, 4);
    const float lg = __shfl(pl, min(lane, kNA - 1) * 8) + b5;   // lanes < 5: logit of action `lane`
    // sampling score 50 l + g, g from word a % 4 of ACT block a / 4 (the
    // draws depend on the agent and the step only: scalar)
    const Draw4 d0 = philox(u, uint32_t(t), kAct, 0u, d.seed_lo, d.seed_hi);
    const Draw4 d1 = philox(u, uint32_t(t), kAct, 1u, d.seed_lo, d.seed_hi);
    const uint32_t word = lane == 0 ? d0.x : (lane == 1 ? d0.y : (lane == 2 ? d0.z : (lane == 3 ? d0.w : d1.x)));
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
    if (d.forced_on) best = forced_of(d, u, best);

    // ---- outputs ----------------------------------------------------------------
    if (lane < 16 && gq == 0) {
        d.h[size_t(slot) * kState + uk] = hnew;
        d.h[size_t(slot) * kState + kHd + uk] = cnew;
    }
    if (lane == 0 && t % kMoveWin == 0) {   // a movement window starts with this step
        d.wcell[slot] = cell;
        d.wuid[slot] = u;
    }
    if (lane == 0) {
        d.action[slot] = uint8_t(best);
        recp->action = best | (seen ? kSeenBit : 0);
        // the claim on the target cell: its observed pixel (no agent and no
        // wall = free)
        const int bits = L.obs[(kRho + 1 + act_dr(best)) * kOb + (kRho + 1 + act_dc(best))];
        act_claim(d, best, r, c, u, t, (bits & 6) == 0, (bits & 1) != 0);
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
