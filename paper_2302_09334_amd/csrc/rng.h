// rng.h -- counter-based random numbers of the world step (host + device).
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11) keyed by the world seed; the counter is
// (entity, step, stream, block) so every draw is addressed, not sequenced,
// and any thread can produce any draw without coordination.
//
// Normal deviates use Box-Muller in single precision.  The logarithm and the
// sine/cosine are evaluated from their series with explicit fma/rounding
// points so that every IEEE-conforming implementation of the same operations
// produces the same bits (the paper specifies N(0, sigma) mutation, App. B.3,
// but not the sampler).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eco {

enum : uint32_t {
    kInitRes = 1,
    kInitPlace = 2,
    kInitW = 3,
    kMove = 4,
    kBirth = 5,
    kMutate = 6,
    kRegrow = 7,
    kAct = 8,   // action sampling of the paper's network
    kEat = 9,   // eater of a shared resource cell under the paper's dynamics
};

struct Draw4 {
    uint32_t x, y, z, w;
};

__host__ __device__ inline Draw4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t m0 = uint64_t(0xD2511F53u) * c0;
        const uint64_t m1 = uint64_t(0xCD9E8D57u) * c2;
        const uint32_t y0 = uint32_t(m1 >> 32) ^ c1 ^ k0;
        const uint32_t y2 = uint32_t(m0 >> 32) ^ c3 ^ k1;
        c0 = y0;
        c1 = uint32_t(m1);
        c2 = y2;
        c3 = uint32_t(m0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Draw4{c0, c1, c2, c3};
}

// ln(m 2^e) for m in [sqrt(1/2), sqrt(2)).  With f = m - 1 (exact) and
// s = f / (2 + f), ln m = 2 atanh(s) = 2s + 2s^3/3 + ...; as 2s = f - s f this
// equals f - (f^2/2 - s (f^2/2 + R)) with R = 2s^2/3 + 2s^4/5 + ... + 2s^10/11:
// the leading term f carries no rounding and only the small correction does
// (at most 0.84 ulp over all floats in [2^-24, 17]).  ln 2 is split into a
// head whose products with e are exact and a tail.
__host__ __device__ inline float ln_of_split(float m, int e) {
    const float f = m - 1.0f;
    const float s = f / (2.0f + f);
    const float z = s * s;
    float R = 2.0f / 11.0f;
    R = fmaf(R, z, 2.0f / 9.0f);
    R = fmaf(R, z, 2.0f / 7.0f);
    R = fmaf(R, z, 2.0f / 5.0f);
    R = fmaf(R, z, 2.0f / 3.0f);
    R = R * z;
    const float hf2 = (0.5f * f) * f;
    const float ef = float(e);
    const float tail = fmaf(s, hf2 + R, ef * 0x1.7f7d1cp-20f);
    const float corr = hf2 - tail;
    return fmaf(ef, 0x1.62e4p-1f, f - corr);
}

// ln(v * 2^-24) for an integer v in [1, 2^24]: the mantissa/exponent split is
// taken from the bit length of v (exact), the mantissa folded into
// [sqrt(1/2), sqrt(2)).
__host__ __device__ inline float ln_of_24bit(uint32_t v) {
#if defined(__HIP_DEVICE_COMPILE__)
    const int bits = 32 - __clz(v);
#else
    const int bits = 32 - __builtin_clz(v);
#endif
    int e = bits - 24;
    float m = ldexpf(float(v), -bits);  // exact, in [0.5, 1)
    if (m < 0x1.6a09e6p-1f) {
        m = m * 2.0f;
        e -= 1;
    }
    return ln_of_split(m, e);
}

// ln(x) for a positive normal float x: the same fold, with the exponent read
// from the float's bits.
__host__ __device__ inline float ln_positive(float x) {
    const uint32_t b = __builtin_bit_cast(uint32_t, x);
    int e = int((b >> 23) & 0xFFu) - 126;
    float m = __builtin_bit_cast(float, (b & 0x807FFFFFu) | 0x3F000000u);  // exact, in [0.5, 1)
    if (m < 0x1.6a09e6p-1f) {
        m = m * 2.0f;
        e -= 1;
    }
    return ln_of_split(m, e);
}

// Standard Gumbel deviate -ln(-ln u) from a 32-bit word, u = (2 j + 1) 2^-24
// with j the word's top 23 bits (u in [2^-24, 1 - 2^-24], exact).
__host__ __device__ inline float gumbel_of_word(uint32_t w) {
    const float ex = -ln_of_24bit(((w >> 9) << 1) | 1u);   // -ln u > 0
    return -ln_positive(ex);
}

// sin((pi/2) g) and cos((pi/2) g) for g in [0, 1/2] from their Taylor series.
__host__ __device__ inline float quarter_sin(float g) {
    const float x = g * 0x1.921fb6p+0f;
    const float x2 = x * x;
    float p = 1.0f / 362880.0f;
    p = fmaf(p, x2, -1.0f / 5040.0f);
    p = fmaf(p, x2, 1.0f / 120.0f);
    p = fmaf(p, x2, -1.0f / 6.0f);
    return fmaf(x2 * x, p, x);
}

__host__ __device__ inline float quarter_cos(float g) {
    const float x = g * 0x1.921fb6p+0f;
    const float x2 = x * x;
    float p = -1.0f / 3628800.0f;
    p = fmaf(p, x2, 1.0f / 40320.0f);
    p = fmaf(p, x2, -1.0f / 720.0f);
    p = fmaf(p, x2, 1.0f / 24.0f);
    p = fmaf(p, x2, -1.0f / 2.0f);
    return fmaf(x2, p, 1.0f);
}

__host__ __device__ inline float negate_if(float v, uint32_t neg) {
    return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v) ^ (neg << 31));
}

// Two standard normals from two 32-bit words: u1 = ((a >> 8) + 1) 2^-24,
// u2 = (b >> 8) 2^-24, z0 = sqrt(-2 ln u1) cos(2 pi u2), z1 = ... sin.
// The angle 2 pi u2 = (pi/2)(q + f) is split exactly into a quadrant q and a
// fraction f; fractions above 1/2 use the complementary quarter angle.  The
// quadrant rotation is written with selects and sign-bit flips only (no
// divergent branches), which keeps the generated code a straight line.
__host__ __device__ inline void box_muller(uint32_t a, uint32_t b, float& z0, float& z1) {
    const float r = sqrtf(-2.0f * ln_of_24bit((a >> 8) + 1u));
    const uint32_t k = b >> 8;         // 24 bits
    const uint32_t q = k >> 22;        // quadrant
    const float f = float(k & 0x3FFFFFu) * 0x1p-22f;  // exact, [0, 1)
    const bool fold = f > 0.5f;
    const float g = fold ? 1.0f - f : f;               // exact
    const float qs = quarter_sin(g);
    const float qc = quarter_cos(g);
    const float sf = fold ? qc : qs;   // sin((pi/2) f)
    const float cf = fold ? qs : qc;   // cos((pi/2) f)
    // rotate by q quarter turns: (s, c) = (sf, cf), (cf, -sf), (-sf, -cf), (-cf, sf)
    const bool odd = (q & 1u) != 0;
    const float s = negate_if(odd ? cf : sf, (q >> 1) & 1u);
    const float c = negate_if(odd ? sf : cf, ((q + 1u) >> 1) & 1u);
    z0 = r * c;
    z1 = r * s;
}

}  // namespace eco
