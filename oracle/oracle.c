/*
 * oracle.c -- plain CPU reference of the world step of the non-episodic
 * neuroevolution simulator of arXiv 2302.09334.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product library.
 *
 * Sources followed, by section of the paper:
 *   App. B.1, Eq. (1)  resource regrowth p = p_I * c(x) + c, in the
 *                      parameterisation of the benchmark workloads: p_I is the
 *                      count of resources in the 24-cell (Chebyshev radius 2)
 *                      neighbourhood divided by 24, c(x) a rate linear in the
 *                      row, c a small constant.
 *   App. B.2           agents: local square observation window, five actions
 *                      (stay, up, down, right, left), a recurrent controller
 *                      with individual weights, energy that decays each step
 *                      and increases when a resource is eaten.
 *   App. B.3           minimal-criterion reproduction (energy held above a
 *                      threshold for a number of steps), Gaussian mutation of
 *                      the parent's weights, death by energy or by age.
 *   App. B.4 / B.5     hyperparameters and architecture (here: a GRU cell with
 *                      a linear head, as the benchmark workloads specify).
 * Where the paper is silent (randomness, ordering, tie-breaking, boundaries)
 * the readings are stated next to the code that implements them.
 *
 * Build: cc -O2 -std=c11 -ffp-contract=off -fPIC -shared oracle.c -lm
 * No fast-math, no contraction: every floating-point operation that decides an
 * integer is written out with explicit rounding points.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ========================================================================= */
/* Counter-based generator: Philox4x32-10 (Salmon et al., SC'11).            */
/* ========================================================================= */

static void philox_block(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                         uint32_t k0, uint32_t k1, uint32_t out[4])
{
    /* Ten rounds; the key is bumped by the Weyl constants between rounds. */
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void oracle_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        philox_block(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3],
                     key[0], key[1], out + 4 * i);
}

/* Draw of the world's generator: counter = (entity, step, stream, block),
 * key = the 64-bit seed split into its low and high words. */
static void draw(uint64_t seed, uint32_t entity, uint32_t step, uint32_t stream,
                 uint32_t block, uint32_t out[4])
{
    philox_block(entity, step, stream, block, (uint32_t)seed, (uint32_t)(seed >> 32), out);
}

/* ========================================================================= */
/* Standard normal deviates.  The paper draws mutations from N(0, sigma)     */
/* without saying how; this reading fixes Box-Muller in single precision     */
/* with a logarithm and a sine/cosine written out from their series, so that */
/* any implementation performing the same IEEE operations gets the same bits.*/
/* ========================================================================= */

/* ln(u) for a positive normal float u (the uniforms of Box-Muller, and the
 * exponential deviate inside a Gumbel draw).  u = m * 2^e with m in
 * [sqrt(1/2), sqrt(2)) and f = m - 1, which is exact.  For s = f / (2 + f),
 * ln m = ln((1 + s) / (1 - s)) = 2 (s + s^3/3 + s^5/5 + ...).  Because
 * s (2 + f) = f, the leading 2s equals f - s f, and
 *     ln m = f - (f^2/2 - s (f^2/2 + R)),  R = 2 s^2/3 + 2 s^4/5 + ... + 2 s^10/11,
 * which keeps the large term f free of rounding.  ln 2 is split into a head
 * whose products with e are exact and a tail. */
static float ln_unit(float u)
{
    int e;
    float m = frexpf(u, &e);                 /* u = m * 2^e, m in [0.5, 1) */
    if (m < 0x1.6a09e6p-1f) {
        m = m * 2.0f;
        e = e - 1;
    }
    float f = m - 1.0f;
    float s = f / (2.0f + f);
    float s2 = s * s;
    float r = 2.0f / 11.0f;                  /* R / s^2 by Horner in s^2 */
    r = fmaf(r, s2, 2.0f / 9.0f);
    r = fmaf(r, s2, 2.0f / 7.0f);
    r = fmaf(r, s2, 2.0f / 5.0f);
    r = fmaf(r, s2, 2.0f / 3.0f);
    float R = r * s2;
    float half_f2 = (0.5f * f) * f;
    float ef = (float)e;
    float small = fmaf(s, half_f2 + R, ef * 0x1.7f7d1cp-20f);   /* + e * (ln 2 tail) */
    float corr = half_f2 - small;
    return fmaf(ef, 0x1.62e4p-1f, f - corr);
}

/* sin and cos of (pi/2) * g for g in [0, 1/2], from the Taylor series. */
static float sin_quarter(float g)
{
    float x = g * 0x1.921fb6p+0f;            /* (pi/2) * g */
    float x2 = x * x;
    float p = 1.0f / 362880.0f;
    p = fmaf(p, x2, -1.0f / 5040.0f);
    p = fmaf(p, x2, 1.0f / 120.0f);
    p = fmaf(p, x2, -1.0f / 6.0f);
    float x3 = x2 * x;
    return fmaf(x3, p, x);
}

static float cos_quarter(float g)
{
    float x = g * 0x1.921fb6p+0f;
    float x2 = x * x;
    float p = -1.0f / 3628800.0f;
    p = fmaf(p, x2, 1.0f / 40320.0f);
    p = fmaf(p, x2, -1.0f / 720.0f);
    p = fmaf(p, x2, 1.0f / 24.0f);
    p = fmaf(p, x2, -1.0f / 2.0f);
    return fmaf(x2, p, 1.0f);
}

/* sin(2 pi u), cos(2 pi u) for dyadic u in [0, 1): the quadrant is split off
 * exactly, the remaining quarter turn is folded to [0, pi/4]. */
static void sincos_2pi(float u, float *s_out, float *c_out)
{
    float t = u * 4.0f;                      /* exact */
    int q = (int)t;                          /* quadrant 0..3 */
    float f = t - (float)q;                  /* exact, in [0, 1) */
    float sf, cf;                            /* sin, cos of (pi/2) f */
    if (f > 0.5f) {
        float g = 1.0f - f;                  /* exact */
        sf = cos_quarter(g);
        cf = sin_quarter(g);
    } else {
        sf = sin_quarter(f);
        cf = cos_quarter(f);
    }
    switch (q) {
    case 0: *s_out = sf;  *c_out = cf;  break;
    case 1: *s_out = cf;  *c_out = -sf; break;
    case 2: *s_out = -sf; *c_out = -cf; break;
    default: *s_out = -cf; *c_out = sf; break;
    }
}

/* Two normals from two words: u1 = ((a >> 8) + 1) 2^-24 in (0, 1],
 * u2 = (b >> 8) 2^-24 in [0, 1); z0 = r cos(2 pi u2), z1 = r sin(2 pi u2),
 * r = sqrt(-2 ln u1). */
static void gauss_pair(uint32_t a, uint32_t b, float *z0, float *z1)
{
    float u1 = (float)((a >> 8) + 1u) * 0x1p-24f;
    float u2 = (float)(b >> 8) * 0x1p-24f;
    float r = sqrtf(-2.0f * ln_unit(u1));
    float s, c;
    sincos_2pi(u2, &s, &c);
    *z0 = r * c;
    *z1 = r * s;
}

void oracle_ln_unit(const float *u, float *out, size_t n)
{
    for (size_t i = 0; i < n; ++i) out[i] = ln_unit(u[i]);
}

void oracle_sincos_2pi(const float *u, float *s, float *c, size_t n)
{
    for (size_t i = 0; i < n; ++i) sincos_2pi(u[i], &s[i], &c[i]);
}

void oracle_gauss_pair(const uint32_t *a, const uint32_t *b, float *z0, float *z1, size_t n)
{
    for (size_t i = 0; i < n; ++i) gauss_pair(a[i], b[i], &z0[i], &z1[i]);
}

/* Four normals from one generator block: (x, y) -> z0, z1 and (z, w) -> z2, z3. */
static void gauss_block(const uint32_t r[4], float z[4])
{
    gauss_pair(r[0], r[1], &z[0], &z[1]);
    gauss_pair(r[2], r[3], &z[2], &z[3]);
}

/* ========================================================================= */
/* Genome layout.  The paper fixes no parameter order; this reading numbers  */
/* the GRU and head parameters as follows (the order also keys the random    */
/* draws of initialisation and mutation):                                    */
/*   W_ih[i][k][g]  input i -> gate g of hidden unit k   (in x Hd x 3)       */
/*   W_hh[j][k][g]  hidden j -> gate g of hidden unit k  (Hd x Hd x 3)       */
/*   b_ih[k][g], b_hh[k][g]                              (Hd x 3 each)       */
/*   W_o[a][k]      hidden k -> logit a                  (5 x Hd)            */
/*   b_o[a]                                              (5)                 */
/* with gates g = 0 (reset r), 1 (update z), 2 (candidate n).                */
/* ========================================================================= */

int32_t oracle_n_inputs(int32_t rho)
{
    int32_t w = 2 * rho + 1;
    return 2 * w * w + 1;
}

typedef struct {
    int32_t n_in, hd;
    int32_t ih, hh, bih, bhh, wo, bo, P;
} genome_layout;

static genome_layout layout_of(int32_t n_in, int32_t hd)
{
    genome_layout g;
    g.n_in = n_in;
    g.hd = hd;
    g.ih = 0;
    g.hh = g.ih + n_in * hd * 3;
    g.bih = g.hh + hd * hd * 3;
    g.bhh = g.bih + hd * 3;
    g.wo = g.bhh + hd * 3;
    g.bo = g.wo + 5 * hd;
    g.P = g.bo + 5;
    return g;
}

int32_t oracle_n_params(int32_t rho, int32_t hd)
{
    return layout_of(oracle_n_inputs(rho), hd).P;
}

/* ========================================================================= */
/* The controller: a GRU cell (gates r, z, n as in the usual GRU cell with   */
/* separate input and hidden biases) followed by a linear head to 5 logits.  */
/* Evaluated in double from the single-precision genome and hidden state.    */
/* ========================================================================= */

static double sigmoid(double v) { return 1.0 / (1.0 + exp(-v)); }

void oracle_gru_eval(int32_t n_in, int32_t hd, const float *th, const double *x,
                     const float *h, double *h_out, double *logits)
{
    genome_layout L = layout_of(n_in, hd);
    for (int k = 0; k < hd; ++k) {
        double gi[3], gh[3];
        for (int g = 0; g < 3; ++g) {
            double si = (double)th[L.bih + k * 3 + g];
            for (int i = 0; i < n_in; ++i)
                si += (double)th[L.ih + (i * hd + k) * 3 + g] * x[i];
            double sh = (double)th[L.bhh + k * 3 + g];
            for (int j = 0; j < hd; ++j)
                sh += (double)th[L.hh + (j * hd + k) * 3 + g] * (double)h[j];
            gi[g] = si;
            gh[g] = sh;
        }
        double r = sigmoid(gi[0] + gh[0]);
        double z = sigmoid(gi[1] + gh[1]);
        double n = tanh(gi[2] + r * gh[2]);
        h_out[k] = (1.0 - z) * n + z * (double)h[k];
    }
    for (int a = 0; a < 5; ++a) {
        double s = (double)th[L.bo + a];
        for (int k = 0; k < hd; ++k) s += (double)th[L.wo + a * hd + k] * h_out[k];
        logits[a] = s;
    }
}

/* ========================================================================= */
/* The paper's controller (App. B.5): a two-layer CNN over the 15 x 15 x 3   */
/* observation, an LSTM cell of 4 units, a dense layer of 8 with tanh and a  */
/* dense layer of 5 action logits.  Readings where the text is open:         */
/*  - each convolution pads its input with zeros on both sides as needed for */
/*    ceil(n / stride) outputs ("SAME"); each pooling keeps only full        */
/*    windows ("VALID"); no nonlinearity follows a convolution (none is      */
/*    named); the flattened feature order is (row, column, channel);         */
/*  - the embedding is [CNN features, one-hot of the previous action (all    */
/*    zero before the agent's first action), 1 if the agent ate in its       */
/*    previous step]; the LSTM's input kernel has no bias, its hidden kernel */
/*    has one; gates in the order i, f, g, o; state (h, c) zero at birth;    */
/*  - the dense layer of 8 reads [embedding, new h].                         */
/* These readings give exactly the 2445 parameters the paper states.         */
/* Genome order (also the key of the initial and mutation draws):            */
/*   conv1 K[ky][kx][ci][co], conv1 b[co], conv2 K[ky][kx][ci][co], conv2 b, */
/*   LSTM Wi[i][gate][unit], Wh[j][gate][unit], b[gate][unit],               */
/*   dense8 W[i][o], b[o], dense5 W[o][a], b[a].                              */
/* ========================================================================= */

enum { CNN_RHO = 7, CNN_HD = 4, CNN_CH = 3, CNN_F1 = 4, CNN_F2 = 8, CNN_K = 3, CNN_S = 2, CNN_POOL = 2,
       CNN_D = 8, CNN_NA = 5 };

typedef struct {
    int32_t win;                 /* observation edge                              */
    int32_t o1, pad1, p1;        /* conv1 output edge, its low padding, pool1 edge */
    int32_t o2, pad2, p2;        /* conv2 output edge, its low padding, pool2 edge */
    int32_t flat, emb, cat;      /* CNN features, LSTM input, dense-8 input        */
    int32_t c1w, c1b, c2w, c2b, lwi, lwh, lb, d8w, d8b, d5w, d5b, P;
} cnn_layout;

/* Output edge of a SAME convolution and its low-side padding. */
static void same_conv(int32_t n, int32_t *out, int32_t *pad_lo)
{
    int32_t o = (n + CNN_S - 1) / CNN_S;
    int32_t total = (o - 1) * CNN_S + CNN_K - n;
    if (total < 0) total = 0;
    *out = o;
    *pad_lo = total / 2;
}

static cnn_layout cnn_layout_of(void)
{
    cnn_layout L;
    L.win = 2 * CNN_RHO + 1;
    same_conv(L.win, &L.o1, &L.pad1);
    L.p1 = L.o1 - CNN_POOL + 1;
    same_conv(L.p1, &L.o2, &L.pad2);
    L.p2 = L.o2 - CNN_POOL + 1;
    L.flat = L.p2 * L.p2 * CNN_F2;
    L.emb = L.flat + CNN_NA + 1;
    L.cat = L.emb + CNN_HD;
    L.c1w = 0;
    L.c1b = L.c1w + CNN_K * CNN_K * CNN_CH * CNN_F1;
    L.c2w = L.c1b + CNN_F1;
    L.c2b = L.c2w + CNN_K * CNN_K * CNN_F1 * CNN_F2;
    L.lwi = L.c2b + CNN_F2;
    L.lwh = L.lwi + L.emb * 4 * CNN_HD;
    L.lb = L.lwh + CNN_HD * 4 * CNN_HD;
    L.d8w = L.lb + 4 * CNN_HD;
    L.d8b = L.d8w + L.cat * CNN_D;
    L.d5w = L.d8b + CNN_D;
    L.d5b = L.d5w + CNN_D * CNN_NA;
    L.P = L.d5b + CNN_NA;
    return L;
}

int32_t oracle_cnn_n_params(void) { return cnn_layout_of().P; }
int32_t oracle_cnn_n_features(void) { return cnn_layout_of().flat; }

/* One evaluation in double.  obs: win x win x 3 (row, column, channel);
 * prev_action in 0..4 or 5 (none); h, c: the 4-unit state (float). */
void oracle_cnn_eval(const float *th, const double *obs, int32_t prev_action, int32_t ate,
                     const float *h, const float *c, double *h_out, double *c_out, double *logits)
{
    cnn_layout L = cnn_layout_of();
    double a1[8 * 8 * CNN_F1], q1[7 * 7 * CNN_F1], a2[4 * 4 * CNN_F2], emb[78], cat[82], y8[CNN_D];
    /* conv1 */
    for (int oy = 0; oy < L.o1; ++oy)
        for (int ox = 0; ox < L.o1; ++ox)
            for (int co = 0; co < CNN_F1; ++co) {
                double s = (double)th[L.c1b + co];
                for (int ky = 0; ky < CNN_K; ++ky)
                    for (int kx = 0; kx < CNN_K; ++kx) {
                        int iy = oy * CNN_S + ky - L.pad1, ix = ox * CNN_S + kx - L.pad1;
                        if (iy < 0 || iy >= L.win || ix < 0 || ix >= L.win) continue;   /* zero padding */
                        for (int ci = 0; ci < CNN_CH; ++ci)
                            s += (double)th[L.c1w + ((ky * CNN_K + kx) * CNN_CH + ci) * CNN_F1 + co] *
                                 obs[(iy * L.win + ix) * CNN_CH + ci];
                    }
                a1[(oy * L.o1 + ox) * CNN_F1 + co] = s;
            }
    /* pool1: mean of each 2 x 2 window, stride 1 */
    for (int y = 0; y < L.p1; ++y)
        for (int x = 0; x < L.p1; ++x)
            for (int ch = 0; ch < CNN_F1; ++ch) {
                double s = 0.0;
                for (int dy = 0; dy < CNN_POOL; ++dy)
                    for (int dx = 0; dx < CNN_POOL; ++dx) s += a1[((y + dy) * L.o1 + x + dx) * CNN_F1 + ch];
                q1[(y * L.p1 + x) * CNN_F1 + ch] = s / (double)(CNN_POOL * CNN_POOL);
            }
    /* conv2 */
    for (int oy = 0; oy < L.o2; ++oy)
        for (int ox = 0; ox < L.o2; ++ox)
            for (int co = 0; co < CNN_F2; ++co) {
                double s = (double)th[L.c2b + co];
                for (int ky = 0; ky < CNN_K; ++ky)
                    for (int kx = 0; kx < CNN_K; ++kx) {
                        int iy = oy * CNN_S + ky - L.pad2, ix = ox * CNN_S + kx - L.pad2;
                        if (iy < 0 || iy >= L.p1 || ix < 0 || ix >= L.p1) continue;
                        for (int ci = 0; ci < CNN_F1; ++ci)
                            s += (double)th[L.c2w + ((ky * CNN_K + kx) * CNN_F1 + ci) * CNN_F2 + co] *
                                 q1[(iy * L.p1 + ix) * CNN_F1 + ci];
                    }
                a2[(oy * L.o2 + ox) * CNN_F2 + co] = s;
            }
    /* pool2, flattened in (row, column, channel) order into the embedding */
    for (int y = 0; y < L.p2; ++y)
        for (int x = 0; x < L.p2; ++x)
            for (int ch = 0; ch < CNN_F2; ++ch) {
                double s = 0.0;
                for (int dy = 0; dy < CNN_POOL; ++dy)
                    for (int dx = 0; dx < CNN_POOL; ++dx) s += a2[((y + dy) * L.o2 + x + dx) * CNN_F2 + ch];
                emb[(y * L.p2 + x) * CNN_F2 + ch] = s / (double)(CNN_POOL * CNN_POOL);
            }
    for (int a = 0; a < CNN_NA; ++a) emb[L.flat + a] = (prev_action == a) ? 1.0 : 0.0;
    emb[L.flat + CNN_NA] = ate ? 1.0 : 0.0;
    /* LSTM cell */
    double z[4][CNN_HD];
    for (int g = 0; g < 4; ++g)
        for (int k = 0; k < CNN_HD; ++k) {
            double s = (double)th[L.lb + g * CNN_HD + k];
            for (int i = 0; i < L.emb; ++i) s += (double)th[L.lwi + (i * 4 + g) * CNN_HD + k] * emb[i];
            for (int j = 0; j < CNN_HD; ++j) s += (double)th[L.lwh + (j * 4 + g) * CNN_HD + k] * (double)h[j];
            z[g][k] = s;
        }
    for (int k = 0; k < CNN_HD; ++k) {
        double ig = sigmoid(z[0][k]), fg = sigmoid(z[1][k]), gg = tanh(z[2][k]), og = sigmoid(z[3][k]);
        c_out[k] = fg * (double)c[k] + ig * gg;
        h_out[k] = og * tanh(c_out[k]);
    }
    /* dense 8 with tanh over [embedding, h'], then the 5 logits */
    for (int i = 0; i < L.emb; ++i) cat[i] = emb[i];
    for (int k = 0; k < CNN_HD; ++k) cat[L.emb + k] = h_out[k];
    for (int o = 0; o < CNN_D; ++o) {
        double s = (double)th[L.d8b + o];
        for (int i = 0; i < L.cat; ++i) s += (double)th[L.d8w + i * CNN_D + o] * cat[i];
        y8[o] = tanh(s);
    }
    for (int a = 0; a < CNN_NA; ++a) {
        double s = (double)th[L.d5b + a];
        for (int o = 0; o < CNN_D; ++o) s += (double)th[L.d5w + o * CNN_NA + a] * y8[o];
        logits[a] = s;
    }
}

/* Action sampling of the paper's controller (App. B.5): a draw from the
 * softmax of the logits at temperature 1/50.  Reading: the Gumbel-max form,
 * arg max_a (50 l_a + g_a) with g_a = -ln(-ln u_a) standard Gumbel, u_a =
 * (2 j + 1) 2^-24 from the top 23 bits j of word a % 4 of block a / 4 of the
 * ACT stream (agent uid, step), in single precision with the logarithm above;
 * lowest index on an exact tie. */
static float gumbel_of_word(uint32_t word)
{
    float u = (float)(((word >> 9) << 1) | 1u) * 0x1p-24f;   /* exact, in [2^-24, 1 - 2^-24] */
    float e = -ln_unit(u);                                     /* exponential(1), > 0 */
    return -ln_unit(e);
}

void oracle_gumbel(const uint32_t *words, float *g, size_t n)
{
    for (size_t i = 0; i < n; ++i) g[i] = gumbel_of_word(words[i]);
}

/* Sampling scores s_a = 50 * l_a + g_a of agent `u` at step `t`. */
static void sample_scores(uint64_t seed, uint32_t u, uint32_t t, const float *lf, float *s)
{
    uint32_t r0[4], r1[4];
    draw(seed, u, t, ORACLE_S_ACT, 0, r0);
    draw(seed, u, t, ORACLE_S_ACT, 1, r1);
    for (int a = 0; a < CNN_NA; ++a) {
        float g = gumbel_of_word(a < 4 ? r0[a] : r1[a - 4]);
        float sc = 50.0f * lf[a];
        s[a] = sc + g;
    }
}

int32_t oracle_sample_action(uint64_t seed, uint32_t uid, uint32_t step, const float *logits, float *scores)
{
    float s[CNN_NA];
    sample_scores(seed, uid, step, logits, s);
    int best = 0;
    for (int a = 1; a < CNN_NA; ++a)
        if (s[a] > s[best]) best = a;
    if (scores) memcpy(scores, s, sizeof(s));
    return best;
}

/* ========================================================================= */
/* Regrowth threshold table (App. B.1, Eq. (1), benchmark parameterisation): */
/*   rate(row) = rate_top + (rate_bottom - rate_top) * row / (H - 1)         */
/*   rate     *= rate_scale                                                  */
/*   p        = rate * n / 24 + spont        (n = resources among the 24)    */
/* A cell grows iff its 32-bit draw is below floor(p * 2^32) (all draws when */
/* p >= 1).  Row 0 is the top (slowest), row H-1 the bottom (fastest).       */
/* ========================================================================= */

static uint64_t prob_threshold(double p)
{
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return (uint64_t)1 << 32;
    return (uint64_t)floor(p * 4294967296.0);
}

int oracle_threshold_table(const oracle_config *cfg, uint64_t *out)
{
    if (cfg->H < 2) return -1;
    if (cfg->dynamics == ORACLE_DYN_PAPER) {
        /* App. B.1, Eq. (1): p = p_I c(x) + c, p_I = regrow_pI when exactly one
         * of the four direct neighbours holds a resource (entry n = that count),
         * c(x) = (alpha^x + 1) / (alpha + 1), x = row / (H - 1): row 0 (top)
         * has the lowest climate value. */
        for (int row = 0; row < cfg->H; ++row) {
            double x = (double)row / (double)(cfg->H - 1);
            double cx = (pow(cfg->regrow_alpha, x) + 1.0) / (cfg->regrow_alpha + 1.0);
            for (int n = 0; n <= 24; ++n) {
                double pI = (n == 1) ? cfg->regrow_pI : 0.0;
                double p = pI * cx + cfg->spont;
                out[row * 25 + n] = prob_threshold(p);
            }
        }
        return 0;
    }
    for (int row = 0; row < cfg->H; ++row) {
        double d = cfg->rate_bottom - cfg->rate_top;
        double a = d * (double)row;
        double b = a / (double)(cfg->H - 1);
        double rate = cfg->rate_top + b;
        rate = rate * cfg->rate_scale;
        for (int n = 0; n <= 24; ++n) {
            double q = rate * (double)n;
            q = q / 24.0;
            double p = q + cfg->spont;
            out[row * 25 + n] = prob_threshold(p);
        }
    }
    return 0;
}

/* ========================================================================= */
/* World state.  Agents are kept in a dense array in uid order.              */
/* ========================================================================= */

typedef struct {
    oracle_config cfg;
    uint64_t seed;
    genome_layout gl;
    int32_t rho, win, n_in;
    int32_t P;                 /* parameters per agent                      */
    int32_t ss;                /* recurrent state floats per agent          */
    int64_t t;
    uint32_t next_uid;
    int32_t n;                 /* live agents                               */
    uint8_t *R;                /* H*W resource bits                         */
    int32_t *occ;              /* H*W: index into the agent arrays or -1    */
    uint64_t *thr;             /* H*25 regrowth thresholds                  */
    /* agents, uid order */
    uint32_t *uid;
    int32_t *row, *col, *e, *age, *streak;
    /* movement metric: position at the start of the current window, and
     * whether the agent was alive then */
    int32_t *wrow, *wcol;
    uint8_t *wvalid;
    int32_t n_windows, windows_cap;
    int32_t *move_hist;        /* n_windows x (ORACLE_MOVE_BINS + 1): bins, count */
    float *h;                  /* cap * ss: h (GRU); h then c (LSTM)        */
    float *theta;              /* cap * P    */
    int32_t *pact;             /* previous action, ORACLE_NO_ACTION if none */
    uint8_t *pate;             /* ate in the previous step                  */
    /* forced actions */
    int32_t *forced;
    int32_t n_forced, forced_default;
    /* controller outputs of the last step */
    int32_t last_n;
    uint32_t *last_uid;
    double *last_logits;
    uint8_t *last_act;
    /* scratch */
    int32_t *act, *claim;
    uint64_t *best;
    int32_t *who;
    uint8_t *alive, *ate, *won;
    int32_t *cnt;              /* H*W agents per cell at the step start     */
    uint8_t *walldead;         /* moved into a wall this step (paper rules) */
    double *x, *hnew;
} world;

static void observe_cnn(const world *w, int a, double *obs);
static void count_cells(world *w);

/* Action deltas: 0 = N (row - 1), 1 = S (row + 1), 2 = E (col + 1),
 * 3 = W (col - 1), 4 = stay. */
static const int DR[5] = {-1, 1, 0, 0, 0};
static const int DC[5] = {0, 0, 1, -1, 0};

static int in_grid(const world *w, int r, int c)
{
    return r >= 0 && r < w->cfg.H && c >= 0 && c < w->cfg.W;
}

static void set_err(char *err, size_t len, const char *msg)
{
    if (err && len) {
        strncpy(err, msg, len - 1);
        err[len - 1] = 0;
    }
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

void oracle_destroy(void *vw)
{
    world *w = (world *)vw;
    if (!w) return;
    free(w->R); free(w->occ); free(w->thr);
    free(w->uid); free(w->row); free(w->col); free(w->e); free(w->age); free(w->streak);
    free(w->wrow); free(w->wcol); free(w->wvalid); free(w->move_hist);
    free(w->h); free(w->theta); free(w->forced); free(w->pact); free(w->pate); free(w->cnt); free(w->walldead);
    free(w->last_uid); free(w->last_logits); free(w->last_act);
    free(w->act); free(w->claim); free(w->best); free(w->who);
    free(w->alive); free(w->ate); free(w->won); free(w->x); free(w->hnew);
    free(w);
}

/* Initial weights of agent `u` (App. B.2: random once at the start): each
 * weight is N(0, gain / sqrt(fan_in)) with fan_in = inputs for W_ih and
 * Hd for W_hh and W_o; biases start at 0.  Parameter p uses lane p % 4 of
 * generator block p / 4 of stream INIT_W keyed by the agent's uid. */
static void init_genome_cnn(const world *w, uint32_t u, float *th);

static void init_genome(const world *w, uint32_t u, float *th)
{
    if (w->cfg.controller == ORACLE_CTRL_CNN_LSTM) {
        init_genome_cnn(w, u, th);
        return;
    }
    const genome_layout *L = &w->gl;
    float std_ih = (float)(w->cfg.w_init_gain / sqrt((double)L->n_in));
    float std_hd = (float)(w->cfg.w_init_gain / sqrt((double)L->hd));
    for (int32_t p = 0; p < L->P; ++p) {
        float std;
        if (p < L->hh) std = std_ih;
        else if (p < L->bih) std = std_hd;
        else if (p < L->wo) std = 0.0f;          /* b_ih, b_hh */
        else if (p < L->bo) std = std_hd;
        else std = 0.0f;                         /* b_o */
        if (std == 0.0f) {
            th[p] = 0.0f;
            continue;
        }
        uint32_t r[4];
        float z[4];
        draw(w->seed, u, 0, ORACLE_S_INIT_W, (uint32_t)(p / 4), r);
        gauss_block(r, z);
        th[p] = std * z[p % 4];
    }
}

/* The paper's controller starts the same way: weight std gain / sqrt(fan_in)
 * (fan_in = 27 and 36 for the convolutions, 78 and 4 for the LSTM's input and
 * hidden kernels, 82 and 8 for the dense layers), biases 0, parameter p from
 * lane p % 4 of block p / 4 of stream INIT_W. */
static void init_genome_cnn(const world *w, uint32_t u, float *th)
{
    cnn_layout L = cnn_layout_of();
    double gain = w->cfg.w_init_gain;
    for (int32_t p = 0; p < L.P; ++p) {
        int fan = 0;
        if (p < L.c1b) fan = CNN_K * CNN_K * CNN_CH;
        else if (p < L.c2w) fan = 0;
        else if (p < L.c2b) fan = CNN_K * CNN_K * CNN_F1;
        else if (p < L.lwi) fan = 0;
        else if (p < L.lwh) fan = L.emb;
        else if (p < L.lb) fan = CNN_HD;
        else if (p < L.d8w) fan = 0;
        else if (p < L.d8b) fan = L.cat;
        else if (p < L.d5w) fan = 0;
        else if (p < L.d5b) fan = CNN_D;
        if (fan == 0) {
            th[p] = 0.0f;
            continue;
        }
        float std = (float)(gain / sqrt((double)fan));
        uint32_t r[4];
        float z[4];
        draw(w->seed, u, 0, ORACLE_S_INIT_W, (uint32_t)(p / 4), r);
        gauss_block(r, z);
        th[p] = std * z[p % 4];
    }
}

void *oracle_create(const oracle_config *cfg, uint64_t seed, char *err, size_t errlen)
{
    if (cfg->H < 2 || cfg->W < 1) { set_err(err, errlen, "grid must be at least 2 x 1"); return NULL; }
    if ((int64_t)cfg->H * cfg->W > (1 << 26)) { set_err(err, errlen, "grid too large"); return NULL; }
    if (cfg->cap < 1) { set_err(err, errlen, "cap must be positive"); return NULL; }
    if (cfg->n_init < 0 || cfg->n_init > cfg->cap || cfg->n_init > cfg->H * cfg->W) {
        set_err(err, errlen, "n_init out of range"); return NULL;
    }
    if (cfg->controller == ORACLE_CTRL_CNN_LSTM) {
        if (cfg->obs_radius != CNN_RHO) { set_err(err, errlen, "the paper's controller needs obs_radius 7"); return NULL; }
        if (cfg->hidden != CNN_HD) { set_err(err, errlen, "the paper's controller needs hidden 4"); return NULL; }
    } else if (cfg->controller == ORACLE_CTRL_GRU) {
        if (cfg->obs_radius < 1 || cfg->obs_radius > 3) { set_err(err, errlen, "obs_radius must be 1..3"); return NULL; }
        if (cfg->hidden != 16 && cfg->hidden != 32) { set_err(err, errlen, "hidden must be 16 or 32"); return NULL; }
    } else {
        set_err(err, errlen, "unknown controller");
        return NULL;
    }
    if (cfg->E0 <= 0) { set_err(err, errlen, "E0 must be positive"); return NULL; }
    if (cfg->dynamics != ORACLE_DYN_BENCH && cfg->dynamics != ORACLE_DYN_PAPER) {
        set_err(err, errlen, "unknown dynamics"); return NULL;
    }
    if (cfg->dynamics == ORACLE_DYN_PAPER && (cfg->E_max < cfg->E0 || cfg->T_death < 1 || !(cfg->regrow_alpha > 0.0))) {
        set_err(err, errlen, "paper dynamics need E_max >= E0, T_death >= 1, alpha > 0"); return NULL;
    }

    world *w = (world *)calloc(1, sizeof(world));
    w->cfg = *cfg;
    w->seed = seed;
    w->rho = cfg->obs_radius;
    w->win = 2 * w->rho + 1;
    int cnn = cfg->controller == ORACLE_CTRL_CNN_LSTM;
    w->n_in = cnn ? w->win * w->win * CNN_CH : oracle_n_inputs(w->rho);
    w->gl = layout_of(cnn ? 1 : w->n_in, cfg->hidden);
    w->P = cnn ? cnn_layout_of().P : w->gl.P;
    w->ss = cnn ? 2 * cfg->hidden : cfg->hidden;
    size_t HW = (size_t)cfg->H * cfg->W;
    size_t cap = (size_t)cfg->cap;
    int hd = w->ss;
    size_t P = (size_t)w->P;

    w->R = (uint8_t *)calloc(HW, 1);
    w->occ = (int32_t *)malloc(HW * sizeof(int32_t));
    w->thr = (uint64_t *)malloc((size_t)cfg->H * 25 * sizeof(uint64_t));
    w->uid = (uint32_t *)calloc(cap, sizeof(uint32_t));
    w->row = (int32_t *)calloc(cap, sizeof(int32_t));
    w->col = (int32_t *)calloc(cap, sizeof(int32_t));
    w->e = (int32_t *)calloc(cap, sizeof(int32_t));
    w->age = (int32_t *)calloc(cap, sizeof(int32_t));
    w->streak = (int32_t *)calloc(cap, sizeof(int32_t));
    w->wrow = (int32_t *)calloc(cap, sizeof(int32_t));
    w->wcol = (int32_t *)calloc(cap, sizeof(int32_t));
    w->wvalid = (uint8_t *)calloc(cap, 1);
    w->h = (float *)calloc(cap * hd, sizeof(float));
    w->theta = (float *)calloc(cap * P, sizeof(float));
    w->pact = (int32_t *)calloc(cap, sizeof(int32_t));
    w->pate = (uint8_t *)calloc(cap, 1);
    w->cnt = (int32_t *)calloc(HW, sizeof(int32_t));
    w->walldead = (uint8_t *)calloc(cap, 1);
    w->last_uid = (uint32_t *)calloc(cap, sizeof(uint32_t));
    w->last_logits = (double *)calloc(cap * 5, sizeof(double));
    w->last_act = (uint8_t *)calloc(cap, 1);
    w->act = (int32_t *)calloc(cap, sizeof(int32_t));
    w->claim = (int32_t *)calloc(cap, sizeof(int32_t));
    w->best = (uint64_t *)malloc(HW * sizeof(uint64_t));
    w->who = (int32_t *)malloc(HW * sizeof(int32_t));
    w->alive = (uint8_t *)calloc(cap, 1);
    w->ate = (uint8_t *)calloc(cap, 1);
    w->won = (uint8_t *)calloc(cap, 1);
    w->x = (double *)calloc((size_t)w->n_in, sizeof(double));
    w->hnew = (double *)calloc((size_t)hd, sizeof(double));
    w->forced_default = -1;
    if (!w->R || !w->occ || !w->thr || !w->uid || !w->h || !w->theta || !w->best || !w->who || !w->wrow ||
        !w->wcol || !w->wvalid || !w->pact || !w->pate || !w->cnt || !w->walldead) {
        set_err(err, errlen, "out of memory");
        oracle_destroy(w);
        return NULL;
    }
    oracle_threshold_table(cfg, w->thr);

    /* Initial resources: i.i.d. Bernoulli(res_init_p) per cell. */
    uint64_t res_thr = prob_threshold(cfg->res_init_p);
    for (size_t i = 0; i < HW; ++i) {
        uint32_t r[4];
        draw(seed, (uint32_t)i, 0, ORACLE_S_INIT_RES, 0, r);
        w->R[i] = (uint8_t)((uint64_t)r[0] < res_thr);
    }

    /* Initial placement (App. B.4: random): cells ranked by (draw, index);
     * the first n_init cells receive agents with uids 0, 1, ... in rank order. */
    uint64_t *keys = (uint64_t *)malloc(HW * sizeof(uint64_t));
    for (size_t i = 0; i < HW; ++i) {
        uint32_t r[4];
        draw(seed, (uint32_t)i, 0, ORACLE_S_INIT_PLACE, 0, r);
        keys[i] = ((uint64_t)r[0] << 32) | (uint64_t)i;
    }
    qsort(keys, HW, sizeof(uint64_t), cmp_u64);
    for (size_t i = 0; i < HW; ++i) w->occ[i] = -1;
    for (int32_t a = 0; a < cfg->n_init; ++a) {
        uint32_t cell = (uint32_t)(keys[a] & 0xFFFFFFFFu);
        w->uid[a] = (uint32_t)a;
        w->row[a] = (int32_t)(cell / (uint32_t)cfg->W);
        w->col[a] = (int32_t)(cell % (uint32_t)cfg->W);
        w->e[a] = cfg->E0;
        w->age[a] = 0;
        w->streak[a] = 0;
        w->occ[cell] = a;
        w->pact[a] = ORACLE_NO_ACTION;
        w->pate[a] = 0;
        init_genome(w, (uint32_t)a, w->theta + (size_t)a * P);
    }
    free(keys);
    w->n = cfg->n_init;
    w->next_uid = (uint32_t)cfg->n_init;
    w->t = 0;
    count_cells(w);
    return w;
}

void oracle_set_forced(void *vw, const int32_t *act, int32_t n, int32_t dflt)
{
    world *w = (world *)vw;
    free(w->forced);
    w->forced = NULL;
    w->n_forced = 0;
    if (n > 0) {
        w->forced = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        memcpy(w->forced, act, (size_t)n * sizeof(int32_t));
        w->n_forced = n;
    }
    w->forced_default = dflt;
}

static int forced_action(const world *w, uint32_t u)
{
    if (u < (uint32_t)w->n_forced && w->forced[u] >= 0) return w->forced[u];
    return w->forced_default;
}

/* Agents per cell (one at most under the benchmark rules). */
static void count_cells(world *w)
{
    size_t HW = (size_t)w->cfg.H * w->cfg.W;
    for (size_t i = 0; i < HW; ++i) w->cnt[i] = 0;
    for (int a = 0; a < w->n; ++a) w->cnt[w->row[a] * w->cfg.W + w->col[a]]++;
}

/* Observation (App. B.2) of agent a: the (2 rho + 1)^2 window of resource
 * bits, then the same window of occupancy bits, row-major (dy outer, dx
 * inner), then energy / E0.  Reading for the boundary (the grid does not
 * wrap): outside cells show no resource and count as occupied.  The agent's
 * own cell shows as occupied. */
static void observe(const world *w, int a, double *x)
{
    int rho = w->rho, win = w->win, W = w->cfg.W;
    for (int dy = -rho; dy <= rho; ++dy) {
        for (int dx = -rho; dx <= rho; ++dx) {
            int k = (dy + rho) * win + (dx + rho);
            int r = w->row[a] + dy, c = w->col[a] + dx;
            if (in_grid(w, r, c)) {
                x[k] = w->R[r * W + c] ? 1.0 : 0.0;
                x[win * win + k] = (w->cnt[r * W + c] > 0) ? 1.0 : 0.0;
            } else {
                x[k] = 0.0;
                x[win * win + k] = 1.0;
            }
        }
    }
    x[2 * win * win] = (double)w->e[a] / (double)w->cfg.E0;
}

/* Observation of the paper's controller (App. B.2): the 15 x 15 square around
 * the agent, three channels per pixel: resource, number of agents (0 or 1
 * here, the agent itself included), wall.  Reading: the only walls are the
 * cells outside the grid, which show no resource and no agent. */
static void observe_cnn(const world *w, int a, double *obs)
{
    int rho = w->rho, win = w->win, W = w->cfg.W;
    for (int dy = -rho; dy <= rho; ++dy)
        for (int dx = -rho; dx <= rho; ++dx) {
            double *px = obs + ((dy + rho) * win + (dx + rho)) * CNN_CH;
            int r = w->row[a] + dy, c = w->col[a] + dx;
            if (in_grid(w, r, c)) {
                px[0] = w->R[r * W + c] ? 1.0 : 0.0;
                px[1] = (double)w->cnt[r * W + c];   /* the number of agents on the pixel */
                px[2] = 0.0;
            } else {
                px[0] = 0.0;
                px[1] = 0.0;
                px[2] = 1.0;
            }
        }
}

static uint64_t claim_key(uint32_t draw_word, uint32_t u)
{
    return ((uint64_t)draw_word << 32) | (uint64_t)u;
}

/* S3-S8 under the paper's rules (App. B.2, B.3), on the actions in w->act.
 * Readings: a move into a wall (outside the grid) kills the agent; agents may
 * share cells; on a cell holding a resource after the moves, the agent with the
 * smallest (EAT draw, uid) eats it; e <- min(e - decay + gain ate, E_max);
 * the signed streak counts consecutive steps above E_repr (positive) or below
 * it (negative), 0 at E_repr; death when it reaches -T_death, when age exceeds
 * L_max or at a wall; an agent whose streak reaches T_repr has one child on its
 * own cell (uid order while slots remain) and its streak restarts. */
static void step_paper(world *w, uint32_t t, oracle_stepinfo *inf)
{
    const oracle_config *cfg = &w->cfg;
    const int W = cfg->W, hd = w->ss;
    const size_t HW = (size_t)cfg->H * W, P = (size_t)w->P;
    /* S3 moves */
    for (int a = 0; a < w->n; ++a) {
        w->walldead[a] = 0;
        int act = w->act[a];
        if (act == 4) continue;
        int r = w->row[a] + DR[act], c = w->col[a] + DC[act];
        if (!in_grid(w, r, c)) {
            w->walldead[a] = 1;
            continue;
        }
        w->row[a] = r;
        w->col[a] = c;
    }
    /* S4 eat: one agent per resource, smallest (EAT draw, uid) */
    for (size_t i = 0; i < HW; ++i) {
        w->best[i] = UINT64_MAX;
        w->who[i] = -1;
    }
    for (int a = 0; a < w->n; ++a) {
        w->ate[a] = 0;
        if (w->walldead[a]) continue;
        int cell = w->row[a] * W + w->col[a];
        if (!w->R[cell]) continue;
        uint32_t rr[4];
        draw(w->seed, w->uid[a], t, ORACLE_S_EAT, 0, rr);
        uint64_t key = claim_key(rr[0], w->uid[a]);
        if (key < w->best[cell]) {
            w->best[cell] = key;
            w->who[cell] = a;
        }
    }
    for (size_t i = 0; i < HW; ++i)
        if (w->who[i] >= 0) {
            w->ate[w->who[i]] = 1;
            w->R[i] = 0;
            inf->eaten++;
        }
    /* S5 energy (clipped) and age; S6 streak and death */
    int n_surv = 0;
    for (int a = 0; a < w->n; ++a) {
        int e = w->e[a] - cfg->decay + cfg->gain * (int32_t)w->ate[a];
        if (e > cfg->E_max) e = cfg->E_max;
        w->e[a] = e;
        w->age[a] = w->age[a] + 1;
        w->pate[a] = w->ate[a];
        int s = w->streak[a];
        if (e > cfg->E_repr) s = (s > 0 ? s : 0) + 1;
        else if (e < cfg->E_repr) s = (s < 0 ? s : 0) - 1;
        else s = 0;
        w->streak[a] = s;
        int dead = w->walldead[a] || (-s >= cfg->T_death) || (w->age[a] > cfg->L_max);
        if (dead) {
            inf->deaths++;
            inf->dead_age += w->age[a];
            continue;
        }
        if (n_surv != a) {
            w->uid[n_surv] = w->uid[a];
            w->row[n_surv] = w->row[a];
            w->col[n_surv] = w->col[a];
            w->e[n_surv] = w->e[a];
            w->age[n_surv] = w->age[a];
            w->streak[n_surv] = w->streak[a];
            w->wrow[n_surv] = w->wrow[a];
            w->wcol[n_surv] = w->wcol[a];
            w->wvalid[n_surv] = w->wvalid[a];
            w->pact[n_surv] = w->pact[a];
            w->pate[n_surv] = w->pate[a];
            memmove(w->h + (size_t)n_surv * hd, w->h + (size_t)a * hd, (size_t)hd * sizeof(float));
            memmove(w->theta + (size_t)n_surv * P, w->theta + (size_t)a * P, P * sizeof(float));
        }
        n_surv++;
    }
    w->n = n_surv;
    /* S8 births on the parent's cell (with no free slot nobody can be born and
     * no claim is counted) */
    int n_elig = 0;
    for (int a = 0; a < w->n; ++a) n_elig += w->streak[a] >= cfg->T_repr;
    int free_slots = cfg->cap - w->n;
    inf->claim_wins = free_slots > 0 ? n_elig : 0;
    int n_born = n_elig < free_slots ? n_elig : free_slots;
    int rank = 0;
    int n_before = w->n;
    for (int a = 0; a < n_before && rank < n_born; ++a) {
        if (w->streak[a] < cfg->T_repr) continue;
        int c = w->n;
        uint32_t cu = w->next_uid + (uint32_t)rank;
        w->uid[c] = cu;
        w->row[c] = w->row[a];
        w->col[c] = w->col[a];
        w->e[c] = cfg->E0;
        w->age[c] = 0;
        w->streak[c] = 0;
        w->wvalid[c] = 0;
        w->pact[c] = ORACLE_NO_ACTION;
        w->pate[c] = 0;
        memset(w->h + (size_t)c * hd, 0, (size_t)hd * sizeof(float));
        const float *pth = w->theta + (size_t)a * P;
        float *cth = w->theta + (size_t)c * P;
        float sigma = (float)cfg->sigma_mut;
        for (int32_t p = 0; p < (int32_t)P; ++p) {
            uint32_t r[4];
            float z[4];
            draw(w->seed, cu, t, ORACLE_S_MUTATE, (uint32_t)(p / 4), r);
            gauss_block(r, z);
            cth[p] = fmaf(sigma, z[p % 4], pth[p]);
        }
        w->streak[a] = 0;
        w->n++;
        rank++;
    }
    w->next_uid += (uint32_t)n_born;
    inf->births = n_born;
}

int oracle_step(void *vw, const uint32_t *hint_uid, const uint8_t *hint_act, int32_t n_hint,
                oracle_stepinfo *info)
{
    world *w = (world *)vw;
    const oracle_config *cfg = &w->cfg;
    const int H = cfg->H, W = cfg->W, hd = w->ss;   /* hd: state floats per agent */
    const size_t HW = (size_t)H * W;
    const size_t P = (size_t)w->P;
    const int cnn = cfg->controller == ORACLE_CTRL_CNN_LSTM;
    const uint32_t t = (uint32_t)w->t;
    oracle_stepinfo inf;
    memset(&inf, 0, sizeof(inf));

    /* Movement metric (App. C): a window starts with this step; remember
     * where every agent alive now stands. */
    if (w->t % ORACLE_MOVE_WINDOW == 0) {
        for (int a = 0; a < w->n; ++a) {
            w->wrow[a] = w->row[a];
            w->wcol[a] = w->col[a];
            w->wvalid[a] = 1;
        }
    }

    /* ---- S1 + S2: observe and act (App. B.2), all on the step-start state. */
    int hi = 0;
    w->last_n = w->n;
    for (int a = 0; a < w->n; ++a) {
        uint32_t u = w->uid[a];
        double *lg = w->last_logits + (size_t)a * 5;
        /* lab greediness: does the field of view hold a resource? */
        int sees = 0;
        for (int dy = -w->rho; dy <= w->rho && !sees; ++dy)
            for (int dx = -w->rho; dx <= w->rho; ++dx) {
                int r = w->row[a] + dy, c = w->col[a] + dx;
                if (in_grid(w, r, c) && w->R[r * W + c]) {
                    sees = 1;
                    break;
                }
            }
        inf.seen += sees;
        float *ha = w->h + (size_t)a * hd;
        float lf[5], sc[5];
        if (cnn) {
            observe_cnn(w, a, w->x);
            oracle_cnn_eval(w->theta + (size_t)a * P, w->x, w->pact[a], w->pate[a], ha, ha + CNN_HD,
                            w->hnew, w->hnew + CNN_HD, lg);
        } else {
            observe(w, a, w->x);
            oracle_gru_eval(w->n_in, hd, w->theta + (size_t)a * P, w->x, ha, w->hnew, lg);
        }
        /* The recurrent state is kept in single precision between steps. */
        for (int k = 0; k < hd; ++k) ha[k] = (float)w->hnew[k];
        for (int k = 0; k < 5; ++k) lf[k] = (float)lg[k];
        /* GRU reading: the action is the arg-max of the logits (lowest index
         * on an exact tie), decided on the single-precision values.  The
         * paper's controller samples: arg-max of the sampling scores. */
        if (cnn) sample_scores(w->seed, u, t, lf, sc);
        else memcpy(sc, lf, sizeof(sc));
        int best = 0;
        for (int k = 1; k < 5; ++k)
            if (sc[k] > sc[best]) best = k;
        int act = best;
        int fa = forced_action(w, u);
        int forced = fa >= 0 && fa < 5;
        if (forced) act = fa;
        /* Near-tie resync: adopt the hinted action when its score lies within
         * the band of this oracle's top score that the logit tolerance allows:
         * 1e-5 * max(1, |top|) for the GRU's logits; for the sampling scores
         * 50 times the logit tolerance plus the same relative band (the
         * Gumbel terms are identical on both sides).  A forced action must be
         * matched exactly. */
        while (hint_uid && hi < n_hint && hint_uid[hi] < u) ++hi;
        if (hint_uid && hi < n_hint && hint_uid[hi] == u) {
            int ha_ = hint_act[hi];
            if (ha_ != act) {
                double top = cnn ? (double)sc[best] : lg[best];
                int hk = (ha_ >= 0 && ha_ < 5) ? ha_ : 0;
                double hv = cnn ? (double)sc[hk] : lg[hk];
                double band = 1e-5 * fmax(1.0, fabs(top));
                if (cnn) {
                    double lmax = 1.0;
                    for (int k = 0; k < 5; ++k) lmax = fmax(lmax, fabs(lg[k]));
                    band += 50.0 * 1e-5 * lmax;
                }
                if (!forced && ha_ >= 0 && ha_ < 5 && top - hv < band) {
                    act = ha_;
                    inf.resyncs++;
                } else {
                    inf.mismatches++;
                }
            }
        }
        w->act[a] = act;
        w->pact[a] = act;
        w->last_uid[a] = u;
        w->last_act[a] = (uint8_t)act;
    }

    if (cfg->dynamics == ORACLE_DYN_PAPER) {
        step_paper(w, t, &inf);
    } else {
        /* ---- S3: moves.  Reading (the paper lets agents share cells; the
         * benchmark forbids it): a move targets an in-grid cell that is empty at
         * the start of the step; among the claimants of one cell the smallest
         * (MOVE draw, uid) wins; everyone else stays.  Moves apply together. */
        for (size_t i = 0; i < HW; ++i) {
            w->best[i] = UINT64_MAX;
            w->who[i] = -1;
        }
        for (int a = 0; a < w->n; ++a) {
            w->claim[a] = -1;
            int act = w->act[a];
            if (act == 4) continue;
            int r = w->row[a] + DR[act], c = w->col[a] + DC[act];
            if (!in_grid(w, r, c)) continue;
            int cell = r * W + c;
            if (w->occ[cell] != -1) continue;
            uint32_t rr[4];
            draw(w->seed, w->uid[a], t, ORACLE_S_MOVE, 0, rr);
            uint64_t key = claim_key(rr[0], w->uid[a]);
            w->claim[a] = cell;
            if (key < w->best[cell]) {
                w->best[cell] = key;
                w->who[cell] = a;
            }
        }
        for (int a = 0; a < w->n; ++a) {
            int cell = w->claim[a];
            if (cell >= 0 && w->who[cell] == a) {
                w->occ[w->row[a] * W + w->col[a]] = -1;
                w->row[a] = cell / W;
                w->col[a] = cell % W;
            }
        }
        for (int a = 0; a < w->n; ++a) w->occ[w->row[a] * W + w->col[a]] = a;

        /* ---- S4 + S5: eat and update energy and age (App. B.2).  Reading: an
         * agent eats the resource of the cell it occupies after moving; energy
         * changes by gain * ate - decay, unclipped; age counts steps lived. */
        for (int a = 0; a < w->n; ++a) {
            int cell = w->row[a] * W + w->col[a];
            w->ate[a] = 0;
            if (w->R[cell]) {
                w->R[cell] = 0;
                w->ate[a] = 1;
                inf.eaten++;
            }
            w->pate[a] = w->ate[a];
            w->e[a] = w->e[a] - cfg->decay + cfg->gain * (int32_t)w->ate[a];
            w->age[a] = w->age[a] + 1;
        }

        /* ---- S6: death (App. B.3): energy at or below zero, or age reaching
         * L_max.  Survivors keep their uid order. */
        int n_surv = 0;
        for (int a = 0; a < w->n; ++a) {
            int dead = (w->e[a] <= 0) || (w->age[a] >= cfg->L_max);
            if (dead) {
                inf.deaths++;
                inf.dead_age += w->age[a];   /* life expectancy (App. C): age at death */
                continue;
            }
            if (n_surv != a) {
                w->uid[n_surv] = w->uid[a];
                w->row[n_surv] = w->row[a];
                w->col[n_surv] = w->col[a];
                w->e[n_surv] = w->e[a];
                w->age[n_surv] = w->age[a];
                w->streak[n_surv] = w->streak[a];
                w->wrow[n_surv] = w->wrow[a];
                w->wcol[n_surv] = w->wcol[a];
                w->wvalid[n_surv] = w->wvalid[a];
                w->pact[n_surv] = w->pact[a];
                w->pate[n_surv] = w->pate[a];
                memmove(w->h + (size_t)n_surv * hd, w->h + (size_t)a * hd, (size_t)hd * sizeof(float));
                memmove(w->theta + (size_t)n_surv * P, w->theta + (size_t)a * P, P * sizeof(float));
            }
            n_surv++;
        }
        w->n = n_surv;
        for (size_t i = 0; i < HW; ++i) w->occ[i] = -1;
        for (int a = 0; a < w->n; ++a) w->occ[w->row[a] * W + w->col[a]] = a;

        /* ---- S7: the minimal criterion (App. B.3): count consecutive steps
         * with energy at or above E_repr; eligible once the count reaches T_repr. */
        for (int a = 0; a < w->n; ++a)
            w->streak[a] = (w->e[a] >= cfg->E_repr) ? w->streak[a] + 1 : 0;

        /* ---- S8: births.  Reading (the paper places the child on the parent's
         * cell; the benchmark forbids sharing): an eligible parent scans its four
         * neighbours in the order N, S, E, W cyclically from a random start and
         * claims the first free in-grid cell; claims resolve like moves with the
         * BIRTH draw; winners are born in uid order while slots remain.  With no
         * free slot (the survivors fill the cap) nobody can be born: no claim is
         * made or resolved, and no winner is counted. */
        int free_slots = cfg->cap - w->n;
        for (size_t i = 0; i < HW; ++i) {
            w->best[i] = UINT64_MAX;
            w->who[i] = -1;
        }
        for (int a = 0; a < w->n; ++a) {
            w->claim[a] = -1;
            w->won[a] = 0;
            if (free_slots <= 0 || w->streak[a] < cfg->T_repr) continue;
            uint32_t rr[4];
            draw(w->seed, w->uid[a], t, ORACLE_S_BIRTH, 0, rr);
            int d0 = (int)(rr[0] & 3u);
            for (int k = 0; k < 4; ++k) {
                int d = (d0 + k) & 3;
                int r = w->row[a] + DR[d], c = w->col[a] + DC[d];
                if (in_grid(w, r, c) && w->occ[r * W + c] == -1) {
                    w->claim[a] = r * W + c;
                    break;
                }
            }
            if (w->claim[a] < 0) continue;
            uint64_t key = claim_key(rr[1], w->uid[a]);
            int cell = w->claim[a];
            if (key < w->best[cell]) {
                w->best[cell] = key;
                w->who[cell] = a;
            }
        }
        int n_win = 0;
        for (int a = 0; a < w->n; ++a)
            if (w->claim[a] >= 0 && w->who[w->claim[a]] == a) {
                w->won[a] = 1;
                n_win++;
            }
        inf.claim_wins = n_win;
        int n_born = n_win < free_slots ? n_win : free_slots;
        int rank = 0;
        int n_before = w->n;
        for (int a = 0; a < n_before && rank < n_born; ++a) {
            if (!w->won[a]) continue;
            int c = w->n;                         /* child index (appended) */
            uint32_t cu = w->next_uid + (uint32_t)rank;
            w->uid[c] = cu;
            w->row[c] = w->claim[a] / W;
            w->col[c] = w->claim[a] % W;
            w->e[c] = cfg->E0;
            w->age[c] = 0;
            w->streak[c] = 0;
            w->wvalid[c] = 0;   /* not alive at the start of the window */
            w->pact[c] = ORACLE_NO_ACTION;
            w->pate[c] = 0;
            memset(w->h + (size_t)c * hd, 0, (size_t)hd * sizeof(float));
            /* Mutation (App. B.3): every parameter gets sigma * z added, z from
             * lane p % 4 of block p / 4 of stream MUTATE keyed by the child uid. */
            const float *pth = w->theta + (size_t)a * P;
            float *cth = w->theta + (size_t)c * P;
            float sigma = (float)cfg->sigma_mut;
            for (int32_t p = 0; p < (int32_t)P; ++p) {
                uint32_t r[4];
                float z[4];
                draw(w->seed, cu, t, ORACLE_S_MUTATE, (uint32_t)(p / 4), r);
                gauss_block(r, z);
                cth[p] = fmaf(sigma, z[p % 4], pth[p]);
            }
            w->streak[a] = 0;
            w->occ[w->claim[a]] = c;
            w->n++;
            rank++;
        }
        w->next_uid += (uint32_t)n_born;
        inf.births = n_born;
    }

    /* ---- S10: regrowth (App. B.1, Eq. (1)), synchronous on the grid left by
     * eating: an empty cell grows iff its REGROW draw is below the threshold
     * for its row and its count of resources among the 24 cells at Chebyshev
     * distance 1..2 (outside cells count 0).  Resources never disappear by
     * themselves. */
    uint8_t *Rn = (uint8_t *)malloc(HW);
    memcpy(Rn, w->R, HW);
    for (int r = 0; r < H; ++r) {
        for (int c = 0; c < W; ++c) {
            if (w->R[r * W + c]) continue;
            int n = 0;
            if (cfg->dynamics == ORACLE_DYN_PAPER) {
                /* the four direct neighbours (App. B.1) */
                for (int k = 0; k < 4; ++k)
                    if (in_grid(w, r + DR[k], c + DC[k]) && w->R[(r + DR[k]) * W + c + DC[k]]) n++;
            } else {
                for (int dy = -2; dy <= 2; ++dy)
                    for (int dx = -2; dx <= 2; ++dx) {
                        if (dy == 0 && dx == 0) continue;
                        if (in_grid(w, r + dy, c + dx) && w->R[(r + dy) * W + c + dx]) n++;
                    }
            }
            uint32_t rr[4];
            draw(w->seed, (uint32_t)(r * W + c), t, ORACLE_S_REGROW, 0, rr);
            if ((uint64_t)rr[0] < w->thr[r * 25 + n]) Rn[r * W + c] = 1;
        }
    }
    memcpy(w->R, Rn, HW);
    free(Rn);
    int res = 0;
    for (size_t i = 0; i < HW; ++i) res += w->R[i];

    inf.n_live = w->n;
    inf.resources = res;

    /* Movement metric: the window ends with this step; the Manhattan distance
     * travelled by every agent alive at both ends goes into bin distance / 3. */
    if ((w->t + 1) % ORACLE_MOVE_WINDOW == 0) {
        if (w->n_windows == w->windows_cap) {
            int32_t nc = w->windows_cap ? 2 * w->windows_cap : 64;
            int32_t *nh = (int32_t *)realloc(w->move_hist, (size_t)nc * (ORACLE_MOVE_BINS + 1) * sizeof(int32_t));
            if (!nh) return -1;
            w->move_hist = nh;
            w->windows_cap = nc;
        }
        int32_t *hist = w->move_hist + (size_t)w->n_windows * (ORACLE_MOVE_BINS + 1);
        memset(hist, 0, (ORACLE_MOVE_BINS + 1) * sizeof(int32_t));
        for (int a = 0; a < w->n; ++a) {
            if (!w->wvalid[a]) continue;
            int dist = abs(w->row[a] - w->wrow[a]) + abs(w->col[a] - w->wcol[a]);
            hist[dist / 3]++;
            hist[ORACLE_MOVE_BINS]++;
        }
        w->n_windows++;
    }
    w->t++;
    count_cells(w);
    if (info) *info = inf;
    return 0;
}

int oracle_load(void *vw, int64_t step, int32_t n, uint32_t next_uid, const uint8_t *R, const uint32_t *uid,
                const int32_t *row, const int32_t *col, const int32_t *energy, const int32_t *age,
                const int32_t *streak, const float *h, const float *theta, const uint8_t *last_action,
                const uint8_t *ate)
{
    world *w = (world *)vw;
    const int H = w->cfg.H, W = w->cfg.W;
    const size_t HW = (size_t)H * W, P = (size_t)w->P, ss = (size_t)w->ss;
    if (n < 0 || n > w->cfg.cap || step < 0) return -1;
    for (int a = 0; a < n; ++a) {
        if (!in_grid(w, row[a], col[a])) return -1;
        if (a > 0 && uid[a] <= uid[a - 1]) return -1;
        if (uid[a] >= next_uid || last_action[a] > ORACLE_NO_ACTION || ate[a] > 1) return -1;
    }
    for (size_t i = 0; i < HW; ++i) w->occ[i] = -1;
    for (int a = 0; a < n; ++a) {
        int cell = row[a] * W + col[a];
        if (w->occ[cell] != -1 && w->cfg.dynamics != ORACLE_DYN_PAPER) return -1;
        w->occ[cell] = a;
    }
    memcpy(w->R, R, HW);
    for (int a = 0; a < n; ++a) {
        w->uid[a] = uid[a];
        w->row[a] = row[a];
        w->col[a] = col[a];
        w->e[a] = energy[a];
        w->age[a] = age[a];
        w->streak[a] = streak[a];
        w->pact[a] = last_action[a];
        w->pate[a] = ate[a];
        w->wvalid[a] = 0;
    }
    memcpy(w->h, h, (size_t)n * ss * sizeof(float));
    memcpy(w->theta, theta, (size_t)n * P * sizeof(float));
    w->n = n;
    w->next_uid = next_uid;
    w->t = step;
    w->last_n = 0;
    count_cells(w);
    return 0;
}

int64_t oracle_t(const void *w) { return ((const world *)w)->t; }
int32_t oracle_n_live(const void *w) { return ((const world *)w)->n; }
uint32_t oracle_next_uid(const void *w) { return ((const world *)w)->next_uid; }

void oracle_get_grid(const void *vw, uint8_t *R)
{
    const world *w = (const world *)vw;
    memcpy(R, w->R, (size_t)w->cfg.H * w->cfg.W);
}

void oracle_get_agents(const void *vw, uint32_t *uid, int32_t *row, int32_t *col,
                       int32_t *energy, int32_t *age, int32_t *streak)
{
    const world *w = (const world *)vw;
    size_t n = (size_t)w->n;
    if (uid) memcpy(uid, w->uid, n * sizeof(uint32_t));
    if (row) memcpy(row, w->row, n * sizeof(int32_t));
    if (col) memcpy(col, w->col, n * sizeof(int32_t));
    if (energy) memcpy(energy, w->e, n * sizeof(int32_t));
    if (age) memcpy(age, w->age, n * sizeof(int32_t));
    if (streak) memcpy(streak, w->streak, n * sizeof(int32_t));
}

void oracle_get_hidden(const void *vw, float *h)
{
    const world *w = (const world *)vw;
    memcpy(h, w->h, (size_t)w->n * w->ss * sizeof(float));
}

void oracle_get_recurrent_inputs(const void *vw, uint8_t *last_action, uint8_t *ate)
{
    const world *w = (const world *)vw;
    for (int a = 0; a < w->n; ++a) {
        if (last_action) last_action[a] = (uint8_t)w->pact[a];
        if (ate) ate[a] = w->pate[a];
    }
}

int oracle_get_obs_cnn(const void *vw, int32_t a, double *obs)
{
    const world *w = (const world *)vw;
    if (w->cfg.controller != ORACLE_CTRL_CNN_LSTM || a < 0 || a >= w->n) return -1;
    observe_cnn(w, a, obs);
    return 0;
}

void oracle_get_theta(const void *vw, float *theta)
{
    const world *w = (const world *)vw;
    memcpy(theta, w->theta, (size_t)w->n * w->P * sizeof(float));
}

int32_t oracle_last_n_acted(const void *w) { return ((const world *)w)->last_n; }

int32_t oracle_n_move_windows(const void *w) { return ((const world *)w)->n_windows; }

int oracle_get_move_hist(const void *vw, int32_t k, int32_t *bins, int32_t *count)
{
    const world *w = (const world *)vw;
    if (k < 0 || k >= w->n_windows) return -1;
    const int32_t *hist = w->move_hist + (size_t)k * (ORACLE_MOVE_BINS + 1);
    if (bins) memcpy(bins, hist, ORACLE_MOVE_BINS * sizeof(int32_t));
    if (count) *count = hist[ORACLE_MOVE_BINS];
    return 0;
}

void oracle_get_last_logits(const void *vw, uint32_t *uid, double *logits, uint8_t *action)
{
    const world *w = (const world *)vw;
    size_t n = (size_t)w->last_n;
    if (uid) memcpy(uid, w->last_uid, n * sizeof(uint32_t));
    if (logits) memcpy(logits, w->last_logits, n * 5 * sizeof(double));
    if (action) memcpy(action, w->last_act, n);
}
