/* Drives the oracle's C code under AddressSanitizer and UndefinedBehavior-
 * Sanitizer (CPU only): worlds under both rule sets and both controllers
 * with births, deaths and a full slot table, forced actions, snapshot ->
 * load -> resume compared with an uninterrupted run, rejected images, the
 * movement windows and the primitives at their extreme inputs.  Exits 0 and
 * prints "ok" when every check holds; any sanitizer report aborts it. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            exit(1);                                                  \
        }                                                             \
    } while (0)

typedef struct {
    int64_t t;
    int32_t n;
    uint32_t next_uid;
    uint8_t *R, *la, *ate;
    uint32_t *uid;
    int32_t *row, *col, *e, *age, *st;
    float *h, *theta;
} image;

static oracle_config base(int H, int W, int cap, int n0, int rho, int hd)
{
    oracle_config c;
    memset(&c, 0, sizeof(c));
    c.H = H; c.W = W; c.cap = cap; c.n_init = n0; c.obs_radius = rho; c.hidden = hd;
    c.res_init_p = 0.4; c.rate_bottom = 0.02; c.rate_top = 0.002; c.rate_scale = 5.0; c.spont = 1e-5;
    c.E0 = 50; c.decay = 1; c.gain = 10; c.E_repr = 40; c.T_repr = 8; c.L_max = 150;
    c.sigma_mut = 0.02; c.w_init_gain = 0.5; c.regrow_alpha = 1.0;
    return c;
}

static int n_params(const oracle_config *c)
{
    return c->controller == ORACLE_CTRL_CNN_LSTM ? oracle_cnn_n_params() : oracle_n_params(c->obs_radius, c->hidden);
}

static int state_of(const oracle_config *c) { return c->controller == ORACLE_CTRL_CNN_LSTM ? 8 : c->hidden; }

static image take(void *w, const oracle_config *c)
{
    image m;
    size_t n = (size_t)oracle_n_live(w), HW = (size_t)c->H * c->W, P = (size_t)n_params(c);
    m.t = oracle_t(w);
    m.n = (int32_t)n;
    m.next_uid = oracle_next_uid(w);
    m.R = malloc(HW);
    m.la = malloc(n + 1);
    m.ate = malloc(n + 1);
    m.uid = malloc(4 * (n + 1));
    m.row = malloc(4 * (n + 1)); m.col = malloc(4 * (n + 1)); m.e = malloc(4 * (n + 1));
    m.age = malloc(4 * (n + 1)); m.st = malloc(4 * (n + 1));
    m.h = malloc(4 * (n * state_of(c) + 1));
    m.theta = malloc(4 * (n * P + 1));
    oracle_get_grid(w, m.R);
    oracle_get_agents(w, m.uid, m.row, m.col, m.e, m.age, m.st);
    oracle_get_hidden(w, m.h);
    oracle_get_theta(w, m.theta);
    oracle_get_recurrent_inputs(w, m.la, m.ate);
    return m;
}

static void drop(image *m)
{
    free(m->R); free(m->la); free(m->ate); free(m->uid); free(m->row); free(m->col); free(m->e);
    free(m->age); free(m->st); free(m->h); free(m->theta);
}

static int same(const image *a, const image *b, const oracle_config *c)
{
    size_t n = (size_t)a->n, HW = (size_t)c->H * c->W, P = (size_t)n_params(c);
    if (a->t != b->t || a->n != b->n || a->next_uid != b->next_uid) return 0;
    if (memcmp(a->R, b->R, HW)) return 0;
    if (memcmp(a->uid, b->uid, 4 * n) || memcmp(a->row, b->row, 4 * n) || memcmp(a->col, b->col, 4 * n)) return 0;
    if (memcmp(a->e, b->e, 4 * n) || memcmp(a->age, b->age, 4 * n) || memcmp(a->st, b->st, 4 * n)) return 0;
    if (memcmp(a->h, b->h, 4 * n * state_of(c)) || memcmp(a->theta, b->theta, 4 * n * P)) return 0;
    if (memcmp(a->la, b->la, n) || memcmp(a->ate, b->ate, n)) return 0;
    return 1;
}

static void *make(const oracle_config *c, uint64_t seed)
{
    char err[256];
    void *w = oracle_create(c, seed, err, sizeof err);
    if (!w) fprintf(stderr, "create: %s\n", err);
    CHECK(w);
    return w;
}

/* `steps` steps in one run against `half` steps, an image, a fresh world
 * loaded from it and the rest: identical end states. */
static void resume_case(const char *name, const oracle_config *c, uint64_t seed, int steps, int half, const int32_t *forced,
                        int n_forced, int dflt)
{
    void *a = make(c, seed), *b = make(c, seed), *r = make(c, seed);
    /* r takes a few steps of its own first: the load must overwrite all of it */
    for (int s = 0; s < 7; ++s) CHECK(oracle_step(r, NULL, NULL, 0, NULL) == 0);
    oracle_stepinfo inf;
    long births = 0, deaths = 0;
    if (forced || dflt >= 0) {
        oracle_set_forced(a, forced, n_forced, dflt);
        oracle_set_forced(b, forced, n_forced, dflt);
        oracle_set_forced(r, forced, n_forced, dflt);
    }
    for (int s = 0; s < steps; ++s) {
        CHECK(oracle_step(a, NULL, NULL, 0, &inf) == 0);
        births += inf.births;
        deaths += inf.deaths;
        CHECK(inf.n_live <= c->cap && inf.mismatches == 0);
    }
    for (int s = 0; s < half; ++s) CHECK(oracle_step(b, NULL, NULL, 0, &inf) == 0);
    image m = take(b, c);
    CHECK(oracle_load(r, m.t, m.n, m.next_uid, m.R, m.uid, m.row, m.col, m.e, m.age, m.st, m.h, m.theta, m.la,
                      m.ate) == 0);
    for (int s = half; s < steps; ++s) CHECK(oracle_step(r, NULL, NULL, 0, &inf) == 0);
    image ea = take(a, c), er = take(r, c);
    CHECK(same(&ea, &er, c));
    /* the logits and movement windows of the last step are readable */
    int32_t na = oracle_last_n_acted(a);
    uint32_t *u = malloc(4 * (size_t)(na + 1));
    double *lg = malloc(8 * 5 * (size_t)(na + 1));
    uint8_t *ac = malloc((size_t)na + 1);
    oracle_get_last_logits(a, u, lg, ac);
    for (int i = 0; i < na; ++i) CHECK(isfinite(lg[5 * i]) && ac[i] < 5);
    int32_t bins[ORACLE_MOVE_BINS], cnt;
    for (int k = 0; k < oracle_n_move_windows(a); ++k) CHECK(oracle_get_move_hist(a, k, bins, &cnt) == 0);
    CHECK(oracle_get_move_hist(a, -1, bins, &cnt) == -1);
    CHECK(oracle_get_move_hist(a, oracle_n_move_windows(a), bins, &cnt) == -1);
    /* an invalid image is rejected and leaves no damage behind */
    if (m.n >= 2) {
        uint32_t keep = m.uid[1];
        m.uid[1] = m.uid[0];
        CHECK(oracle_load(r, m.t, m.n, m.next_uid, m.R, m.uid, m.row, m.col, m.e, m.age, m.st, m.h, m.theta, m.la,
                          m.ate) == -1);
        m.uid[1] = keep;
        int32_t kr = m.row[0];
        m.row[0] = c->H;
        CHECK(oracle_load(r, m.t, m.n, m.next_uid, m.R, m.uid, m.row, m.col, m.e, m.age, m.st, m.h, m.theta, m.la,
                          m.ate) == -1);
        m.row[0] = kr;
    }
    CHECK(oracle_load(r, m.t, c->cap + 1, m.next_uid, m.R, m.uid, m.row, m.col, m.e, m.age, m.st, m.h, m.theta,
                      m.la, m.ate) == -1);
    printf("%s: %d steps, %ld births, %ld deaths, final population %d\n", name, steps, births, deaths, ea.n);
    free(u); free(lg); free(ac);
    drop(&m); drop(&ea); drop(&er);
    oracle_destroy(a); oracle_destroy(b); oracle_destroy(r);
}

int main(void)
{
    /* primitives at their extreme inputs */
    {
        uint32_t ctr[8] = {0, 0, 0, 0, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, key[2] = {0xFFFFFFFFu, 1},
                 out[8];
        oracle_philox4x32_10(ctr, key, out, 2);
        float u[4] = {5.9604645e-08f, 0.5f, 0.99999994f, 1.0f}, l[4], s[4], co[4];
        oracle_ln_unit(u, l, 4);
        oracle_sincos_2pi(u, s, co, 4);
        for (int i = 0; i < 4; ++i) CHECK(isfinite(l[i]) && isfinite(s[i]) && isfinite(co[i]));
        uint32_t a[3] = {0, 0xFFFFFFFFu, 12345}, b[3] = {0xFFFFFFFFu, 0, 54321};
        float z0[3], z1[3], g[3];
        oracle_gauss_pair(a, b, z0, z1, 3);
        oracle_gumbel(a, g, 3);
        for (int i = 0; i < 3; ++i) CHECK(isfinite(z0[i]) && isfinite(z1[i]) && isfinite(g[i]));
    }
    /* regrowth tables of both rule sets */
    {
        oracle_config c = base(200, 400, 4608, 4096, 3, 32);
        uint64_t *thr = malloc(sizeof(uint64_t) * 200 * 25);
        CHECK(oracle_threshold_table(&c, thr) == 0);
        c.dynamics = ORACLE_DYN_PAPER; c.regrow_pI = 0.002; c.regrow_alpha = 200.0; c.spont = 5e-5;
        CHECK(oracle_threshold_table(&c, thr) == 0);
        free(thr);
    }
    /* benchmark rules, GRU: small windows, a crowded world with a full slot table */
    oracle_config c0 = base(32, 64, 256, 32, 2, 16);
    c0.res_init_p = 0.1; c0.rate_scale = 1.0; c0.T_repr = 20; c0.L_max = 2000;
    resume_case("cfg0", &c0, 0, 300, 150, NULL, 0, -1);
    oracle_config cd = base(40, 72, 300, 200, 3, 32);
    resume_case("dense_h32_r3", &cd, 1, 200, 97, NULL, 0, -1);
    oracle_config c1 = base(17, 33, 250, 150, 1, 16);
    resume_case("dense_h16_r1", &c1, 3, 200, 100, NULL, 0, -1);
    oracle_config full = base(12, 12, 40, 40, 2, 16);
    resume_case("full_slots", &full, 4, 120, 61, NULL, 0, -1);
    /* forced actions by uid: walks into the walls and a stay default */
    int32_t fa[64];
    for (int i = 0; i < 64; ++i) fa[i] = (i % 6) - 1;
    resume_case("forced", &cd, 5, 150, 75, fa, 64, 4);
    /* the paper's network, both rule sets */
    oracle_config cn = base(30, 40, 120, 80, 7, 4);
    cn.controller = ORACLE_CTRL_CNN_LSTM; cn.w_init_gain = 1.0;
    resume_case("network_bench", &cn, 6, 100, 50, NULL, 0, -1);
    oracle_config cp = cn;
    cp.dynamics = ORACLE_DYN_PAPER; cp.E0 = 120; cp.E_max = 120; cp.gain = 40; cp.E_repr = 0; cp.T_repr = 40;
    cp.T_death = 30; cp.L_max = 100; cp.T_repr = 20; cp.spont = 5e-5; cp.regrow_pI = 0.002; cp.regrow_alpha = 200.0;
    cp.rate_top = 0.0; cp.rate_bottom = 0.0;
    resume_case("network_paper", &cp, 7, 120, 59, NULL, 0, -1);
    oracle_config cg = cp;
    cg.controller = ORACLE_CTRL_GRU; cg.obs_radius = 2; cg.hidden = 16; cg.w_init_gain = 0.5;
    resume_case("gru_paper", &cg, 8, 200, 101, NULL, 0, -1);
    /* an empty world and invalid configurations */
    oracle_config ce = base(10, 10, 16, 0, 2, 16);
    resume_case("empty", &ce, 9, 60, 30, NULL, 0, -1);
    char err[256];
    oracle_config bad = base(1, 10, 16, 4, 2, 16);
    CHECK(oracle_create(&bad, 0, err, sizeof err) == NULL);
    bad = base(10, 10, 16, 40, 2, 16);
    CHECK(oracle_create(&bad, 0, err, sizeof err) == NULL);
    puts("ok");
    return 0;
}
