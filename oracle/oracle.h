/*
 * oracle.h -- plain CPU reference of the non-episodic neuroevolution world
 * step (arXiv 2302.09334, App. B).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links
 * or calls this code; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load liboracle.so.  It shares no header,
 * helper, table or constant generator with the GPU path: both sides are
 * written independently against the same written semantics.
 *
 * Everything here is deliberately slow and literal: floating point for the
 * controller is IEEE double, loops follow the definitions, and no step is
 * blocked, fused or reordered.
 */
#ifndef ECO_ORACLE_H
#define ECO_ORACLE_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Parameters of one world.  Field meanings follow App. B.4 (hyperparameters)
 * in the parameterisation of the benchmark workloads (integer energies). */
typedef struct oracle_config {
    int32_t H, W;          /* grid rows x cols; row 0 is the top (lowest regrowth) */
    int32_t cap;           /* maximum number of live agents                       */
    int32_t n_init;        /* agents placed at step 0                              */
    int32_t obs_radius;    /* rho: observation window is (2 rho + 1)^2             */
    int32_t hidden;        /* GRU hidden size                                      */
    double  res_init_p;    /* initial Bernoulli resource probability               */
    double  rate_bottom;   /* regrowth rate at row H-1                             */
    double  rate_top;      /* regrowth rate at row 0                               */
    double  rate_scale;    /* multiplier on the latitude rate                      */
    double  spont;         /* spontaneous growth probability (the constant c)      */
    int32_t E0;            /* energy at birth                                      */
    int32_t decay;         /* energy lost per step                                 */
    int32_t gain;          /* energy gained per resource eaten                     */
    int32_t E_repr;        /* reproduction energy threshold                        */
    int32_t T_repr;        /* consecutive steps at or above E_repr to reproduce    */
    int32_t L_max;         /* age at which an agent dies                           */
    double  sigma_mut;     /* std of the Gaussian weight mutation                  */
    double  w_init_gain;   /* initial weight std = gain / sqrt(fan_in)             */
    int32_t controller;    /* ORACLE_CTRL_GRU or ORACLE_CTRL_CNN_LSTM              */
    int32_t dynamics;      /* ORACLE_DYN_BENCH or ORACLE_DYN_PAPER                 */
    int32_t E_max;         /* paper dynamics: energy clip                          */
    int32_t T_death;       /* paper dynamics: steps below E_repr before death      */
    int32_t pad;
    double  regrow_pI;     /* paper dynamics: p_I of Eq. (1)                       */
    double  regrow_alpha;  /* paper dynamics: alpha of the climate c(x)            */
} oracle_config;

/* Dynamics.  BENCH: the benchmark workloads' rules (one agent per cell, move
 * and birth claims, regrowth from the 24-cell neighbourhood, no energy clip,
 * death at energy <= 0).  PAPER: the rules of App. B (stacking, walls that
 * kill, offspring on the parent's cell, regrowth p = p_I 1[one of the four
 * neighbours holds a resource] c(x) + c with c(x) = (alpha^x + 1)/(alpha + 1),
 * energy clipped at E_max, reproduction after T_repr steps above E_repr and
 * death after T_death steps below it or past L_max). */
#define ORACLE_DYN_BENCH 0
#define ORACLE_DYN_PAPER 1

/* Controllers.  GRU: the benchmark workloads' GRU cell with a linear head,
 * actions by arg-max.  CNN_LSTM: the paper's network (App. B.5) over the
 * 15 x 15 x 3 observation (obs_radius 7, hidden 4), actions sampled from the
 * softmax at temperature 1/50. */
#define ORACLE_CTRL_GRU 0
#define ORACLE_CTRL_CNN_LSTM 1
/* "No previous action" (an agent that has not acted yet). */
#define ORACLE_NO_ACTION 5

/* Result of one oracle step. */
typedef struct oracle_stepinfo {
    int32_t n_live;      /* live agents after the step                         */
    int32_t births;      /* children created                                   */
    int32_t deaths;      /* agents removed                                     */
    int32_t eaten;       /* resources consumed                                 */
    int32_t resources;   /* resources on the grid after regrowth               */
    int32_t resyncs;     /* near-tie actions adopted from the supplied hints   */
    int32_t mismatches;  /* hints that disagreed outside the near-tie band     */
    int32_t claim_wins;  /* birth-claim winners before the slot cap (0 when no
                            slot is free: no claim is made)                   */
    int64_t dead_age;    /* sum of the ages of the agents that died (App. C)   */
    int32_t seen;        /* acting agents with a resource in their field of view
                            at the step start (greediness, Sec. 2.2)          */
    int32_t pad;
} oracle_stepinfo;

/* Movement metric (App. C): windows of ORACLE_MOVE_WINDOW steps, window k
 * covering steps [k * W, (k + 1) * W).  For every agent alive at both the
 * start of the window (before its first step) and its end (after its last
 * step, deaths applied), the Manhattan distance between the two positions
 * (0..W) falls into bin distance / 3 of ORACLE_MOVE_BINS bins. */
#define ORACLE_MOVE_WINDOW 50
#define ORACLE_MOVE_BINS 17

/* Random stream identifiers of the counter-based generator. */
enum {
    ORACLE_S_INIT_RES = 1,
    ORACLE_S_INIT_PLACE = 2,
    ORACLE_S_INIT_W = 3,
    ORACLE_S_MOVE = 4,
    ORACLE_S_BIRTH = 5,
    ORACLE_S_MUTATE = 6,
    ORACLE_S_REGROW = 7,
    ORACLE_S_ACT = 8,
    ORACLE_S_EAT = 9
};

/* ---- primitives (exposed so that tests can pin them one by one) ---------- */

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) on n counters.
 * ctr: n x 4 words, key: 2 words, out: n x 4 words. */
void oracle_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out, size_t n);

/* Natural log of u in (0, 1] in single precision (project definition). */
void oracle_ln_unit(const float *u, float *out, size_t n);
/* sin and cos of 2*pi*u for dyadic u in [0, 1) (project definition). */
void oracle_sincos_2pi(const float *u, float *s, float *c, size_t n);
/* Box-Muller: two standard normals from two 32-bit words, n pairs. */
void oracle_gauss_pair(const uint32_t *a, const uint32_t *b, float *z0, float *z1, size_t n);

/* Number of inputs, parameters, and the parameter offsets of the genome. */
int32_t oracle_n_inputs(int32_t obs_radius);
int32_t oracle_n_params(int32_t obs_radius, int32_t hidden);

/* Regrowth threshold table, H x 25 entries: grow iff draw < table[row*25+n]. */
int oracle_threshold_table(const oracle_config *cfg, uint64_t *out);

/* One GRU controller evaluation in double (used to pin the gate convention).
 * theta: genome (n_params floats), x: inputs, h: hidden (float),
 * h_out: new hidden (double), logits: 5 doubles. */
void oracle_gru_eval(int32_t n_in, int32_t hidden, const float *theta, const double *x,
                     const float *h, double *h_out, double *logits);

/* The paper's controller (App. B.5).  n_params is 2445, n_features 72.
 * obs: 15 x 15 x 3 (row, column, channel: resource, agents, wall);
 * prev_action 0..4 or ORACLE_NO_ACTION; h, c: 4 floats each. */
int32_t oracle_cnn_n_params(void);
int32_t oracle_cnn_n_features(void);
void oracle_cnn_eval(const float *theta, const double *obs, int32_t prev_action, int32_t ate,
                     const float *h, const float *c, double *h_out, double *c_out, double *logits);
/* Standard Gumbel deviates from generator words (the sampling reading). */
void oracle_gumbel(const uint32_t *words, float *g, size_t n);
/* Sampled action of agent `uid` at `step` from single-precision logits; the
 * five sampling scores go to `scores` (may be NULL). */
int32_t oracle_sample_action(uint64_t seed, uint32_t uid, uint32_t step, const float *logits, float *scores);

/* ---- the world ------------------------------------------------------------ */

void *oracle_create(const oracle_config *cfg, uint64_t seed, char *err, size_t errlen);
void  oracle_destroy(void *w);

/* Force actions by uid: act[u] in 0..4 forces agent u; -1 (or uid >= n) uses
 * `dflt`; dflt = -1 means the controller decides. Pass n = 0 to clear. */
void oracle_set_forced(void *w, const int32_t *act, int32_t n, int32_t dflt);

/* Advance one step.  hint_uid/hint_act (sorted by uid, may be NULL) are the
 * actions another implementation took; where this oracle's own top logits are
 * closer than 1e-5 * max(1, |top|) the hinted action is adopted (resync). */
int oracle_step(void *w, const uint32_t *hint_uid, const uint8_t *hint_act, int32_t n_hint,
                oracle_stepinfo *info);

int64_t  oracle_t(const void *w);
int32_t  oracle_n_live(const void *w);
uint32_t oracle_next_uid(const void *w);

/* Copy out the state.  Agents are in uid order.  Any pointer may be NULL. */
void oracle_get_grid(const void *w, uint8_t *R);
void oracle_get_agents(const void *w, uint32_t *uid, int32_t *row, int32_t *col,
                       int32_t *energy, int32_t *age, int32_t *streak);
void oracle_get_hidden(const void *w, float *h);          /* n_live x state: h (GRU); h then c (LSTM) */
/* Overwrite the state (the canonical image: agents in increasing uid, genomes
 * in genome order, recurrent state h (and c), previous action, ate bit).  A
 * movement window in progress counts no agent afterwards.  Returns 0, or -1 on
 * an invalid image (positions, order, sizes). */
int oracle_load(void *w, int64_t step, int32_t n, uint32_t next_uid, const uint8_t *R, const uint32_t *uid,
                const int32_t *row, const int32_t *col, const int32_t *energy, const int32_t *age,
                const int32_t *streak, const float *h, const float *theta, const uint8_t *last_action,
                const uint8_t *ate);

/* Previous action (0..4, ORACLE_NO_ACTION) and whether the agent ate in its
 * previous step, per live agent. */
void oracle_get_recurrent_inputs(const void *w, uint8_t *last_action, uint8_t *ate);
/* Observation of the paper's controller for live agent `a` (uid order). */
int oracle_get_obs_cnn(const void *w, int32_t a, double *obs);
void oracle_get_theta(const void *w, float *theta);       /* n_live x n_params      */
/* Controller outputs of the last step, for the agents that acted in it (uid
 * order, the population at the start of that step). */
int32_t oracle_last_n_acted(const void *w);
void oracle_get_last_logits(const void *w, uint32_t *uid, double *logits, uint8_t *action);
/* Movement windows that have ended, and the histogram of window k:
 * bins[ORACLE_MOVE_BINS] and the number of agents counted. */
int32_t oracle_n_move_windows(const void *w);
int oracle_get_move_hist(const void *w, int32_t k, int32_t *bins, int32_t *count);

#ifdef __cplusplus
}
#endif
#endif
