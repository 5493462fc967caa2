/*
 * world.h -- C-ABI of the MI355X (gfx950) world-step library libworld.so.
 *
 * The library advances worlds of the non-episodic neuroevolution simulator of
 * arXiv 2302.09334 on the GPU.  One step of a world is the method of App. B:
 * latitude-dependent resource regrowth (App. B.1, Eq. (1)), per-agent local
 * observation and recurrent controller with individual weights (App. B.2,
 * B.5), moves, eating and the energy update (App. B.2), minimal-criterion
 * reproduction with Gaussian mutation and death (App. B.3), here in the
 * parameterisation of the benchmark workloads (integer energies, one agent
 * per cell).  Two controllers: a GRU cell with a linear head and arg-max
 * actions, or the paper's network (App. B.5: two convolutions with average
 * pooling, an LSTM cell of 4 units, dense layers of 8 and 5) with actions
 * sampled from the softmax at temperature 1/50.
 *
 * Conventions
 *  - Plain C; every function returns an int status: WORLD_OK (0) or a
 *    negative WORLD_E_* code.  No exceptions cross the ABI and nothing aborts.
 *  - Memory: the caller owns the device arena (device memory of at least
 *    world_required_bytes, 256-byte aligned) and the HIP stream; the library
 *    owns only the small host handle.  Host buffers passed to snapshot/load
 *    are owned by the caller and only used during the call.
 *  - Asynchrony: world_create, world_step and world_step_many enqueue work on
 *    the world's stream and return; errors raised by the device surface at
 *    the next synchronising call (world_sync, world_snapshot, ...).
 *  - After a HIP error the handle is poisoned: every later call except
 *    world_destroy returns WORLD_E_POISONED.
 *  - A handle is not thread-safe; distinct handles may be used from
 *    different threads.  Copies and fills run on the world's own stream
 *    (never the legacy default stream, which HIP makes depend on the other
 *    streams).  While another thread launches on a world's stream (and may
 *    capture graphs there), only world_set_stream and world_destroy may be
 *    called for that world: they enqueue nothing and wait for its last launch
 *    in step with this library's graph captures.  Move a world to a stream of
 *    its own before reading it (world_snapshot, world_counters_get, ...).
 */
#ifndef ECO_WORLD_H
#define ECO_WORLD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WORLD_OK 0
#define WORLD_E_INVALID_ARG (-1)       /* NULL pointer, bad K, mismatched worlds */
#define WORLD_E_INVALID_CONFIG (-2)    /* world_config outside the supported range */
#define WORLD_E_BUFFER_TOO_SMALL (-3)  /* arena or host buffer too small */
#define WORLD_E_HIP (-4)               /* HIP runtime or device-side failure */
#define WORLD_E_POISONED (-5)          /* an earlier call failed on the device */
#define WORLD_E_STATE (-6)             /* request outside what the world holds */

/* Execution modes of world_step / world_step_many. */
#define WORLD_MODE_KERNELS 0      /* one launch per phase per step            */
#define WORLD_MODE_GRAPH 1        /* K steps of phase launches in a HIP graph */

/* Controllers (world_config.controller). */
#define WORLD_CTRL_GRU 0        /* GRU + linear head, arg-max of the logits          */
#define WORLD_CTRL_CNN_LSTM 1   /* the paper's network (App. B.5), sampled actions   */
/* Previous action of an agent that has not acted yet (world_image.last_action). */
#define WORLD_NO_ACTION 5

/* Dynamics (world_config.dynamics).
 * WORLD_DYN_BENCH: the benchmark workloads' rules -- one agent per cell (moves
 *   into cells empty at the step start, claims resolved by a random key),
 *   children on a free neighbouring cell, regrowth from the count of
 *   resources among the 24 cells around (rates linear in the row), energy
 *   e - decay + gain * ate without clip, death at e <= 0 or age >= L_max,
 *   reproduction after T_repr consecutive steps with e >= E_repr.
 * WORLD_DYN_PAPER: the rules of App. B -- agents share cells (the paper
 *   network's agent channel counts them); a move into a wall (outside the
 *   grid) kills the agent; on a cell holding a resource the agent with the
 *   smallest random key eats it; e <- min(e - decay + gain * ate, E_max);
 *   a signed streak counts consecutive steps above E_repr (positive) or below
 *   it (negative): reproduction at +T_repr (one child on the parent's own
 *   cell, the streak restarts), death at -T_death or when age > L_max;
 *   regrowth p = p_I c(x) + spont where p_I = regrow_pI when exactly one of
 *   the four direct neighbours holds a resource, c(x) = (alpha^x + 1) /
 *   (alpha + 1), x = row / (H - 1) (App. B.1, Eq. (1)). */
#define WORLD_DYN_BENCH 0
#define WORLD_DYN_PAPER 1

/* Parameters of one world (App. B.4 hyperparameters, benchmark form).
 * Supported: H >= 2, W >= 1, H*W <= 2^26, 1 <= cap <= 2^20,
 * 0 <= n_init <= min(cap, H*W), E0 > 0, decay >= 0, gain >= 0, T_repr >= 1,
 * L_max >= 1, log_steps >= 0; with WORLD_CTRL_GRU obs_radius in 1..3 and
 * hidden in {16, 32}; with WORLD_CTRL_CNN_LSTM obs_radius 7 (the 15 x 15
 * field of view) and hidden 4 (the LSTM's units). */
typedef struct world_config {
    uint32_t struct_size;   /* sizeof(world_config)                               */
    int32_t H, W;           /* grid rows x cols; row 0 = top = slowest regrowth    */
    int32_t cap;            /* agent slots (maximum population)                    */
    int32_t n_init;         /* agents placed at step 0                              */
    int32_t obs_radius;     /* rho: observation window (2 rho + 1)^2                 */
    int32_t hidden;         /* GRU hidden size, or the LSTM's (4)                   */
    double res_init_p;      /* initial resource probability per cell               */
    double rate_bottom;     /* latitude regrowth rate at row H-1                    */
    double rate_top;        /* latitude regrowth rate at row 0                      */
    double rate_scale;      /* multiplier of the latitude rate                      */
    double spont;           /* spontaneous growth probability                       */
    int32_t E0;             /* energy at birth                                      */
    int32_t decay;          /* energy lost per step                                 */
    int32_t gain;           /* energy per resource eaten                            */
    int32_t E_repr;         /* reproduction energy threshold                        */
    int32_t T_repr;         /* consecutive steps at/above E_repr needed to reproduce*/
    int32_t L_max;          /* age of death                                         */
    double sigma_mut;       /* mutation std                                          */
    double w_init_gain;     /* initial weight std = w_init_gain / sqrt(fan_in)       */
    int32_t log_steps;      /* steps of controller log kept on device (0 = none)     */
    uint32_t flags;         /* reserved, must be 0                                    */
    int32_t controller;     /* WORLD_CTRL_*                                           */
    int32_t dynamics;       /* WORLD_DYN_*                                            */
    int32_t E_max;          /* paper dynamics: energy clip (>= E0)                    */
    int32_t T_death;        /* paper dynamics: steps below E_repr before death (>= 1) */
    int32_t pad;
    double regrow_pI;       /* paper dynamics: p_I of Eq. (1)                         */
    double regrow_alpha;    /* paper dynamics: alpha of the climate c(x) (> 0)        */
} world_config;

typedef struct world world_t;

/* Per-step counters kept on device for the last 8192 steps. */
typedef struct world_counters {
    int32_t n_live;      /* live agents after the step          */
    int32_t births;      /* children created in the step        */
    int32_t deaths;      /* agents that died in the step        */
    int32_t eaten;       /* resources eaten in the step         */
    int32_t resources;   /* resources on the grid after regrowth*/
    int32_t claim_wins;  /* birth claims won before the slot cap (0 when the survivors fill the cap) */
    int64_t dead_age_sum;/* sum of the ages of the agents that died in the step
                            (life expectancy over a window, App. C: the sum of
                            this field over the window / the sum of deaths) */
    int32_t seen_resource;/* acting agents with a resource in their field of
                            view at the step start (greediness of the lab
                            environments, Sec. 2.2)                         */
    int32_t rows_read;   /* GRU controller: input-weight rows (3 x hidden
                            floats each) the act phase read in the step --
                            per binary window the rows of its ones, or its
                            column total and the rows of its zeros; 0 for the
                            paper's network.  The bytes a step really reads. */
} world_counters;

/* Movement metric (App. C).  Window k covers steps [k * WORLD_MOVE_WINDOW,
 * (k + 1) * WORLD_MOVE_WINDOW).  An agent counts in window k iff it is alive
 * before the window's first step and after its last step; it falls into bin
 * d / 3 of WORLD_MOVE_BINS, d = Manhattan distance between its cells at the
 * two ends (0..WORLD_MOVE_WINDOW).  A window in progress when a world is
 * created or loaded counts no agent. */
#define WORLD_MOVE_WINDOW 50
#define WORLD_MOVE_BINS 17

#define WORLD_SNAP_HIDDEN 1u   /* fill h, last_action, ate                  */
#define WORLD_SNAP_THETA 2u    /* fill theta (agent_capacity x n_params)    */

/* Canonical host image of a world.  Agents are listed in increasing uid.
 * Recurrent state h: agent_capacity x hidden floats for the GRU; for the
 * paper's network agent_capacity x 8 floats, the LSTM's h (4) then c (4).
 * last_action: the action the agent took in its previous step (0..4) or
 * WORLD_NO_ACTION; ate: 1 if it ate in its previous step (both are inputs of
 * the paper's network and are kept for both controllers).
 * theta uses the genome order.  GRU: W_ih[i][k][g] (inputs x hidden x gates
 * r,z,n), W_hh[j][k][g], b_ih[k][g], b_hh[k][g], W_o[a][k] (5 x hidden),
 * b_o[a].  Paper's network (2445 parameters): conv1 K[ky][kx][ci][co]
 * (3x3x3x4), b[4]; conv2 K[ky][kx][ci][co] (3x3x4x8), b[8]; LSTM input kernel
 * [i][gate][unit] (78x4x4, gates i,f,g,o), hidden kernel [j][gate][unit]
 * (4x4x4), bias [gate][unit]; dense W[i][o] (82x8), b[8]; dense W[o][a]
 * (8x5), b[5]. */
typedef struct world_image {
    uint32_t struct_size;    /* sizeof(world_image)                             */
    uint32_t flags;          /* WORLD_SNAP_* bits                               */
    int64_t step;            /* steps taken                                      */
    int32_t n_live;          /* agents listed                                    */
    uint32_t next_uid;       /* uid the next child receives                      */
    int32_t agent_capacity;  /* length of the per-agent arrays (>= n_live)       */
    int32_t reserved;
    uint8_t *R;              /* H*W resource bits, row-major                     */
    uint32_t *uid;
    int32_t *row, *col, *energy, *age, *streak;
    float *h;
    float *theta;
    uint8_t *last_action;
    uint8_t *ate;
} world_image;

/* Sizes for a configuration (pure host function, no device access):
 * *device_bytes = the arena world_create needs (the whole state of App. B:
 * grid, agents, genomes, lists, counters); *snapshot_bytes = the host bytes
 * of a complete world_image with agent_capacity = cap (R, the six int32
 * agent arrays, h, theta, last_action, ate).  Either pointer may be NULL, not
 * both.  Errors: WORLD_E_INVALID_ARG, WORLD_E_INVALID_CONFIG. */
int world_required_bytes(const world_config *cfg, size_t *device_bytes, size_t *snapshot_bytes);

/* Inputs and parameters per agent for this configuration (GRU: window cells
 * x 2 + energy; paper's network: 15 x 15 x 3 observation values, 2445
 * parameters as App. B.5 counts them).  Pure host; either pointer may be
 * NULL.  Errors: WORLD_E_INVALID_CONFIG. */
int world_dims(const world_config *cfg, int32_t *n_inputs, int32_t *n_params);

/* Lay out a world in `device_arena` (device memory, >= world_required_bytes,
 * 256-byte aligned, owned by the caller and kept alive until world_destroy),
 * initialise it from `seed` on `hip_stream` (a hipStream_t owned by the
 * caller; NULL = default stream) and synchronise the stream.  The initial
 * world is App. B.4's: agents at distinct random cells with energy E0, i.i.d.
 * random resources; the genomes are random (App. B.2: the population starts
 * from random controllers), drawn from the counter-based generator.  *out
 * receives the host handle (owned by the library until world_destroy).
 * Errors: WORLD_E_INVALID_ARG (NULL, misaligned), WORLD_E_INVALID_CONFIG,
 * WORLD_E_BUFFER_TOO_SMALL (arena), WORLD_E_HIP (nothing is created). */
int world_create(const world_config *cfg, uint64_t seed, void *device_arena, size_t arena_bytes,
                 void *hip_stream, world_t **out);

/* Enqueue K >= 1 world steps on the world's stream and return.  One step is
 * App. B in order: observation and controller of every agent (B.2, B.5),
 * moves, eating and energy (B.2), death and minimal-criterion reproduction
 * with mutation (B.3), resource regrowth (B.1, Eq. (1)); the K steps run
 * without a host round trip (App. B.4: one long run, no resets).  Device
 * failures surface at the next synchronising call.  Errors:
 * WORLD_E_INVALID_ARG (K < 1), WORLD_E_POISONED, WORLD_E_HIP. */
int world_step(world_t *w, int32_t K);

/* Enqueue K steps (the step of world_step, App. B) of n worlds in shared
 * launches.  All worlds must use the same stream, controller and dynamics,
 * and no world may be listed twice; the result of every world is
 * bit-identical to stepping it alone.  The library keeps a small device
 * launch table per distinct list (allocated on first use, released by
 * world_destroy of any listed world or by LRU eviction).  Errors:
 * WORLD_E_INVALID_ARG, WORLD_E_POISONED, WORLD_E_HIP. */
int world_step_many(world_t *const *ws, int32_t n, int32_t K);

/* world_step_many for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same steps and results (bit-identical to stepping each world alone),
 * launched as per-phase kernels whatever the worlds' mode, with the batch's
 * launch table written into a fixed device array of the library (48 KB per
 * GPU, held until the process ends) by small kernels whose arguments carry
 * it -- no hipMalloc, hipFree, host-to-device copy or graph instantiation.
 * At most 2048 worlds per call (WORLD_E_INVALID_ARG beyond).  Call it with
 * the worlds' device current.  Every call on one GPU shares the array and
 * rewrites all of it before its kernels read it: calls that overlap on one
 * GPU (other streams or threads) race and must not be issued.  When the
 * stream is being captured into a caller's graph, the launches are recorded
 * into it (each replay then advances the worlds as one such call does) and
 * the caller waits for its replays before moving or releasing the worlds.
 * Errors as world_step_many. */
int world_step_many_noalloc(world_t *const *ws, int32_t n, int32_t K);

/* Select WORLD_MODE_* for later steps (how the App. B step is launched:
 * per-phase kernels, or K steps captured once into a HIP graph and replayed;
 * results are identical).  Errors: WORLD_E_INVALID_ARG. */
int world_set_mode(world_t *w, int32_t mode);

/* Move the world to another HIP stream (caller-owned).  First waits on the
 * host for the last launch that included the world (an event the library
 * records after each launch, polled while no graph capture of this library
 * is in progress), not for other work on the old stream, and enqueues
 * nothing on either stream: another thread may meanwhile launch other worlds
 * on the old stream, capturing graphs through this library (a capture on it
 * by other code must not overlap this call).  Lets a world be created on one
 * stream and then join a batch of world_step_many, and leave it again.
 * Errors: WORLD_E_INVALID_ARG, WORLD_E_POISONED, WORLD_E_HIP. */
int world_set_stream(world_t *w, void *hip_stream);

/* Launch-shape knobs of the step (none changes any result; an autotuner picks
 * them): act_rows = input rows of the controller (App. B.2) fetched per wave
 * per round trip (8, 16 or 32; default 16); act_waves = agents per block of
 * the GRU act kernel (2, 4 or 8; default 4; the paper's network always runs
 * 4); regrow_tile = edge of the square regrowth tiles (App. B.1, Eq. (1);
 * 8, 16 or 32; default 16).  A batched step uses the first world's setting.
 * Synchronises when the shape changes.  Errors: WORLD_E_INVALID_ARG,
 * WORLD_E_POISONED, WORLD_E_HIP. */
int world_set_tuning(world_t *w, int32_t act_rows, int32_t act_waves, int32_t regrow_tile);

/* Wait for the world's stream; report device-side failures (WORLD_E_HIP
 * poisons the handle). */
int world_sync(world_t *w);

/* Synchronise and copy the canonical state (the state App. B's step acts on:
 * grid resources, agents with position, energy, age, reproduction streak,
 * recurrent state and genome) into caller-owned host buffers; any array
 * pointer may be NULL to skip it.  Agents are listed by increasing uid.  If
 * agent_capacity < n_live, returns WORLD_E_BUFFER_TOO_SMALL with n_live set.
 * Errors: WORLD_E_INVALID_ARG, WORLD_E_POISONED, WORLD_E_HIP. */
int world_snapshot(world_t *w, world_image *out);

/* Overwrite the world's state from a canonical image (resume or resync of a
 * long run, App. B.4; both WORLD_SNAP_HIDDEN and WORLD_SNAP_THETA must be set,
 * every array present; the caller keeps `in`).  Validates positions, uids,
 * actions and sizes before touching the device.  Synchronises.  Errors:
 * WORLD_E_INVALID_ARG, WORLD_E_POISONED, WORLD_E_HIP. */
int world_load(world_t *w, const world_image *in);

/* Check, on the host only, that world_load would accept `in` for a world of
 * configuration `cfg`: the full state present, agents inside the grid (one
 * per cell under WORLD_DYN_BENCH), uids increasing and below next_uid, ages
 * >= 0, resource bytes 0 or 1, previous actions 0..5, ate bits 0 or 1.  No
 * device access.  Returns WORLD_OK, WORLD_E_INVALID_CONFIG or
 * WORLD_E_INVALID_ARG (world_last_error(NULL) names the problem). */
int world_validate_image(const world_config *cfg, const world_image *in);

/* Synchronise and copy counters of steps [first_step, first_step + n) into
 * out (caller-owned, n entries): population, births, deaths, resources (the
 * App. C population and resource series) and the per-step sums behind its
 * life expectancy.  The last 8192 steps are held (WORLD_E_STATE otherwise). */
int world_counters_get(world_t *w, int64_t first_step, int32_t n, world_counters *out);

/* Synchronise and copy the movement histograms of windows [first_window,
 * first_window + n): out holds n x (WORLD_MOVE_BINS + 1) int32, the bin
 * counts followed by the number of agents counted.  The windows must have
 * ended and be among the last 64 (WORLD_E_STATE otherwise).  App. C. */
int world_move_hist(world_t *w, int64_t first_window, int32_t n, int32_t *out);

/* Wait for the world's last launch (as world_set_stream does: no stream is
 * synchronised) and release the handle, its graphs and every batch launch
 * table that lists it (after that batch's last launch).  The arena and the
 * stream are not freed (the caller owns them).  NULL is accepted. */
int world_destroy(world_t *w);

/* Message of the last failure of `w` (or of the calling thread if w is NULL). */
const char *world_last_error(const world_t *w);

/* ---- test hooks ----------------------------------------------------------- */

/* Force every agent's action (0 = N, 1 = S, 2 = E, 3 = W, 4 = stay; the
 * actions of App. B.2); -1 returns control to the controller.  Clears the
 * by-uid table of world_set_forced_actions.  Synchronises. */
int world_set_forced_action(world_t *w, int32_t action);

/* Scripted policy by agent (test hook): the agent with uid u takes
 * act_by_uid[u] (0..4) when u < n and that entry is >= 0, otherwise
 * default_action (-1 = its controller's choice).  act_by_uid is a host array
 * of n int32 read during the call; n may be 0 (then act_by_uid may be NULL)
 * and at most max(4 * cap, 4096).  The controller still runs and is logged;
 * only the action taken changes.  Synchronises.  Errors: WORLD_E_INVALID_ARG
 * (n out of range, an action outside -1..4), WORLD_E_POISONED, WORLD_E_HIP. */
int world_set_forced_actions(world_t *w, const int32_t *act_by_uid, int32_t n, int32_t default_action);

/* Failure injection for the look-back scans: from the next step on, move
 * tile `tile` (0 <= tile < ceil(cap / 64); -1 = none) publishes no look-back
 * word, and a wait ends after `spin_ticks` ticks of the 100 MHz wall clock
 * (0 = the default bound of 2 s).  The next tile's wait then times out: the
 * device sets the world's error word and stops stepping it, and the next
 * synchronising call returns WORLD_E_HIP and poisons the handle.  Every wait
 * stays bounded.  Synchronises. */
int world_test_stall_lookback(world_t *w, int32_t tile, uint32_t spin_ticks);

/* Synchronise and copy the controller log of `step` (needs log_steps > 0 and
 * the step among the last log_steps) into caller-owned host arrays of
 * `capacity` entries (any may be NULL): per acting agent in uid order its
 * uid, the action taken and the 5 logits of its controller (App. B.2, B.5),
 * and in margin the device's top-2 margin of its decision values (the
 * logits for the GRU's arg-max; the sampling scores 50 l + g of the paper's
 * network), which a checker uses to recognise near ties.  *n receives the
 * number of agents; WORLD_E_BUFFER_TOO_SMALL if capacity < *n. */
int world_action_log(world_t *w, int64_t step, int32_t capacity, uint32_t *uid, uint8_t *action,
                     float *logits, float *margin, int32_t *n);

/* Philox4x32-10 (Salmon et al., SC'11: the counter-based generator behind
 * every random choice of the step) on the device: n counters (device, n x 4
 * words) under key (k0, k1) into out (device, n x 4 words), on hip_stream.
 * Synchronises hip_stream.  Errors: WORLD_E_INVALID_ARG, WORLD_E_HIP. */
int world_test_philox(const uint32_t *d_ctr, size_t n, uint32_t k0, uint32_t k1, uint32_t *d_out,
                      void *hip_stream);

/* Box-Muller normals on the device from n word pairs (device buffers): the
 * Gaussian of the mutation (App. B.3) and of the initial genomes.
 * Synchronises hip_stream. */
int world_test_gauss(const uint32_t *d_a, const uint32_t *d_b, size_t n, float *d_z0, float *d_z1,
                     void *hip_stream);

/* Gumbel deviates of the paper's action sampling (App. B.2: softmax at
 * temperature 1/50, sampled as the arg-max of 50 l + g) on the device: one
 * per 32-bit word, n words (device) into d_g (device floats), on hip_stream.
 * Synchronises hip_stream. */
int world_test_gumbel(const uint32_t *d_words, size_t n, float *d_g, void *hip_stream);

/* Run K steps as per-phase kernels on the world's stream and return the mean
 * execution time in milliseconds of each phase kernel (start / end events
 * stamped by the kernel's own dispatch, so launch gaps are excluded) in
 * ms[0..2] = act (child genomes of the previous step, observation and
 * controller), move (moves, energy, death, survivor scan, part of the GRU's
 * recurrent projection), claim (birth claims, birth scan, regrowth, the rest
 * of the projection).  The
 * steps are real: the world advances by K.  Synchronises. */
int world_phase_times(world_t *w, int32_t K, float *ms);

/* Plain device-to-device copy kernel (16-byte vector loads/stores) of `bytes`
 * (multiple of 16) between caller-owned device buffers on hip_stream; a
 * known-size reference for memory counters (not part of the method).
 * Synchronises hip_stream. */
int world_test_copy(const void *d_src, void *d_dst, size_t bytes, void *hip_stream);

/* Regrowth threshold table of a configuration, as the library builds it
 * (App. B.1, Eq. (1); out = caller-owned host memory, H x 25 entries indexed
 * [row][resource neighbours]; a cell grows iff its 32-bit draw < entry).
 * Pure host.  Errors: WORLD_E_INVALID_ARG, WORLD_E_INVALID_CONFIG. */
int world_threshold_table(const world_config *cfg, uint64_t *out);

#ifdef __cplusplus
}
#endif
#endif
