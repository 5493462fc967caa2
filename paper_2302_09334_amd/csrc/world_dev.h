// world_dev.h -- device-side description of one world and its arena layout.
//
// Everything a kernel needs about a world is reachable from one WorldDev
// record that lives in the world's own arena, so a launch over one or many
// worlds only passes pointers to these records.
//
// HBM layout (structure of arrays, every array 256-byte aligned):
//   grid      R[2] (u8, double-buffered for the synchronous regrowth),
//             occA/occB (i32 slot or -1; occA = state at the step start,
//             read by the act phase; occB = state after moves and deaths,
//             read by the claim phase; children enter occA when they are
//             born and occB when they are created); under the paper's
//             dynamics occA holds the number of agents on the cell minus one
//             (so -1 is still "empty") and occB is unused,
//             thr (u64 H x 25 regrowth thresholds)
//   agents    uid, cell, prev_cell, energy, age, streak (i32 per slot),
//             action (the last one taken), alive, ate (u8), claim (i32),
//             h (f32 slot x state: the GRU's h, or the LSTM's h then c),
//             theta (f32 slot x Ppad, the genome order; for the GRU each
//             input's 3*hidden gate weights are contiguous so that skipping
//             a zero input skips one contiguous row)
//   lists     live[2] (slots in uid order), freeq (ring of free slots),
//             child (per step: child slot, parent slot, cell, uid)
//   scalars   WorldScal, counters ring (8192 steps), optional controller log
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace eco {

constexpr int kRing = 8192;     // steps of counters kept on device
constexpr int kCtrWords = 10;   // words per counter record
constexpr int kBlock = 256;     // threads per block in every kernel
constexpr uint32_t kSpinTicks = 200000000u;   // look-back wait bound: 2 s at the 100 MHz wall clock

// Counter record fields (match world_counters in world.h).
enum : int { kCtrLive = 0, kCtrBirths, kCtrDeaths, kCtrEaten, kCtrRes, kCtrWins, kCtrDeadAgeLo, kCtrDeadAgeHi,
             kCtrSeen, kCtrRows };

// The act phase marks in the agent record's action word whether the agent had
// a resource in its field of view (greediness of the lab environments, Sec.
// 2.2); the move phase counts and strips the mark.
constexpr int kSeenBit = 1 << 8;
constexpr int kActMask = 0xFF;
// The GRU act phase also stores there how many input rows of W_ih it read
// (window rows and window totals, at most 2 * 25); the move phase sums them
// per step into the counter ring (the bytes the step really read).
constexpr int kRowsShift = 9;
constexpr int kRowsMask = 0x7F;

// Movement metric (App. C): windows of kMoveWin steps (window k covers steps
// [k * kMoveWin, (k + 1) * kMoveWin)), distances binned by 3 into kMoveBins
// bins; the last kMoveRing windows are kept, kMoveBins counts and the number
// of agents counted per window.
constexpr int kMoveWin = 50;
constexpr int kMoveBins = 17;
constexpr int kMoveRing = 64;

// Controllers and dynamics.
enum : int { kCtrlGru = 0, kCtrlNet = 1 };
enum : int { kDynBench = 0, kDynPaper = 1 };
constexpr int kNoAction = 5;   // previous action of an agent that has not acted yet

// Agent record by live-list position (the order of the live list): what the
// act and move phases need about an agent in one 32-byte read.  `action` is
// the previous step's action until the act phase overwrites it with this
// step's; `ate` says whether the agent ate in its previous step.
struct alignas(16) AgentRec {
    int32_t slot, cell, energy;
    uint32_t uid;
    int32_t age, streak, action, ate;
};

// Post-move record by live-list position, for the claim phase (next_pos =
// the survivor's position in the next live list, -1 for the dead).
struct alignas(16) PostRec {
    int32_t slot, prev_cell, cell, alive;
    int32_t streak, action;
    uint32_t uid;
    int32_t next_pos;
};

// Everything about live-list position i, together: the agent's record in
// each of the two live lists and its post-move record.
struct alignas(32) PosRec {
    AgentRec r[2];
    PostRec post;
};

// Read-only views of memory that no kernel writes while the reader runs
// (descriptors, launch tables, scalars of an earlier kernel): loads through a
// constant-address-space pointer are scalar loads when the address is uniform.
#define ECO_KAS __attribute__((address_space(4)))
template <class T>
using kptr = const ECO_KAS T*;
template <class T>
__device__ __forceinline__ kptr<T> kconst(const T* p) {
    return (kptr<T>)p;
}

struct WorldScal {
    int64_t t;          // steps taken
    int32_t n_live;
    uint32_t next_uid;
    int32_t free_head;  // ring of free slots: [head, head + n_free) mod cap
    int32_t free_tail;
    int32_t live_sel;   // which live[] buffer is current
    int32_t n_child;    // children created by the last step
    int64_t spawn_t;    // step of the pending children
    int32_t err;        // device-side failure code (2 look-back time-out)
    int32_t n_prev;     // live agents at the start of the last closed step
    int32_t ctr_open;   // 1: eaten/resource totals of step spawn_t not yet summed
    int32_t n_grow;     // live agents of the running claim phase's step (written by its move phase)
    int64_t t_grow;     // step of the running claim phase (written by its move phase)
    int32_t n_surv;     // survivors of the running step's move phase (written by its last tile)
    int32_t pad_surv;
};

struct WorldDev {
    // configuration
    int32_t H, W, cap, rho, hd, n_in, P, Ppad;
    int32_t E0, decay, gain, E_repr, T_repr, L_max;
    float sigma;
    uint32_t seed_lo, seed_hi;
    int32_t forced;     // forced action of every agent not in forced_tab, or -1 (the controller decides)
    int32_t n_forced;   // entries of forced_tab (forced action by uid, -1 = use `forced`)
    int32_t forced_on;  // forced >= 0 || n_forced > 0
    int32_t log_steps;
    int32_t off_hh, off_bih, off_bhh, off_wo, off_bo;  // genome offsets (floats)
    int32_t nblk;       // float4 blocks per genome, ceil(P / 4)
    int32_t tot_row;    // theta row (of 3*hd floats) of the window totals, after the genome; tot_row + 2 is zeros
    int32_t ctrl;       // kCtrlGru or kCtrlNet
    int32_t ss;         // recurrent state floats per slot (hd for the GRU, 2 hd for the LSTM)
    int32_t dyn;        // kDynBench or kDynPaper
    int32_t E_max, T_death;   // paper dynamics
    int32_t stall_tile;       // test hook: move tile that publishes no look-back word (-1: none)
    uint32_t spin_ticks;      // bound of a look-back wait, in 100 MHz wall-clock ticks
    // grid
    uint8_t* R[2];
    int32_t* occA;
    int32_t* occB;
    const uint64_t* thr;
    uint64_t* mclaim;     // per cell: smallest move-claim key of the step (~0 = none)
    // agents
    uint32_t* uid;
    int32_t* cell;
    int32_t* prev_cell;
    int32_t* energy;
    int32_t* age;
    int32_t* streak;
    uint8_t* action;
    uint8_t* alive;
    uint8_t* ate;         // per slot: ate in its last step
    int32_t* claim;
    uint64_t* bkey;       // birth-claim key by cell of eligible agents (written in P2)
    float* h;
    float* gh;            // recurrent projection W_hh h + b_hh for the next act (slot x 3 hidden)
    float* theta;
    // lists
    int32_t* live[2];
    PosRec* pos;          // per-position records (at kPosOff from the descriptor)
    int32_t* freeq;
    int4* child;
    // scalars and logs
    WorldScal* scal;
    int32_t* ring;        // kRing x kCtrWords
    uint32_t* log_uid;    // log_steps x cap
    uint8_t* log_act;     // log_steps x cap
    float* log_logits;    // log_steps x cap x 5
    int32_t* log_n;       // log_steps
    int32_t* deadlist;    // slots of the agents that died this step, uid order
    uint64_t* lb_move;    // look-back status words of the move phase (per tile)
    uint64_t* lb_claim;   // look-back status words of the claim phase (per tile)
    int32_t* eat_part;    // per-wave eaten counts | seen counts << 16 of the move phase (cap / 64)
    int32_t* dage_part;   // per-wave sums of the ages of the dead (cap / 64)
    int32_t* wcell;       // per slot: cell at the start of the current movement window
    uint32_t* wuid;       // per slot: uid of the agent the window start was recorded for
    int32_t* mhist;       // kMoveRing x (kMoveBins + 1) movement histograms
    int32_t* res_part;    // per-tile resource counts of the regrowth phase (room for the smallest tile edge)
    int32_t* rows_part;   // per-wave sums of the input rows read by the act phase (cap / 64)
    int32_t* res_ntiles;  // regrowth tiles (resource partials) of the last claim phase
    const int8_t* forced_tab;   // test hook: forced action by uid (n_forced entries)
    int32_t pad1, pad2;
};

// A world's arena starts with its descriptor; the scalars and the
// per-position records follow at fixed offsets, so a kernel that knows the
// descriptor's address reaches them without reading the descriptor first.
constexpr size_t kArenaAlign = 256;
constexpr size_t arena_round(size_t v) { return (v + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }
constexpr size_t kScalOff = arena_round(sizeof(WorldDev));
constexpr size_t kPosOff = kScalOff + arena_round(sizeof(WorldScal));

// A world descriptor as the kernels see it: written by the host only, read
// through the constant address space.
using DevRef = const ECO_KAS WorldDev&;

}  // namespace eco
