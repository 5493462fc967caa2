// world.hip -- host side of libworld.so: configuration checks, arena layout,
// initialisation, step launches (per-phase kernels, HIP graphs, persistent
// cooperative kernel), snapshots and the C-ABI of include/world.h.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cassert>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "world.h"
#include "kernels.h"

using namespace eco;

namespace {

thread_local std::string g_thread_err;

// A roctx range around one call of the C-ABI (rocprofv3 --marker-trace shows
// them beside the kernels: one range per K-step chunk, snapshot or load).
struct TraceRange {
    explicit TraceRange(const char* what) { roctxRangePushA(what); }
    TraceRange(const char* fmt, int a, int b = 0) {
        char msg[96];
        std::snprintf(msg, sizeof(msg), fmt, a, b);
        roctxRangePushA(msg);
    }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

constexpr size_t kAlign = 256;

size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

int n_inputs_of(int rho) {
    const int w = 2 * rho + 1;
    return 2 * w * w + 1;
}

struct Dims {
    int n_in, P, Ppad, off_hh, off_bih, off_bhh, off_wo, off_bo, nblk, tot_row;
};

bool is_net(const world_config& c) { return c.controller == WORLD_CTRL_CNN_LSTM; }

// Recurrent state floats per agent: the GRU's h, or the LSTM's h and c.
int state_of(const world_config& c) { return is_net(c) ? 2 * c.hidden : c.hidden; }

Dims dims_of(const world_config& c) {
    Dims d;
    if (is_net(c)) {
        std::memset(&d, 0, sizeof(d));
        d.n_in = net::kPix * 3;
        d.P = net::kP;
        d.Ppad = int(align_up(size_t(d.P), 64));
        d.nblk = (d.P + 3) / 4;
        return d;
    }
    d.n_in = n_inputs_of(c.obs_radius);
    const int hd = c.hidden;
    d.off_hh = d.n_in * hd * 3;
    d.off_bih = d.off_hh + hd * hd * 3;
    d.off_bhh = d.off_bih + hd * 3;
    d.off_wo = d.off_bhh + hd * 3;
    d.off_bo = d.off_wo + 5 * hd;
    d.P = d.off_bo + 5;
    // after the genome, at a whole number of input rows: the two window totals
    // of the input weights (rows tot_row, tot_row + 1) and a row of zeros
    // (tot_row + 2, never written after the arena is cleared), then padding to
    // 256 bytes
    d.tot_row = (d.P + 3 * hd - 1) / (3 * hd);
    d.Ppad = int(align_up(size_t(d.tot_row + 3) * 3 * hd, 64));
    d.nblk = (d.P + 3) / 4;
    return d;
}

const char* check_config(const world_config* c) {
    if (!c) return "config is NULL";
    if (c->struct_size != sizeof(world_config)) return "world_config.struct_size mismatch";
    if (c->H < 2 || c->W < 1) return "grid must be at least 2 x 1";
    if (int64_t(c->H) * c->W > (int64_t(1) << 26)) return "grid larger than 2^26 cells";
    if (c->cap < 1 || c->cap > (1 << 20)) return "cap must be in 1..2^20";
    if (c->n_init < 0 || c->n_init > c->cap || int64_t(c->n_init) > int64_t(c->H) * c->W)
        return "n_init must be in 0..min(cap, H*W)";
    if (c->controller == WORLD_CTRL_CNN_LSTM) {
        if (c->obs_radius != net::kRho) return "the paper's network needs obs_radius 7";
        if (c->hidden != net::kHd) return "the paper's network needs hidden 4";
    } else if (c->controller == WORLD_CTRL_GRU) {
        if (c->obs_radius < 1 || c->obs_radius > 3) return "obs_radius must be 1..3";
        if (c->hidden != 16 && c->hidden != 32) return "hidden must be 16 or 32";
    } else {
        return "unknown controller";
    }
    if (c->E0 <= 0 || c->decay < 0 || c->gain < 0) return "E0 > 0, decay >= 0, gain >= 0 required";
    if (c->T_repr < 1 || c->L_max < 1) return "T_repr and L_max must be positive";
    if (c->log_steps < 0) return "log_steps must be >= 0";
    if (c->dynamics != WORLD_DYN_BENCH && c->dynamics != WORLD_DYN_PAPER) return "unknown dynamics";
    if (c->dynamics == WORLD_DYN_PAPER &&
        (c->E_max < c->E0 || c->T_death < 1 || !(c->regrow_alpha > 0.0) || !std::isfinite(c->regrow_alpha) ||
         !std::isfinite(c->regrow_pI)))
        return "paper dynamics need E_max >= E0, T_death >= 1 and a finite alpha > 0";
    if (c->flags != 0) return "flags must be 0";
    if (!std::isfinite(c->res_init_p) || !std::isfinite(c->rate_bottom) || !std::isfinite(c->rate_top) ||
        !std::isfinite(c->rate_scale) || !std::isfinite(c->spont) || !std::isfinite(c->sigma_mut) ||
        !std::isfinite(c->w_init_gain))
        return "non-finite parameter";
    return nullptr;
}

// Entries of the forced-action table by uid (a test hook for scripted
// policies): uids at or beyond it take the world's default.
int32_t forced_capacity(const world_config& c) { return std::max(4 * c.cap, 4096); }

// Host bytes of a complete canonical image with agent_capacity = cap.
size_t snapshot_bytes_of(const world_config& c, const Dims& dm) {
    const size_t cap = size_t(c.cap);
    return size_t(c.H) * c.W + cap * (6 * 4 + 4 * size_t(state_of(c)) + 4 * size_t(dm.P) + 2);
}

// Byte offsets of every array inside the arena.
struct Layout {
    size_t desc, scal, ring, batch, thr, R0, R1, occA, occB, mclaim;
    size_t uid, cell, prev_cell, energy, age, streak, action, alive, ate, claim, bkey;
    size_t live0, live1, pos, freeq, child, h, gh, theta;
    size_t log_uid, log_act, log_logits, log_n, eat_part, dage_part, rows_part, wcell, wuid, mhist, res_part, deadlist,
        lb_move, lb_claim, forced, res_ntiles;
    size_t total;
};

Layout layout_of(const world_config& c) {
    const Dims dm = dims_of(c);
    const size_t HW = size_t(c.H) * c.W;
    const size_t cap = size_t(c.cap);
    const size_t L = size_t(c.log_steps);
    Layout l;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    l.desc = take(sizeof(WorldDev));
    l.scal = take(sizeof(WorldScal));
    l.pos = take(sizeof(PosRec) * cap);
    l.ring = take(sizeof(int32_t) * kRing * kCtrWords);
    l.batch = take(256);   // single-world launch table
    l.thr = take(sizeof(uint64_t) * size_t(c.H) * 25);
    l.R0 = take(HW);
    l.R1 = take(HW);
    l.occA = take(4 * HW);
    l.occB = take(4 * HW);
    l.mclaim = take(8 * HW);
    l.bkey = take(8 * HW);
    l.uid = take(4 * cap);
    l.cell = take(4 * cap);
    l.prev_cell = take(4 * cap);
    l.energy = take(4 * cap);
    l.age = take(4 * cap);
    l.streak = take(4 * cap);
    l.action = take(cap);
    l.alive = take(cap);
    l.ate = take(cap);
    l.claim = take(4 * cap);
    l.live0 = take(4 * cap);
    l.live1 = take(4 * cap);
    l.freeq = take(4 * cap);
    l.child = take(16 * cap);
    l.h = take(4 * cap * size_t(state_of(c)));
    l.gh = take(is_net(c) ? 0 : 4 * cap * 3 * size_t(c.hidden));
    l.theta = take(4 * cap * size_t(dm.Ppad));
    l.log_uid = take(4 * L * cap);
    l.log_act = take(L * cap);
    l.log_logits = take(4 * 5 * L * cap);
    l.log_n = take(4 * L);
    l.eat_part = take(4 * (cap / 64 + 1));
    l.dage_part = take(4 * (cap / 64 + 1));
    l.rows_part = take(4 * (cap / 64 + 1));
    l.wcell = take(4 * cap);
    l.wuid = take(4 * cap);
    l.mhist = take(4 * size_t(kMoveRing) * (kMoveBins + 1));
    l.deadlist = take(4 * cap);
    l.lb_move = take(8 * ((cap + kTileN - 1) / kTileN));
    l.lb_claim = take(8 * ((cap + kTileN - 1) / kTileN));
    l.res_part = take(4 * size_t(((c.H + kTileMin - 1) / kTileMin) * ((c.W + kTileMin - 1) / kTileMin)));
    l.res_ntiles = take(4);
    l.forced = take(size_t(forced_capacity(c)));
    l.total = o;
    static_assert(kArenaAlign == kAlign, "arena alignment");
    assert(l.scal == kScalOff && l.pos == kPosOff);
    return l;
}

// Regrowth thresholds (App. B.1, Eq. (1) in the workload parameterisation):
// p(row, n) = (rate_top + (rate_bottom - rate_top) * row / (H - 1)) * scale
//             * n / 24 + spont, grow iff draw < floor(p * 2^32), IEEE double.
uint64_t threshold_of(double p) {
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return uint64_t(1) << 32;
    return uint64_t(std::floor(p * 4294967296.0));
}

void build_thresholds(const world_config& c, uint64_t* out) {
    if (c.dynamics == WORLD_DYN_PAPER) {
        // App. B.1, Eq. (1): entry n = the number of the four direct
        // neighbours holding a resource; p_I applies when it is exactly one
        for (int row = 0; row < c.H; ++row) {
            const double x = double(row) / double(c.H - 1);
            const double climate = (std::pow(c.regrow_alpha, x) + 1.0) / (c.regrow_alpha + 1.0);
            for (int n = 0; n <= 24; ++n) out[row * 25 + n] = threshold_of((n == 1 ? c.regrow_pI : 0.0) * climate + c.spont);
        }
        return;
    }
    for (int row = 0; row < c.H; ++row) {
        const double span = c.rate_bottom - c.rate_top;
        const double lat = (span * double(row)) / double(c.H - 1);
        const double rate = (c.rate_top + lat) * c.rate_scale;
        for (int n = 0; n <= 24; ++n) {
            const double q = (rate * double(n)) / 24.0;
            out[row * 25 + n] = threshold_of(q + c.spont);
        }
    }
}

// Initial weight spread by parameter range (App. B.2: random at the start):
// std = w_init_gain / sqrt(fan_in) for the weights, 0 for the biases.
InitSegs init_segments(const world_config& c, const Dims& dm) {
    InitSegs g;
    std::memset(&g, 0, sizeof(g));
    auto add = [&](int end, int fan_in) {
        g.end[g.n] = end;
        g.sd[g.n] = fan_in > 0 ? float(c.w_init_gain / std::sqrt(double(fan_in))) : 0.f;
        g.n++;
    };
    if (is_net(c)) {
        using namespace net;
        add(kC1b, 9 * 3);           // conv1 kernel
        add(kC2w, 0);
        add(kC2b, 9 * kF1);         // conv2 kernel
        add(kLwi, 0);
        add(kLwh, kEmb);            // LSTM input kernel
        add(kLb, kHd);              // LSTM hidden kernel
        add(kD8w, 0);
        add(kD8b, kCat);            // dense 8
        add(kD5w, 0);
        add(kD5b, kD);              // dense 5
        add(kP, 0);
    } else {
        add(dm.off_hh, dm.n_in);    // W_ih
        add(dm.off_bih, c.hidden);  // W_hh
        add(dm.off_wo, 0);          // b_ih, b_hh
        add(dm.off_bo, c.hidden);   // W_o
        add(dm.P, 0);               // b_o
    }
    return g;
}

}  // namespace

// The end of a launch: an event recorded on the launch stream right after
// it.  Released with its last holder.
struct WorkEvent {
    hipEvent_t ev = nullptr;
    ~WorkEvent() {
        if (ev) (void)hipEventDestroy(ev);
    }
};

struct world {
    world_config cfg;
    Dims dm;
    Layout lay;
    uint64_t seed;
    char* base;            // device arena
    WorldDev dev;          // host copy of the descriptor
    WorldDev* d_dev;       // device address of the descriptor
    struct {
        const WorldDev* const* w;
        const int* block_pre;
        int slots;
        int may_stream;
    } tv;                  // single-world launch table (inside the arena)
    std::vector<int> host_bp;
    int max_useful = 1;
    hipStream_t stream;
    int mode = WORLD_MODE_KERNELS;
    int act_rows = 16;     // act-kernel tuning knob (8, 16, 32)
    int act_waves = 4;     // agents per GRU act block (2, 4, 8)
    int tile = 16;         // regrowth tile edge (8, 16, 32)
    bool poisoned = false;
    std::string err;
    std::map<int, hipGraphExec_t> graphs;
    std::map<int, hipGraph_t> graph_defs;
    // Completion of this world's launches: `own` is recorded after each
    // launch the world leads (alone, or first of a batch); `last` is the
    // event recorded after the last launch that included the world (a batch
    // leader's `own`), null when nothing is pending.  Moving or releasing a
    // world waits for `last` (wait_launch) instead of synchronising a stream
    // that another thread may be launching on.
    std::shared_ptr<WorkEvent> own;
    std::shared_ptr<WorkEvent> last;
};

namespace {

int fail(world* w, int code, const std::string& msg) {
    if (w) {
        w->err = msg;
        if (code == WORLD_E_HIP) w->poisoned = true;
    } else {
        g_thread_err = msg;
    }
    return code;
}

#define HIP_TRY(w, expr)                                                              \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail((w), WORLD_E_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

// Agent blocks of the act phase: `waves` agents per block (the paper's
// network always runs four per block).
int blocks_act(const world_config& c, int waves) {
    const int per = is_net(c) ? kBlock / 64 : waves;
    return (c.cap + per - 1) / per;
}
int blocks_of_agents(const world_config& c) { return (c.cap + kBlock / 64 - 1) / (kBlock / 64); }   // 4 per block
int tiles_agent(const world_config& c) { return (c.cap + kTileN - 1) / kTileN; }   // move / claim tiles
int tiles_of(const world_config& c, int tile) { return ((c.H + tile - 1) / tile) * ((c.W + tile - 1) / tile); }

// Host table of block prefixes for a batch of worlds (kPreKinds x (n + 1)).
std::vector<int> batch_prefix(const std::vector<const world*>& ws, int waves, int tile) {
    const int n = int(ws.size());
    std::vector<int> pre(size_t(kPreKinds) * (n + 1), 0);
    for (int i = 0; i < n; ++i) {
        const world_config& c = ws[i]->cfg;
        pre[kPreAct * (n + 1) + i + 1] = pre[kPreAct * (n + 1) + i] + newborn_blocks(c.cap) + blocks_act(c, waves);
        pre[kPreMove * (n + 1) + i + 1] =
            pre[kPreMove * (n + 1) + i] + tiles_agent(c) + (is_net(c) ? 0 : proj_waves_move(c.cap));
        // GRU worlds add the recurrent-projection blocks to the claim phase
        pre[kPreClaim * (n + 1) + i + 1] =
            pre[kPreClaim * (n + 1) + i] + tiles_agent(c) + tiles_of(c, tile) + (is_net(c) ? 0 : proj_waves(c.cap));
    }
    return pre;
}

// The GRU act kernel for the batch's rows per round trip and agents per block.
template <int ROWS>
void launch_act_rows(const Batch& b, int grid, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    if (b.act_waves == 2)
        hipExtLaunchKernelGGL(b.may_stream ? k_act_gru<ROWS, 2, true> : k_act_gru<ROWS, 2, false>, dim3(grid), dim3(128),
                              0, s, t0, t1, 0, b);
    else if (b.act_waves == 8)
        hipExtLaunchKernelGGL(b.may_stream ? k_act_gru<ROWS, 8, true> : k_act_gru<ROWS, 8, false>, dim3(grid), dim3(512),
                              0, s, t0, t1, 0, b);
    else
        hipExtLaunchKernelGGL(b.may_stream ? k_act_gru<ROWS, 4, true> : k_act_gru<ROWS, 4, false>, dim3(grid), dim3(256),
                              0, s, t0, t1, 0, b);
}

void launch_act_gru(const Batch& b, int grid, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    if (b.act_rows == 8) launch_act_rows<8>(b, grid, s, t0, t1);
    else if (b.act_rows == 32) launch_act_rows<32>(b, grid, s, t0, t1);
    else launch_act_rows<16>(b, grid, s, t0, t1);
}

// `t0` / `t1` (optional): events the dispatch itself stamps when the kernel
// starts and ends (its execution time, without launch overhead).
void launch_act(const Batch& b, int grid, hipStream_t s, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr) {
    if (b.ctrl == kCtrlNet && b.dyn == kDynPaper)
        hipExtLaunchKernelGGL(b.net_wide ? k_act_net_paper_wide : k_act_net_paper, dim3(grid), dim3(kBlock), 0, s,
                              t0, t1, 0, b);
    else if (b.ctrl == kCtrlNet)
        hipExtLaunchKernelGGL(b.net_wide ? k_act_net_wide : k_act_net, dim3(grid), dim3(kBlock), 0, s, t0, t1, 0, b);
    else launch_act_gru(b, grid, s, t0, t1);
}

template <bool PAPER>
void launch_claim_t(const Batch& b, int grid, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    if (b.tile == 8) hipExtLaunchKernelGGL(PAPER ? k_claim_paper<8> : k_claim<8>, dim3(grid), dim3(64), 0, s, t0, t1, 0, b);
    else if (b.tile == 32)
        hipExtLaunchKernelGGL(PAPER ? k_claim_paper<32> : k_claim<32>, dim3(grid), dim3(64), 0, s, t0, t1, 0, b);
    else hipExtLaunchKernelGGL(PAPER ? k_claim_paper<16> : k_claim<16>, dim3(grid), dim3(64), 0, s, t0, t1, 0, b);
}

void launch_claim(const Batch& b, int grid, hipStream_t s, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr) {
    if (b.dyn == kDynPaper) launch_claim_t<true>(b, grid, s, t0, t1);
    else launch_claim_t<false>(b, grid, s, t0, t1);
}

// Enqueue one step of the per-phase kernels for a batch.
hipError_t launch_step(const Batch& b, const int* host_pre, int n, hipStream_t s) {
    const int np = n + 1;
    launch_act(b, host_pre[kPreAct * np + n], s);
    hipLaunchKernelGGL(k_move, dim3(host_pre[kPreMove * np + n]), dim3(64), 0, s, b);
    launch_claim(b, host_pre[kPreClaim * np + n], s);
    return hipGetLastError();
}

int device_cus() {
    static int cus = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (cus <= 0) cus = 1;
    });
    return cus;
}

// Whether a launch over `slots` agent slots in all uses the network act
// kernels compiled for five waves per SIMD: at four, a CU holds 16 agent waves.
int net_wide(int slots) { return slots > 16 * device_cus() ? 1 : 0; }

// Records the end of a launch of ws[0..n) (all on ws[0]'s stream, after
// the library's own capture has ended) as the last launch of each.  Launches
// that a caller records into a graph of its own (the stream is capturing)
// are the caller's to wait for: no event is recorded into its graph, and the
// worlds keep their last eager launch.
int mark_launch(world* const* ws, int n) {
    world* w0 = ws[0];
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(w0, hipStreamIsCapturing(w0->stream, &cs));
    if (cs != hipStreamCaptureStatusNone) return WORLD_OK;
    HIP_TRY(w0, hipEventRecord(w0->own->ev, w0->stream));
    for (int i = 0; i < n; ++i) ws[i]->last = w0->own;
    return WORLD_OK;
}

// Held while the library captures a graph.  HIP invalidates a capture in
// progress on a stream (and fails the call) when another thread
// synchronises with, queries or waits for an event last recorded on that
// stream, so a thread that waits for a launch polls its event under this
// lock: the library's own captures never overlap the query.
std::mutex g_capture_mu;

hipError_t wait_launch(hipEvent_t launch) {
    for (;;) {
        hipError_t q;
        {
            std::lock_guard<std::mutex> lk(g_capture_mu);
            q = hipEventQuery(launch);
        }
        if (q != hipErrorNotReady) return q;
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

// Waits on the host for the last launch that included `w`; nothing is
// pending afterwards.
int wait_world(world* w) {
    if (w->last) {
        HIP_TRY(w, wait_launch(w->last->ev));
        w->last.reset();
    }
    return WORLD_OK;
}

// A copy or fill on the world's own stream, complete when it returns.  Never
// the synchronous hipMemcpy / hipMemset: they run on the legacy default
// stream, which HIP makes depend on the other streams, and they fail (and
// invalidate the capture) while another thread captures a graph on one.
hipError_t copy_now(world* w, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
    hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, w->stream);
    return e == hipSuccess ? hipStreamSynchronize(w->stream) : e;
}

hipError_t fill_now(world* w, void* dst, int value, size_t bytes) {
    hipError_t e = hipMemsetAsync(dst, value, bytes, w->stream);
    return e == hipSuccess ? hipStreamSynchronize(w->stream) : e;
}

int check_device_error(world* w) {
    WorldScal sc;
    HIP_TRY(w, hipMemcpyAsync(&sc, w->base + w->lay.scal, sizeof(sc), hipMemcpyDeviceToHost, w->stream));
    HIP_TRY(w, hipStreamSynchronize(w->stream));
    if (sc.err != 0)
        return fail(w, WORLD_E_HIP, std::string("look-back scan") +
                                        " wait timed out on the device");
    return WORLD_OK;
}

int wall_rate_khz() {
    static int rate = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev);
        if (rate <= 0) rate = 100000;
    });
    return rate;
}

// Device table of a batch: world pointers and per-phase block prefixes.
struct TableView {
    const WorldDev* const* w;
    const int* block_pre;
    int slots = 0;        // agent slots of all worlds of the batch
    int may_stream = 0;   // some world's live genomes can exceed the last-level cache
};

// A GRU world whose genomes, with every slot live, exceed the last-level
// cache: its act phase may stream the input rows (decided on the device from
// the live count of each step), so its launches use the act kernel that holds
// the streaming copy; every other launch uses the kernel without it (smaller
// code, about 0.5% faster per step).
static int may_stream(const world* x) {
    return x->dev.ctrl == kCtrlGru && size_t(x->cfg.cap) * size_t(x->dev.Ppad) * sizeof(float) > kRowsStreamBytes;
}

size_t table_bytes(int n) { return align_up(sizeof(void*) * size_t(n), 16) + sizeof(int) * size_t(kPreKinds) * (n + 1); }

std::vector<char> build_table(const std::vector<const world*>& ws, char* dev_base, TableView* view,
                              std::vector<int>* host_block_pre, int* max_useful) {
    const int n = int(ws.size());
    const std::vector<int> bp = batch_prefix(ws, ws[0]->act_waves, ws[0]->tile);
    view->slots = 0;
    view->may_stream = 0;
    for (const world* x : ws) {
        view->slots += x->cfg.cap;
        view->may_stream |= may_stream(x);
    }
    int useful = 1;
    for (int k = 0; k < kPreKinds; ++k) useful = std::max(useful, bp[size_t(k) * (n + 1) + n]);
    const size_t ptr_bytes = align_up(sizeof(void*) * size_t(n), 16);
    std::vector<char> host(ptr_bytes + sizeof(int) * bp.size());
    for (int i = 0; i < n; ++i) {
        const WorldDev* p = ws[i]->d_dev;
        std::memcpy(host.data() + sizeof(void*) * i, &p, sizeof(p));
    }
    std::memcpy(host.data() + ptr_bytes, bp.data(), sizeof(int) * bp.size());
    view->w = reinterpret_cast<const WorldDev* const*>(dev_base);
    view->block_pre = reinterpret_cast<const int*>(dev_base + ptr_bytes);
    *host_block_pre = bp;
    *max_useful = useful;
    return host;
}

// K steps of a batch in the given mode.  `graphs` caches captured graphs.
int run_steps(world* w0, int mode, const TableView& tv, const std::vector<int>& host_bp, int n, int max_useful,
              int K, std::map<int, hipGraphExec_t>& graphs, std::map<int, hipGraph_t>& defs) {
    hipStream_t s = w0->stream;
    Batch b{tv.w, tv.block_pre, n, w0->act_rows, n == 1 ? static_cast<const WorldDev*>(w0->d_dev) : nullptr,
            w0->cfg.cap, w0->dev.ctrl, w0->dev.dyn, net_wide(tv.slots), w0->act_waves, w0->tile, tv.may_stream};
    if (mode == WORLD_MODE_KERNELS) {
        for (int k = 0; k < K; ++k) HIP_TRY(w0, launch_step(b, host_bp.data(), n, s));
        return WORLD_OK;
    }
    if (mode == WORLD_MODE_GRAPH) {
        const int gkey = ((K * 16 + w0->act_waves) * 64 + w0->tile) * 64 + w0->act_rows;
        auto it = graphs.find(gkey);
        if (it == graphs.end()) {
            hipGraph_t g = nullptr;
            hipGraphExec_t ge = nullptr;
            hipError_t le = hipSuccess, ce = hipSuccess;
            {
                std::lock_guard<std::mutex> lk(g_capture_mu);
                HIP_TRY(w0, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                for (int k = 0; k < K && le == hipSuccess; ++k) le = launch_step(b, host_bp.data(), n, s);
                ce = hipStreamEndCapture(s, &g);
            }
            if (le != hipSuccess) return fail(w0, WORLD_E_HIP, std::string("graph capture: ") + hipGetErrorString(le));
            if (ce != hipSuccess) return fail(w0, WORLD_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
            HIP_TRY(w0, hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
            defs[gkey] = g;
            it = graphs.emplace(gkey, ge).first;
        }
        HIP_TRY(w0, hipGraphLaunch(it->second, s));
        return WORLD_OK;
    }
    return fail(w0, WORLD_E_INVALID_ARG, "unknown mode");
}

}  // namespace

// Why a canonical image cannot be loaded into a world of configuration `c`
// (nullptr if it can): the full state must be present; positions inside the
// grid (one agent per cell under the benchmark rules); uids increasing and
// below next_uid; resource bytes, previous actions and ate bits in range.
static const char* image_problem(const world_config& c, const world_image* in) {
    if (in->struct_size != sizeof(world_image)) return "world_image.struct_size mismatch";
    const int n = in->n_live;
    if (n < 0 || n > c.cap) return "n_live out of range";
    if (!(in->flags & WORLD_SNAP_HIDDEN) || !(in->flags & WORLD_SNAP_THETA) || !in->R || !in->uid || !in->row ||
        !in->col || !in->energy || !in->age || !in->streak ||
        (n > 0 && (!in->h || !in->theta || !in->last_action || !in->ate)))
        return "loading needs the full state";
    if (in->step < 0) return "negative step";
    const size_t HW = size_t(c.H) * c.W;
    for (size_t i = 0; i < HW; ++i)
        if (in->R[i] > 1) return "resource bytes must be 0 or 1";
    std::vector<uint8_t> held(c.dynamics == WORLD_DYN_PAPER ? 0 : HW, 0);
    for (int i = 0; i < n; ++i) {
        if (in->row[i] < 0 || in->row[i] >= c.H || in->col[i] < 0 || in->col[i] >= c.W) return "agent outside the grid";
        if (i > 0 && in->uid[i] <= in->uid[i - 1]) return "uids must increase";
        if (in->uid[i] >= in->next_uid) return "uid >= next_uid";
        if (in->age[i] < 0) return "negative age";
        if (in->last_action[i] > kNoAction || in->ate[i] > 1) return "last_action must be 0..5 and ate 0 or 1";
        if (c.dynamics != WORLD_DYN_PAPER) {
            const size_t cell = size_t(in->row[i]) * c.W + in->col[i];
            if (held[cell]) return "two agents in one cell";
            held[cell] = 1;
        }
    }
    return nullptr;
}

// =========================================================================
// C-ABI
// =========================================================================

extern "C" {

int world_required_bytes(const world_config* cfg, size_t* device_bytes, size_t* snapshot_bytes) {
    if (!device_bytes && !snapshot_bytes)
        return fail(nullptr, WORLD_E_INVALID_ARG, "device_bytes and snapshot_bytes are both NULL");
    if (const char* m = check_config(cfg)) return fail(nullptr, WORLD_E_INVALID_CONFIG, m);
    if (device_bytes) *device_bytes = layout_of(*cfg).total;
    if (snapshot_bytes) *snapshot_bytes = snapshot_bytes_of(*cfg, dims_of(*cfg));
    return WORLD_OK;
}

int world_dims(const world_config* cfg, int32_t* n_in, int32_t* n_params) {
    if (const char* m = check_config(cfg)) return fail(nullptr, WORLD_E_INVALID_CONFIG, m);
    const Dims d = dims_of(*cfg);
    if (n_in) *n_in = d.n_in;
    if (n_params) *n_params = d.P;
    return WORLD_OK;
}

int world_threshold_table(const world_config* cfg, uint64_t* out) {
    if (!out) return fail(nullptr, WORLD_E_INVALID_ARG, "out is NULL");
    if (const char* m = check_config(cfg)) return fail(nullptr, WORLD_E_INVALID_CONFIG, m);
    build_thresholds(*cfg, out);
    return WORLD_OK;
}

int world_create(const world_config* cfg, uint64_t seed, void* arena, size_t arena_bytes, void* hip_stream,
                 world_t** out) {
    TraceRange trace("world_create");
    if (!out || !arena) return fail(nullptr, WORLD_E_INVALID_ARG, "arena and out must be non-NULL");
    *out = nullptr;
    if (const char* m = check_config(cfg)) return fail(nullptr, WORLD_E_INVALID_CONFIG, m);
    if (reinterpret_cast<uintptr_t>(arena) % kAlign != 0)
        return fail(nullptr, WORLD_E_INVALID_ARG, "arena must be 256-byte aligned");
    const Layout lay = layout_of(*cfg);
    if (arena_bytes < lay.total) return fail(nullptr, WORLD_E_BUFFER_TOO_SMALL, "arena smaller than world_required_bytes");

    world* w = new world();
    w->own = std::make_shared<WorkEvent>();
    {
        const hipError_t e = hipEventCreateWithFlags(&w->own->ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            delete w;
            return fail(nullptr, WORLD_E_HIP, std::string("world_create: ") + hipGetErrorString(e));
        }
    }
    w->cfg = *cfg;
    w->dm = dims_of(*cfg);
    w->lay = lay;
    w->seed = seed;
    w->base = static_cast<char*>(arena);
    w->stream = static_cast<hipStream_t>(hip_stream);
    const world_config& c = *cfg;
    const Dims& dm = w->dm;
    char* b = w->base;

    WorldDev& d = w->dev;
    std::memset(&d, 0, sizeof(d));
    d.H = c.H; d.W = c.W; d.cap = c.cap; d.rho = c.obs_radius; d.hd = c.hidden;
    d.n_in = dm.n_in; d.P = dm.P; d.Ppad = dm.Ppad;
    d.E0 = c.E0; d.decay = c.decay; d.gain = c.gain; d.E_repr = c.E_repr; d.T_repr = c.T_repr; d.L_max = c.L_max;
    d.sigma = float(c.sigma_mut);
    d.seed_lo = uint32_t(seed); d.seed_hi = uint32_t(seed >> 32);
    d.forced = -1;
    d.stall_tile = -1;
    d.spin_ticks = kSpinTicks;
    d.log_steps = c.log_steps;
    d.off_hh = dm.off_hh; d.off_bih = dm.off_bih; d.off_bhh = dm.off_bhh; d.off_wo = dm.off_wo; d.off_bo = dm.off_bo;
    d.tot_row = dm.tot_row;
    d.nblk = dm.nblk;
    d.ctrl = is_net(c) ? kCtrlNet : kCtrlGru;
    d.ss = state_of(c);
    d.dyn = c.dynamics == WORLD_DYN_PAPER ? kDynPaper : kDynBench;
    d.E_max = c.E_max;
    d.T_death = c.T_death;
    d.R[0] = reinterpret_cast<uint8_t*>(b + lay.R0);
    d.R[1] = reinterpret_cast<uint8_t*>(b + lay.R1);
    d.occA = reinterpret_cast<int32_t*>(b + lay.occA);
    d.occB = reinterpret_cast<int32_t*>(b + lay.occB);
    d.thr = reinterpret_cast<const uint64_t*>(b + lay.thr);
    d.mclaim = reinterpret_cast<uint64_t*>(b + lay.mclaim);
    d.uid = reinterpret_cast<uint32_t*>(b + lay.uid);
    d.cell = reinterpret_cast<int32_t*>(b + lay.cell);
    d.prev_cell = reinterpret_cast<int32_t*>(b + lay.prev_cell);
    d.energy = reinterpret_cast<int32_t*>(b + lay.energy);
    d.age = reinterpret_cast<int32_t*>(b + lay.age);
    d.streak = reinterpret_cast<int32_t*>(b + lay.streak);
    d.action = reinterpret_cast<uint8_t*>(b + lay.action);
    d.alive = reinterpret_cast<uint8_t*>(b + lay.alive);
    d.ate = reinterpret_cast<uint8_t*>(b + lay.ate);
    d.claim = reinterpret_cast<int32_t*>(b + lay.claim);
    d.bkey = reinterpret_cast<uint64_t*>(b + lay.bkey);
    d.h = reinterpret_cast<float*>(b + lay.h);
    d.gh = reinterpret_cast<float*>(b + lay.gh);
    d.theta = reinterpret_cast<float*>(b + lay.theta);
    d.live[0] = reinterpret_cast<int32_t*>(b + lay.live0);
    d.live[1] = reinterpret_cast<int32_t*>(b + lay.live1);
    d.pos = reinterpret_cast<PosRec*>(b + lay.pos);
    d.freeq = reinterpret_cast<int32_t*>(b + lay.freeq);
    d.child = reinterpret_cast<int4*>(b + lay.child);
    d.scal = reinterpret_cast<WorldScal*>(b + lay.scal);
    d.ring = reinterpret_cast<int32_t*>(b + lay.ring);
    d.log_uid = reinterpret_cast<uint32_t*>(b + lay.log_uid);
    d.log_act = reinterpret_cast<uint8_t*>(b + lay.log_act);
    d.log_logits = reinterpret_cast<float*>(b + lay.log_logits);
    d.log_n = reinterpret_cast<int32_t*>(b + lay.log_n);
    d.eat_part = reinterpret_cast<int32_t*>(b + lay.eat_part);
    d.dage_part = reinterpret_cast<int32_t*>(b + lay.dage_part);
    d.wcell = reinterpret_cast<int32_t*>(b + lay.wcell);
    d.wuid = reinterpret_cast<uint32_t*>(b + lay.wuid);
    d.mhist = reinterpret_cast<int32_t*>(b + lay.mhist);
    d.deadlist = reinterpret_cast<int32_t*>(b + lay.deadlist);
    d.lb_move = reinterpret_cast<uint64_t*>(b + lay.lb_move);
    d.lb_claim = reinterpret_cast<uint64_t*>(b + lay.lb_claim);
    d.res_part = reinterpret_cast<int32_t*>(b + lay.res_part);
    d.rows_part = reinterpret_cast<int32_t*>(b + lay.rows_part);
    d.forced_tab = reinterpret_cast<const int8_t*>(b + lay.forced);
    d.n_forced = 0;
    d.forced_on = 0;
    d.res_ntiles = reinterpret_cast<int32_t*>(b + lay.res_ntiles);
    w->d_dev = reinterpret_cast<WorldDev*>(b + lay.desc);

    // Host initialisation (not timed): resources, placement, lists.
    const size_t HW = size_t(c.H) * c.W;
    std::vector<uint8_t> R(HW);
    const uint64_t res_thr = threshold_of(c.res_init_p);
    std::vector<uint64_t> keys(HW);
    for (size_t i = 0; i < HW; ++i) {
        R[i] = uint64_t(philox(uint32_t(i), 0, kInitRes, 0, d.seed_lo, d.seed_hi).x) < res_thr ? 1 : 0;
        keys[i] = (uint64_t(philox(uint32_t(i), 0, kInitPlace, 0, d.seed_lo, d.seed_hi).x) << 32) | i;
    }
    const size_t n0 = size_t(c.n_init);
    std::partial_sort(keys.begin(), keys.begin() + n0, keys.end());
    std::vector<int32_t> occ(HW, -1);
    std::vector<int32_t> cells(c.cap, 0), energy(c.cap, 0), zeros(c.cap, 0), live(c.cap, 0), freeq(c.cap, 0);
    std::vector<uint32_t> uid(c.cap, 0);
    std::vector<uint8_t> alive(c.cap, 0);
    const bool paper = c.dynamics == WORLD_DYN_PAPER;
    for (size_t a = 0; a < n0; ++a) {
        const int32_t cell = int32_t(keys[a] & 0xFFFFFFFFu);
        occ[cell] = paper ? 0 : int32_t(a);   // paper dynamics: agents on the cell minus one
        cells[a] = cell;
        energy[a] = c.E0;
        uid[a] = uint32_t(a);
        alive[a] = 1;
        live[a] = int32_t(a);
    }
    for (int s = int(n0); s < c.cap; ++s) freeq[s - int(n0)] = s;
    std::vector<PosRec> recs(c.cap);
    std::memset(recs.data(), 0, sizeof(PosRec) * recs.size());
    for (size_t a = 0; a < n0; ++a)
        recs[a].r[0] = AgentRec{int32_t(a), cells[a], c.E0, uint32_t(a), 0, 0, kNoAction, 0};
    std::vector<uint64_t> thr(size_t(c.H) * 25);
    build_thresholds(c, thr.data());
    WorldScal sc;
    std::memset(&sc, 0, sizeof(sc));
    sc.n_live = int32_t(n0);
    sc.next_uid = uint32_t(n0);
    sc.free_head = 0;
    sc.free_tail = (c.cap - int(n0)) % c.cap;
    // Single-world launch table.
    TableView tv;
    std::vector<const world*> one{w};
    const std::vector<char> table = build_table(one, b + lay.batch, &tv, &w->host_bp, &w->max_useful);
    w->tv.w = tv.w;
    w->tv.block_pre = tv.block_pre;
    w->tv.slots = tv.slots;
    w->tv.may_stream = tv.may_stream;

    hipStream_t s = w->stream;
    auto up = [&](size_t off, const void* src, size_t bytes) {
        return hipMemcpyAsync(b + off, src, bytes, hipMemcpyHostToDevice, s);
    };
    hipError_t e = hipSuccess;
#define UP(off, src, bytes) \
    if (e == hipSuccess) e = up(off, src, bytes)
    UP(lay.desc, &d, sizeof(d));
    UP(lay.scal, &sc, sizeof(sc));
    UP(lay.batch, table.data(), table.size());
    UP(lay.thr, thr.data(), thr.size() * sizeof(uint64_t));
    UP(lay.R0, R.data(), HW);
    UP(lay.R1, R.data(), HW);
    UP(lay.occA, occ.data(), HW * 4);
    UP(lay.occB, occ.data(), HW * 4);
    UP(lay.uid, uid.data(), size_t(c.cap) * 4);
    UP(lay.cell, cells.data(), size_t(c.cap) * 4);
    UP(lay.prev_cell, cells.data(), size_t(c.cap) * 4);
    UP(lay.energy, energy.data(), size_t(c.cap) * 4);
    UP(lay.age, zeros.data(), size_t(c.cap) * 4);
    UP(lay.streak, zeros.data(), size_t(c.cap) * 4);
    UP(lay.claim, zeros.data(), size_t(c.cap) * 4);
    UP(lay.alive, alive.data(), size_t(c.cap));
    UP(lay.live0, live.data(), size_t(c.cap) * 4);
    UP(lay.live1, live.data(), size_t(c.cap) * 4);
    UP(lay.pos, recs.data(), sizeof(PosRec) * size_t(c.cap));
    UP(lay.freeq, freeq.data(), size_t(c.cap) * 4);
#undef UP
    if (e == hipSuccess) e = hipMemsetAsync(b + lay.ring, 0, sizeof(int32_t) * kRing * kCtrWords, s);
    if (e == hipSuccess) e = hipMemsetAsync(b + lay.mclaim, 0xFF, 8 * HW, s);
    if (e == hipSuccess) e = hipMemsetAsync(b + lay.wuid, 0xFF, 4 * size_t(c.cap), s);
    // tables a step fills before reading: zeroed so that no entry ever holds
    // a slot index out of range
    if (e == hipSuccess) e = hipMemsetAsync(b + lay.child, 0, 16 * size_t(c.cap), s);
    if (e == hipSuccess) e = hipMemsetAsync(b + lay.deadlist, 0, 4 * size_t(c.cap), s);
    if (e == hipSuccess) e = hipMemsetAsync(b + lay.mhist, 0, 4 * size_t(kMoveRing) * (kMoveBins + 1), s);
    if (e == hipSuccess) e = hipMemsetAsync(b + lay.res_ntiles, 0, 4, s);
    if (e == hipSuccess) e = hipMemsetAsync(b + lay.lb_move, 0, 8 * size_t(tiles_agent(c)), s);
    if (e == hipSuccess) e = hipMemsetAsync(b + lay.lb_claim, 0, 8 * size_t(tiles_agent(c)), s);
    if (e == hipSuccess) e = hipMemsetAsync(b + lay.h, 0, 4 * size_t(c.cap) * state_of(c), s);
    if (e == hipSuccess) e = hipMemsetAsync(b + lay.action, kNoAction, size_t(c.cap), s);
    if (e == hipSuccess) e = hipMemsetAsync(b + lay.ate, 0, size_t(c.cap), s);
    if (e == hipSuccess) e = hipMemsetAsync(b + lay.theta, 0, 4 * size_t(c.cap) * dm.Ppad, s);
    if (e == hipSuccess && c.log_steps > 0) e = hipMemsetAsync(b + lay.log_n, 0, 4 * size_t(c.log_steps), s);
    if (e == hipSuccess && n0 > 0) {
        const InitSegs segs = init_segments(c, dm);
        const int64_t items = int64_t(n0) * dm.nblk;
        const int grid = int(std::min<int64_t>((items + kBlock - 1) / kBlock, 65536));
        hipLaunchKernelGGL(k_init_theta, dim3(grid), dim3(kBlock), 0, s, w->d_dev, int(n0), segs);
        e = hipGetLastError();
    }
    if (e == hipSuccess && n0 > 0 && !is_net(c)) {
        hipLaunchKernelGGL(k_proj_all, dim3(blocks_of_agents(c)), dim3(kBlock), 0, s, static_cast<const WorldDev*>(w->d_dev));
        hipLaunchKernelGGL(k_rsum_all, dim3(c.cap), dim3(kBlock), 0, s, static_cast<const WorldDev*>(w->d_dev));
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        fail(nullptr, WORLD_E_HIP, std::string("world_create: ") + hipGetErrorString(e));
        delete w;
        return WORLD_E_HIP;
    }
    *out = w;
    return WORLD_OK;
}

int world_set_stream(world_t* w, void* hip_stream) {
    if (!w) return fail(nullptr, WORLD_E_INVALID_ARG, "world is NULL");
    if (w->poisoned) return WORLD_E_POISONED;
    if (int rc = wait_world(w)) return rc;
    w->stream = static_cast<hipStream_t>(hip_stream);
    return WORLD_OK;
}

int world_set_tuning(world_t* w, int32_t act_rows, int32_t act_waves, int32_t regrow_tile) {
    if (!w) return fail(nullptr, WORLD_E_INVALID_ARG, "world is NULL");
    if (w->poisoned) return WORLD_E_POISONED;
    if (act_rows != 8 && act_rows != 16 && act_rows != 32) return fail(w, WORLD_E_INVALID_ARG, "act_rows must be 8, 16 or 32");
    if (act_waves != 2 && act_waves != 4 && act_waves != 8)
        return fail(w, WORLD_E_INVALID_ARG, "act_waves must be 2, 4 or 8");
    if (regrow_tile != 8 && regrow_tile != 16 && regrow_tile != 32)
        return fail(w, WORLD_E_INVALID_ARG, "regrow_tile must be 8, 16 or 32");
    w->act_rows = act_rows;
    if (act_waves == w->act_waves && regrow_tile == w->tile) return WORLD_OK;
    // the single-world launch table (block prefixes) depends on the shape
    HIP_TRY(w, hipStreamSynchronize(w->stream));
    w->act_waves = act_waves;
    w->tile = regrow_tile;
    TableView tv;
    std::vector<const world*> one{w};
    const std::vector<char> table = build_table(one, w->base + w->lay.batch, &tv, &w->host_bp, &w->max_useful);
    HIP_TRY(w, copy_now(w, w->base + w->lay.batch, table.data(), table.size(), hipMemcpyHostToDevice));
    return WORLD_OK;
}

int world_set_mode(world_t* w, int32_t mode) {
    if (!w) return fail(nullptr, WORLD_E_INVALID_ARG, "world is NULL");
    if (mode != WORLD_MODE_KERNELS && mode != WORLD_MODE_GRAPH)
        return fail(w, WORLD_E_INVALID_ARG, "unknown mode");
    w->mode = mode;
    return WORLD_OK;
}

static int step_single(world* w, int K) {
    TableView tv;
    tv.w = w->tv.w;
    tv.block_pre = w->tv.block_pre;
    tv.slots = w->tv.slots;
    tv.may_stream = w->tv.may_stream;
    if (int rc = run_steps(w, w->mode, tv, w->host_bp, 1, w->max_useful, K, w->graphs, w->graph_defs)) return rc;
    return mark_launch(&w, 1);
}

// Launch tables of batches (device memory owned by the library, one per
// distinct list of worlds), with their captured graphs.  At most kBatchCache
// tables are kept (more only while every one is being launched from); the
// least recently used idle one is released (after its last launch) when a new
// list needs a table.
struct BatchEntry {
    void* dev = nullptr;
    TableView tv;
    std::vector<int> host_bp;
    int max_useful = 1;
    uint64_t last_use = 0;
    std::shared_ptr<WorkEvent> done;   // recorded after the entry's last launch
    std::vector<char> host_table;      // source of the table's upload
    int busy = 0;                      // calls launching from the entry (guarded by g_batch_mu)
    std::map<int, hipGraphExec_t> graphs;
    std::map<int, hipGraph_t> defs;
};

constexpr size_t kBatchCache = 64;
static std::mutex g_batch_mu;
static std::map<std::vector<uintptr_t>, BatchEntry*> g_batches;
static uint64_t g_batch_clock = 0;

constexpr size_t kBatchKeyWords = 8;   // key words per world (the handle first)

static std::vector<uintptr_t> batch_key(world_t* const* ws, int n) {
    std::vector<uintptr_t> key;
    for (int i = 0; i < n; ++i) {
        key.push_back(reinterpret_cast<uintptr_t>(ws[i]));
        key.push_back(reinterpret_cast<uintptr_t>(ws[i]->d_dev));
        key.push_back(uintptr_t(ws[i]->cfg.cap));
        key.push_back(uintptr_t(ws[i]->cfg.H) << 32 | uintptr_t(ws[i]->cfg.W));
        key.push_back(uintptr_t(ws[i]->cfg.hidden));
        key.push_back(uintptr_t(ws[i]->cfg.controller));
        key.push_back(uintptr_t(ws[i]->cfg.dynamics));
        key.push_back(uintptr_t(ws[0]->act_waves) << 8 | uintptr_t(ws[0]->tile));   // the launch shape
    }
    return key;
}

static void release_entry(BatchEntry* be) {
    if (be->done) (void)wait_launch(be->done->ev);
    for (auto& kv : be->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto& kv : be->defs) (void)hipGraphDestroy(kv.second);
    if (be->dev) (void)hipFree(be->dev);
    delete be;
}

static int batch_step(world_t* const* ws, int n, int K) {
    world* w0 = ws[0];
    BatchEntry* be = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_batch_mu);
        auto key = batch_key(ws, n);
        auto it = g_batches.find(key);
        if (it == g_batches.end()) {
            if (g_batches.size() >= kBatchCache) {
                // the least recently used entry that no other thread is
                // launching from (the cache overflows while all are busy)
                auto lru = g_batches.end();
                for (auto jt = g_batches.begin(); jt != g_batches.end(); ++jt)
                    if (jt->second->busy == 0 && (lru == g_batches.end() || jt->second->last_use < lru->second->last_use))
                        lru = jt;
                if (lru != g_batches.end()) {
                    release_entry(lru->second);
                    g_batches.erase(lru);
                }
            }
            be = new BatchEntry();
            hipError_t e = hipMalloc(&be->dev, table_bytes(n));
            if (e != hipSuccess) {
                delete be;
                return fail(w0, WORLD_E_HIP, std::string("hipMalloc(batch table): ") + hipGetErrorString(e));
            }
            std::vector<const world*> list(ws, ws + n);
            const std::vector<char> host = build_table(list, static_cast<char*>(be->dev), &be->tv, &be->host_bp,
                                                       &be->max_useful);
            // on the launch stream, ahead of the launches that read it; the
            // host copy lives with the entry, so nothing waits for the copy
            be->host_table = host;
            e = hipMemcpyAsync(be->dev, be->host_table.data(), be->host_table.size(), hipMemcpyHostToDevice, w0->stream);
            if (e != hipSuccess) {
                (void)hipFree(be->dev);
                delete be;
                return fail(w0, WORLD_E_HIP, std::string("batch table upload: ") + hipGetErrorString(e));
            }
            it = g_batches.emplace(std::move(key), be).first;
        }
        be = it->second;
        be->last_use = ++g_batch_clock;
        be->busy += 1;   // not evicted while this call launches from it
    }
    int rc = run_steps(w0, w0->mode, be->tv, be->host_bp, n, be->max_useful, K, be->graphs, be->defs);
    if (rc == WORLD_OK) rc = mark_launch(ws, n);
    std::lock_guard<std::mutex> lk(g_batch_mu);
    if (rc == WORLD_OK) be->done = w0->own;
    be->busy -= 1;
    return rc;
}

int world_step(world_t* w, int32_t K) {
    TraceRange trace("world_step K=%d", K);
    if (!w) return fail(nullptr, WORLD_E_INVALID_ARG, "world is NULL");
    if (w->poisoned) return WORLD_E_POISONED;
    if (K < 1) return fail(w, WORLD_E_INVALID_ARG, "K must be >= 1");
    return step_single(w, K);
}

int world_sync(world_t* w) {
    if (!w) return fail(nullptr, WORLD_E_INVALID_ARG, "world is NULL");
    if (w->poisoned) return WORLD_E_POISONED;
    HIP_TRY(w, hipStreamSynchronize(w->stream));
    return check_device_error(w);
}

int world_snapshot(world_t* w, world_image* out) {
    TraceRange trace("world_snapshot");
    if (!w || !out) return fail(w, WORLD_E_INVALID_ARG, "NULL argument");
    if (w->poisoned) return WORLD_E_POISONED;
    if (out->struct_size != sizeof(world_image)) return fail(w, WORLD_E_INVALID_ARG, "world_image.struct_size mismatch");
    if (int rc = world_sync(w)) return rc;
    const world_config& c = w->cfg;
    const Layout& l = w->lay;
    WorldScal sc;
    HIP_TRY(w, copy_now(w, &sc, w->base + l.scal, sizeof(sc), hipMemcpyDeviceToHost));
    if (sc.n_child > 0) {
        // children of the last step are created at the start of the next
        // one; create them now so that the image is complete
        const WorldDev* dp = w->d_dev;
        hipLaunchKernelGGL(k_materialize, dim3(std::min(sc.n_child, 1024)), dim3(kBlock), 0, w->stream, dp);
        hipLaunchKernelGGL(k_clear_pending, dim3(1), dim3(64), 0, w->stream, dp);
        HIP_TRY(w, hipGetLastError());
        HIP_TRY(w, hipStreamSynchronize(w->stream));
        HIP_TRY(w, copy_now(w, &sc, w->base + l.scal, sizeof(sc), hipMemcpyDeviceToHost));
    }
    out->step = sc.t;
    out->n_live = sc.n_live;
    out->next_uid = sc.next_uid;
    if (out->agent_capacity < sc.n_live) return fail(w, WORLD_E_BUFFER_TOO_SMALL, "agent_capacity < n_live");
    const size_t HW = size_t(c.H) * c.W;
    if (out->R) HIP_TRY(w, copy_now(w, out->R, w->base + (sc.t & 1 ? l.R1 : l.R0), HW, hipMemcpyDeviceToHost));
    const int n = sc.n_live;
    std::vector<int32_t> live(std::max(n, 1));
    HIP_TRY(w, copy_now(w, live.data(), w->base + (sc.live_sel ? l.live1 : l.live0), 4 * size_t(n), hipMemcpyDeviceToHost));
    auto gather_i32 = [&](size_t off, int32_t* dst) -> int {
        if (!dst) return WORLD_OK;
        std::vector<int32_t> all(c.cap);
        HIP_TRY(w, copy_now(w, all.data(), w->base + off, 4 * size_t(c.cap), hipMemcpyDeviceToHost));
        for (int i = 0; i < n; ++i) dst[i] = all[live[i]];
        return WORLD_OK;
    };
    if (int rc = gather_i32(l.uid, reinterpret_cast<int32_t*>(out->uid))) return rc;
    if (out->row || out->col) {
        std::vector<int32_t> cells(std::max(n, 1));
        if (int rc = gather_i32(l.cell, cells.data())) return rc;
        for (int i = 0; i < n; ++i) {
            if (out->row) out->row[i] = cells[i] / c.W;
            if (out->col) out->col[i] = cells[i] % c.W;
        }
    }
    if (int rc = gather_i32(l.energy, out->energy)) return rc;
    if (int rc = gather_i32(l.age, out->age)) return rc;
    if (int rc = gather_i32(l.streak, out->streak)) return rc;
    const size_t ss = size_t(state_of(c));
    if ((out->flags & WORLD_SNAP_HIDDEN) && out->h) {
        std::vector<float> hs(size_t(c.cap) * ss);
        HIP_TRY(w, copy_now(w, hs.data(), w->base + l.h, 4 * hs.size(), hipMemcpyDeviceToHost));
        for (int i = 0; i < n; ++i) std::memcpy(out->h + size_t(i) * ss, hs.data() + size_t(live[i]) * ss, 4 * ss);
    }
    auto gather_u8 = [&](size_t off, uint8_t* dst) -> int {
        if (!dst) return WORLD_OK;
        std::vector<uint8_t> all(c.cap);
        HIP_TRY(w, copy_now(w, all.data(), w->base + off, size_t(c.cap), hipMemcpyDeviceToHost));
        for (int i = 0; i < n; ++i) dst[i] = all[live[i]];
        return WORLD_OK;
    };
    if (out->flags & WORLD_SNAP_HIDDEN) {
        if (int rc = gather_u8(l.action, out->last_action)) return rc;
        if (int rc = gather_u8(l.ate, out->ate)) return rc;
    }
    if ((out->flags & WORLD_SNAP_THETA) && out->theta) {
        // whole slot ranges of at most 64 MB, one copy each, then the rows of
        // the live agents in them (in uid order in the image)
        const size_t P = size_t(w->dm.P), Pp = size_t(w->dm.Ppad);
        std::vector<int> by_slot(static_cast<size_t>(n));
        for (int i = 0; i < n; ++i) by_slot[size_t(i)] = i;
        std::sort(by_slot.begin(), by_slot.end(), [&](int a, int b) { return live[a] < live[b]; });
        const size_t chunk = std::max<size_t>(1, (size_t(64) << 20) / (4 * Pp));
        std::vector<float> buf(std::min(chunk, size_t(c.cap)) * Pp);
        size_t k = 0;
        for (size_t s0 = 0; s0 < size_t(c.cap) && k < by_slot.size(); s0 += chunk) {
            const size_t s1 = std::min(size_t(c.cap), s0 + chunk);
            if (size_t(live[by_slot[k]]) >= s1) continue;   // no live agent in these slots
            HIP_TRY(w, copy_now(w, buf.data(), w->base + l.theta + 4 * Pp * s0, 4 * Pp * (s1 - s0),
                                 hipMemcpyDeviceToHost));
            for (; k < by_slot.size() && size_t(live[by_slot[k]]) < s1; ++k)
                std::memcpy(out->theta + size_t(by_slot[k]) * P, buf.data() + (size_t(live[by_slot[k]]) - s0) * Pp,
                            4 * P);
        }
    }
    return WORLD_OK;
}

int world_load(world_t* w, const world_image* in) {
    TraceRange trace("world_load");
    if (!w || !in) return fail(w, WORLD_E_INVALID_ARG, "NULL argument");
    if (w->poisoned) return WORLD_E_POISONED;
    const world_config& c = w->cfg;
    if (const char* m = image_problem(c, in)) return fail(w, WORLD_E_INVALID_ARG, m);
    const int n = in->n_live;
    const size_t HW = size_t(c.H) * c.W;
    std::vector<int32_t> occ(HW, -1), cells(c.cap, 0), live(c.cap, 0), freeq(c.cap, 0);
    for (int i = 0; i < n; ++i) {
        const int cell = in->row[i] * c.W + in->col[i];
        if (c.dynamics == WORLD_DYN_PAPER) occ[cell] += 1;   // agents on the cell minus one (-1 = empty)
        else occ[cell] = i;
        cells[i] = cell;
        live[i] = i;
    }
    for (int s = n; s < c.cap; ++s) freeq[s - n] = s;
    std::vector<uint8_t> alive(c.cap, 0);
    for (int i = 0; i < n; ++i) alive[i] = 1;
    WorldScal sc;
    std::memset(&sc, 0, sizeof(sc));
    sc.t = in->step;
    sc.n_live = n;
    sc.next_uid = in->next_uid;
    sc.free_tail = (c.cap - n) % c.cap;
    const Layout& l = w->lay;
    char* b = w->base;
    const size_t P = size_t(w->dm.P), Pp = size_t(w->dm.Ppad);
    std::vector<float> th(size_t(std::max(n, 1)) * Pp, 0.f);
    for (int i = 0; i < n; ++i) std::memcpy(th.data() + size_t(i) * Pp, in->theta + size_t(i) * P, 4 * P);
    std::vector<int32_t> ages(c.cap, 0), streaks(c.cap, 0), energies(c.cap, 0);
    std::vector<uint32_t> uids(c.cap, 0);
    std::vector<uint8_t> acts(c.cap, uint8_t(kNoAction)), ates(c.cap, 0);
    for (int i = 0; i < n; ++i) {
        ages[i] = in->age[i];
        streaks[i] = in->streak[i];
        energies[i] = in->energy[i];
        uids[i] = in->uid[i];
        acts[i] = in->last_action[i];
        ates[i] = in->ate[i];
    }
    HIP_TRY(w, hipStreamSynchronize(w->stream));
    HIP_TRY(w, copy_now(w, b + l.scal, &sc, sizeof(sc), hipMemcpyHostToDevice));
    HIP_TRY(w, copy_now(w, b + (in->step & 1 ? l.R1 : l.R0), in->R, HW, hipMemcpyHostToDevice));
    HIP_TRY(w, copy_now(w, b + l.occA, occ.data(), 4 * HW, hipMemcpyHostToDevice));
    HIP_TRY(w, copy_now(w, b + l.occB, occ.data(), 4 * HW, hipMemcpyHostToDevice));
    HIP_TRY(w, copy_now(w, b + l.uid, uids.data(), 4 * size_t(c.cap), hipMemcpyHostToDevice));
    HIP_TRY(w, copy_now(w, b + l.cell, cells.data(), 4 * size_t(c.cap), hipMemcpyHostToDevice));
    HIP_TRY(w, copy_now(w, b + l.prev_cell, cells.data(), 4 * size_t(c.cap), hipMemcpyHostToDevice));
    HIP_TRY(w, copy_now(w, b + l.energy, energies.data(), 4 * size_t(c.cap), hipMemcpyHostToDevice));
    HIP_TRY(w, copy_now(w, b + l.age, ages.data(), 4 * size_t(c.cap), hipMemcpyHostToDevice));
    HIP_TRY(w, copy_now(w, b + l.streak, streaks.data(), 4 * size_t(c.cap), hipMemcpyHostToDevice));
    HIP_TRY(w, copy_now(w, b + l.alive, alive.data(), size_t(c.cap), hipMemcpyHostToDevice));
    HIP_TRY(w, copy_now(w, b + l.action, acts.data(), size_t(c.cap), hipMemcpyHostToDevice));
    HIP_TRY(w, copy_now(w, b + l.ate, ates.data(), size_t(c.cap), hipMemcpyHostToDevice));
    HIP_TRY(w, copy_now(w, b + l.live0, live.data(), 4 * size_t(c.cap), hipMemcpyHostToDevice));
    {
        std::vector<PosRec> recs(c.cap);
        std::memset(recs.data(), 0, sizeof(PosRec) * recs.size());
        for (int i = 0; i < n; ++i)
            recs[i].r[0] = AgentRec{i, cells[i], energies[i], uids[i], ages[i], streaks[i], int32_t(acts[i]),
                                    int32_t(ates[i])};
        HIP_TRY(w, copy_now(w, b + l.pos, recs.data(), sizeof(PosRec) * size_t(c.cap), hipMemcpyHostToDevice));
    }
    HIP_TRY(w, copy_now(w, b + l.freeq, freeq.data(), 4 * size_t(c.cap), hipMemcpyHostToDevice));
    HIP_TRY(w, fill_now(w, b + l.lb_move, 0, 8 * size_t(tiles_agent(c))));
    HIP_TRY(w, fill_now(w, b + l.lb_claim, 0, 8 * size_t(tiles_agent(c))));
    HIP_TRY(w, fill_now(w, b + l.mclaim, 0xFF, 8 * HW));
    HIP_TRY(w, fill_now(w, b + l.wuid, 0xFF, 4 * size_t(c.cap)));   // no agent counts in the window in progress
    HIP_TRY(w, fill_now(w, b + l.mhist, 0, 4 * size_t(kMoveRing) * (kMoveBins + 1)));
    if (n > 0) {
        const size_t ss = size_t(state_of(c));
        std::vector<float> hs(size_t(c.cap) * ss, 0.f);
        std::memcpy(hs.data(), in->h, 4 * size_t(n) * ss);
        HIP_TRY(w, copy_now(w, b + l.h, hs.data(), 4 * hs.size(), hipMemcpyHostToDevice));
        HIP_TRY(w, copy_now(w, b + l.theta, th.data(), 4 * size_t(n) * Pp, hipMemcpyHostToDevice));
    }
    if (n > 0 && !is_net(c)) {
        hipLaunchKernelGGL(k_proj_all, dim3(blocks_of_agents(c)), dim3(kBlock), 0, w->stream,
                           static_cast<const WorldDev*>(w->d_dev));
        hipLaunchKernelGGL(k_rsum_all, dim3(c.cap), dim3(kBlock), 0, w->stream,
                           static_cast<const WorldDev*>(w->d_dev));
        HIP_TRY(w, hipGetLastError());
        HIP_TRY(w, hipStreamSynchronize(w->stream));
    }
    return WORLD_OK;
}

int world_validate_image(const world_config* cfg, const world_image* in) {
    if (!in) return fail(nullptr, WORLD_E_INVALID_ARG, "image is NULL");
    if (const char* m = check_config(cfg)) return fail(nullptr, WORLD_E_INVALID_CONFIG, m);
    if (const char* m = image_problem(*cfg, in)) return fail(nullptr, WORLD_E_INVALID_ARG, m);
    return WORLD_OK;
}

int world_counters_get(world_t* w, int64_t first, int32_t n, world_counters* out) {
    if (!w || (!out && n > 0)) return fail(w, WORLD_E_INVALID_ARG, "NULL argument");
    if (w->poisoned) return WORLD_E_POISONED;
    // the eaten / resource totals of the last step are summed at the start of
    // the next step; sum them now if that has not happened yet
    hipLaunchKernelGGL(k_close_counters, dim3(1), dim3(kBlock), 0, w->stream, static_cast<const WorldDev*>(w->d_dev));
    HIP_TRY(w, hipGetLastError());
    if (int rc = world_sync(w)) return rc;
    WorldScal sc;
    HIP_TRY(w, copy_now(w, &sc, w->base + w->lay.scal, sizeof(sc), hipMemcpyDeviceToHost));
    if (n < 0 || first < 0 || first + n > sc.t || first < sc.t - kRing)
        return fail(w, WORLD_E_STATE, "requested steps are not held in the counter ring");
    std::vector<int32_t> ring(size_t(kRing) * kCtrWords);
    HIP_TRY(w, copy_now(w, ring.data(), w->base + w->lay.ring, 4 * ring.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i) {
        const int32_t* r = ring.data() + ((first + i) % kRing) * kCtrWords;
        out[i].n_live = r[kCtrLive];
        out[i].births = r[kCtrBirths];
        out[i].deaths = r[kCtrDeaths];
        out[i].eaten = r[kCtrEaten];
        out[i].resources = r[kCtrRes];
        out[i].claim_wins = r[kCtrWins];
        out[i].dead_age_sum = int64_t((uint64_t(uint32_t(r[kCtrDeadAgeHi])) << 32) | uint32_t(r[kCtrDeadAgeLo]));
        out[i].seen_resource = r[kCtrSeen];
        out[i].rows_read = r[kCtrRows];
    }
    return WORLD_OK;
}

int world_move_hist(world_t* w, int64_t first, int32_t n, int32_t* out) {
    if (!w || (!out && n > 0)) return fail(w, WORLD_E_INVALID_ARG, "NULL argument");
    if (w->poisoned) return WORLD_E_POISONED;
    if (int rc = world_sync(w)) return rc;
    WorldScal sc;
    HIP_TRY(w, copy_now(w, &sc, w->base + w->lay.scal, sizeof(sc), hipMemcpyDeviceToHost));
    // window k has ended once (k + 1) * kMoveWin steps are done; its record is
    // overwritten when window k + kMoveRing starts
    const int64_t started = sc.t > 0 ? (sc.t - 1) / kMoveWin : -1;   // last window begun
    if (n < 0 || first < 0 || (first + n) * kMoveWin > sc.t || (n > 0 && first <= started - kMoveRing))
        return fail(w, WORLD_E_STATE, "requested windows have not ended or are no longer held");
    std::vector<int32_t> ring(size_t(kMoveRing) * (kMoveBins + 1));
    HIP_TRY(w, copy_now(w, ring.data(), w->base + w->lay.mhist, 4 * ring.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i)
        std::memcpy(out + size_t(i) * (kMoveBins + 1), ring.data() + ((first + i) % kMoveRing) * (kMoveBins + 1),
                    4 * (kMoveBins + 1));
    return WORLD_OK;
}

int world_destroy(world_t* w) {
    if (!w) return WORLD_OK;
    if (w->last) (void)wait_launch(w->last->ev);
    {
        // launch tables and graphs of batches that list this world go with it
        // (their streams are synchronised before anything is released)
        std::lock_guard<std::mutex> lk(g_batch_mu);
        const uintptr_t key = reinterpret_cast<uintptr_t>(w);
        for (auto it = g_batches.begin(); it != g_batches.end();) {
            bool has = false;
            for (size_t i = 0; i < it->first.size(); i += kBatchKeyWords) has = has || it->first[i] == key;
            if (has) {
                release_entry(it->second);
                it = g_batches.erase(it);
            } else {
                ++it;
            }
        }
    }
    for (auto& kv : w->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto& kv : w->graph_defs) (void)hipGraphDestroy(kv.second);
    delete w;
    return WORLD_OK;
}

const char* world_last_error(const world_t* w) {
    if (w) return w->err.c_str();
    return g_thread_err.c_str();
}

// Writes the forced-action fields of the descriptor (forced, n_forced,
// forced_on are contiguous) after the table, once the stream is idle.
static int write_forced(world* w, const int8_t* tab, int32_t n, int32_t dflt) {
    HIP_TRY(w, hipStreamSynchronize(w->stream));
    if (n > 0) HIP_TRY(w, copy_now(w, w->base + w->lay.forced, tab, size_t(n), hipMemcpyHostToDevice));
    w->dev.forced = dflt;
    w->dev.n_forced = n;
    w->dev.forced_on = (dflt >= 0 || n > 0) ? 1 : 0;
    static_assert(offsetof(WorldDev, n_forced) == offsetof(WorldDev, forced) + 4 &&
                      offsetof(WorldDev, forced_on) == offsetof(WorldDev, forced) + 8,
                  "forced fields must be contiguous");
    HIP_TRY(w, copy_now(w, w->base + w->lay.desc + offsetof(WorldDev, forced), &w->dev.forced, 12,
                         hipMemcpyHostToDevice));
    return WORLD_OK;
}

int world_set_forced_action(world_t* w, int32_t action) {
    if (!w) return fail(nullptr, WORLD_E_INVALID_ARG, "world is NULL");
    if (w->poisoned) return WORLD_E_POISONED;
    if (action < -1 || action > 4) return fail(w, WORLD_E_INVALID_ARG, "action must be -1..4");
    return write_forced(w, nullptr, 0, action);
}

int world_set_forced_actions(world_t* w, const int32_t* act_by_uid, int32_t n, int32_t default_action) {
    if (!w) return fail(nullptr, WORLD_E_INVALID_ARG, "world is NULL");
    if (w->poisoned) return WORLD_E_POISONED;
    if (n < 0 || (n > 0 && !act_by_uid)) return fail(w, WORLD_E_INVALID_ARG, "n < 0 or a NULL table");
    if (n > forced_capacity(w->cfg))
        return fail(w, WORLD_E_INVALID_ARG, "table longer than max(4 * cap, 4096) uids");
    if (default_action < -1 || default_action > 4) return fail(w, WORLD_E_INVALID_ARG, "default must be -1..4");
    std::vector<int8_t> tab(size_t(std::max(n, 1)));
    for (int i = 0; i < n; ++i) {
        if (act_by_uid[i] < -1 || act_by_uid[i] > 4) return fail(w, WORLD_E_INVALID_ARG, "actions must be -1..4");
        tab[size_t(i)] = int8_t(act_by_uid[i]);
    }
    return write_forced(w, tab.data(), n, default_action);
}

int world_test_stall_lookback(world_t* w, int32_t tile, uint32_t spin_ticks) {
    if (!w) return fail(nullptr, WORLD_E_INVALID_ARG, "world is NULL");
    if (w->poisoned) return WORLD_E_POISONED;
    if (tile < -1 || tile >= tiles_agent(w->cfg)) return fail(w, WORLD_E_INVALID_ARG, "tile out of range");
    const uint32_t ticks = spin_ticks ? spin_ticks : kSpinTicks;
    w->dev.stall_tile = tile;
    w->dev.spin_ticks = ticks;
    HIP_TRY(w, hipStreamSynchronize(w->stream));
    HIP_TRY(w, copy_now(w, w->base + w->lay.desc + offsetof(WorldDev, stall_tile), &tile, sizeof(tile),
                         hipMemcpyHostToDevice));
    HIP_TRY(w, copy_now(w, w->base + w->lay.desc + offsetof(WorldDev, spin_ticks), &ticks, sizeof(ticks),
                         hipMemcpyHostToDevice));
    return WORLD_OK;
}

int world_action_log(world_t* w, int64_t step, int32_t capacity, uint32_t* uid, uint8_t* action, float* logits,
                     float* margin, int32_t* n) {
    if (!w || !n) return fail(w, WORLD_E_INVALID_ARG, "NULL argument");
    if (w->poisoned) return WORLD_E_POISONED;
    const world_config& c = w->cfg;
    if (c.log_steps <= 0) return fail(w, WORLD_E_STATE, "world created without a controller log");
    if (int rc = world_sync(w)) return rc;
    WorldScal sc;
    HIP_TRY(w, copy_now(w, &sc, w->base + w->lay.scal, sizeof(sc), hipMemcpyDeviceToHost));
    if (step < 0 || step >= sc.t || step < sc.t - c.log_steps) return fail(w, WORLD_E_STATE, "step not held in the log");
    const size_t row = size_t(step % c.log_steps);
    int32_t cnt = 0;
    HIP_TRY(w, copy_now(w, &cnt, w->base + w->lay.log_n + 4 * row, 4, hipMemcpyDeviceToHost));
    *n = cnt;
    if (capacity < cnt) return fail(w, WORLD_E_BUFFER_TOO_SMALL, "capacity < agents in the step");
    const size_t base = row * size_t(c.cap);
    if (uid) HIP_TRY(w, copy_now(w, uid, w->base + w->lay.log_uid + 4 * base, 4 * size_t(cnt), hipMemcpyDeviceToHost));
    if (action) HIP_TRY(w, copy_now(w, action, w->base + w->lay.log_act + base, size_t(cnt), hipMemcpyDeviceToHost));
    if (logits)
        HIP_TRY(w, copy_now(w, logits, w->base + w->lay.log_logits + 4 * 5 * base, 4 * 5 * size_t(cnt), hipMemcpyDeviceToHost));
    if (margin && cnt > 0) {
        // the device's decision values: the logits (GRU, arg-max) or the
        // sampling scores 50 l + g of the paper's network, whose Gumbel terms
        // g the same counter-based draws give on the host bit for bit
        std::vector<float> lg(size_t(cnt) * 5);
        std::vector<uint32_t> us(static_cast<size_t>(cnt));
        HIP_TRY(w, copy_now(w, lg.data(), w->base + w->lay.log_logits + 4 * 5 * base, 4 * lg.size(), hipMemcpyDeviceToHost));
        HIP_TRY(w, copy_now(w, us.data(), w->base + w->lay.log_uid + 4 * base, 4 * us.size(), hipMemcpyDeviceToHost));
        const bool net_ctrl = is_net(c);
        for (int i = 0; i < cnt; ++i) {
            float sc[5];
            for (int a = 0; a < 5; ++a) sc[a] = lg[size_t(i) * 5 + a];
            if (net_ctrl) {
                const Draw4 d0 = philox(us[size_t(i)], uint32_t(step), kAct, 0u, w->dev.seed_lo, w->dev.seed_hi);
                const Draw4 d1 = philox(us[size_t(i)], uint32_t(step), kAct, 1u, w->dev.seed_lo, w->dev.seed_hi);
                const uint32_t words[5] = {d0.x, d0.y, d0.z, d0.w, d1.x};
                for (int a = 0; a < 5; ++a) sc[a] = 50.0f * sc[a] + gumbel_of_word(words[a]);
            }
            int best = 0;
            for (int a = 1; a < 5; ++a)
                if (sc[a] > sc[best]) best = a;
            float second = -INFINITY;
            for (int a = 0; a < 5; ++a)
                if (a != best && sc[a] > second) second = sc[a];
            margin[i] = sc[best] - second;
        }
    }
    return WORLD_OK;
}

int world_test_philox(const uint32_t* d_ctr, size_t n, uint32_t k0, uint32_t k1, uint32_t* d_out, void* stream) {
    if (!d_ctr || !d_out) return fail(nullptr, WORLD_E_INVALID_ARG, "NULL argument");
    if (n == 0) return WORLD_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_test_philox, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, d_ctr, n, k0, k1, d_out);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(nullptr, WORLD_E_HIP, hipGetErrorString(e));
    return WORLD_OK;
}

int world_test_gauss(const uint32_t* d_a, const uint32_t* d_b, size_t n, float* d_z0, float* d_z1, void* stream) {
    if (!d_a || !d_b || !d_z0 || !d_z1) return fail(nullptr, WORLD_E_INVALID_ARG, "NULL argument");
    if (n == 0) return WORLD_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_test_gauss, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, d_a, d_b, n, d_z0, d_z1);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(nullptr, WORLD_E_HIP, hipGetErrorString(e));
    return WORLD_OK;
}

int world_test_gumbel(const uint32_t* d_words, size_t n, float* d_g, void* stream) {
    if (!d_words || !d_g) return fail(nullptr, WORLD_E_INVALID_ARG, "NULL argument");
    if (n == 0) return WORLD_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_test_gumbel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, d_words, n, d_g);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(nullptr, WORLD_E_HIP, hipGetErrorString(e));
    return WORLD_OK;
}

int world_phase_times(world_t* w, int32_t K, float* ms) {
    TraceRange trace("world_phase_times K=%d", K);
    if (!w || !ms) return fail(w, WORLD_E_INVALID_ARG, "NULL argument");
    if (w->poisoned) return WORLD_E_POISONED;
    if (K < 1) return fail(w, WORLD_E_INVALID_ARG, "K must be >= 1");
    const int np = 2;
    const int* hp = w->host_bp.data();
    Batch b{w->tv.w, w->tv.block_pre, 1, w->act_rows, static_cast<const WorldDev*>(w->d_dev), w->cfg.cap, w->dev.ctrl,
            w->dev.dyn, net_wide(w->tv.slots), w->act_waves, w->tile, w->tv.may_stream};
    hipStream_t s = w->stream;
    // each kernel between start / end events stamped by its own dispatch
    std::vector<hipEvent_t> ev(size_t(K) * 6);
    for (auto& e : ev) HIP_TRY(w, hipEventCreate(&e));
    hipError_t le = hipSuccess;
    for (int k = 0; k < K && le == hipSuccess; ++k) {
        hipEvent_t* e = ev.data() + size_t(k) * 6;
        launch_act(b, hp[kPreAct * np + 1], s, e[0], e[1]);
        hipExtLaunchKernelGGL(k_move, dim3(hp[kPreMove * np + 1]), dim3(64), 0, s, e[2], e[3], 0, b);
        launch_claim(b, hp[kPreClaim * np + 1], s, e[4], e[5]);
        le = hipGetLastError();
    }
    hipError_t se = hipStreamSynchronize(s);
    double acc[3] = {0, 0, 0};
    for (int k = 0; k < K && le == hipSuccess && se == hipSuccess; ++k) {
        hipEvent_t* e = ev.data() + size_t(k) * 6;
        for (int p = 0; p < 3; ++p) {
            float v = 0.f;
            if (hipEventElapsedTime(&v, e[2 * p], e[2 * p + 1]) == hipSuccess) acc[p] += v;
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (le != hipSuccess) return fail(w, WORLD_E_HIP, std::string("phase launch: ") + hipGetErrorString(le));
    if (se != hipSuccess) return fail(w, WORLD_E_HIP, std::string("phase sync: ") + hipGetErrorString(se));
    for (int p = 0; p < 3; ++p) ms[p] = float(acc[p] / K);
    return check_device_error(w);
}

int world_test_copy(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst || bytes % 16 != 0) return fail(nullptr, WORLD_E_INVALID_ARG, "bad copy arguments");
    if (bytes == 0) return WORLD_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t n = bytes / 16;
    const int grid = int(std::min<size_t>((n + kBlock - 1) / kBlock, size_t(device_cus()) * 16));
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(kBlock), 0, s, static_cast<const int4*>(src), static_cast<int4*>(dst), n);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(nullptr, WORLD_E_HIP, hipGetErrorString(e));
    return WORLD_OK;
}

// Checks shared by the batched entry points: a non-empty list of distinct,
// healthy worlds on one stream with one controller and one rule set.
static int check_batch(world_t* const* ws, int32_t n, int32_t K) {
    if (!ws || n < 1) return fail(nullptr, WORLD_E_INVALID_ARG, "empty world list");
    if (K < 1) return fail(nullptr, WORLD_E_INVALID_ARG, "K must be >= 1");
    for (int i = 0; i < n; ++i) {
        if (!ws[i]) return fail(nullptr, WORLD_E_INVALID_ARG, "NULL world in list");
        if (ws[i]->poisoned) return WORLD_E_POISONED;
        if (ws[i]->stream != ws[0]->stream) return fail(nullptr, WORLD_E_INVALID_ARG, "worlds must share one stream");
        if (ws[i]->cfg.controller != ws[0]->cfg.controller || ws[i]->cfg.dynamics != ws[0]->cfg.dynamics)
            return fail(nullptr, WORLD_E_INVALID_ARG, "worlds of one batch must use the same controller and dynamics");
    }
    {
        // a world listed twice would be stepped by two block ranges at once
        std::vector<const world*> sorted(ws, ws + n);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            return fail(nullptr, WORLD_E_INVALID_ARG, "a world is listed twice");
    }
    return WORLD_OK;
}

int world_step_many(world_t* const* ws, int32_t n, int32_t K) {
    TraceRange trace("world_step_many n=%d K=%d", n, K);
    if (int rc = check_batch(ws, n, K)) return rc;
    return batch_step(ws, n, K);
}

// ---- batched steps without allocation -----------------------------------
// world_step_many keeps each batch's launch table in device memory it
// allocates (and caches).  For callers that cannot allocate (graph capture,
// tight serving loops), world_step_many_noalloc writes the table into a
// fixed device array instead, with small fill kernels whose arguments carry
// the table (no copy from host memory), and launches the per-phase kernels
// (no graph instantiation).  Each GPU holds its own copy of the array for the
// life of the process; its device address comes from hipGetSymbolAddress,
// once per device.  Every call rewrites the whole table before its step
// kernels read it; calls that overlap on one GPU (other streams or threads)
// race on it.
constexpr int kNoAllocMaxWorlds = 2048;
constexpr size_t kScratchBytes = 49152;
static_assert(kScratchBytes >= (sizeof(void*) * kNoAllocMaxWorlds + 15) / 16 * 16 +
                                   sizeof(int) * size_t(kPreKinds) * (kNoAllocMaxWorlds + 1),
              "scratch holds the launch table of the largest batch");
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kFillChunk = 96;   // worlds per fill launch (arguments stay under 4 KB)
struct TableChunk {
    int n_total;                          // worlds in the table
    int first;                            // first world of this chunk
    int count;                            // worlds in this chunk
    const WorldDev* w[kFillChunk];        // their descriptors
    int pre[kPreKinds][kFillChunk + 1];   // prefix entries first .. first + count
};
static_assert(sizeof(TableChunk) < 4000, "kernel arguments");

__global__ void k_fill_table(char* table, TableChunk c) {
    const int i = threadIdx.x;
    const size_t ptr_bytes = (sizeof(void*) * size_t(c.n_total) + 15) / 16 * 16;
    const WorldDev** wp = reinterpret_cast<const WorldDev**>(table);
    int* pre = reinterpret_cast<int*>(table + ptr_bytes);
    if (i < c.count) wp[c.first + i] = c.w[i];
    if (i <= c.count)
        for (int k = 0; k < kPreKinds; ++k) pre[k * (c.n_total + 1) + c.first + i] = c.pre[k][i];
}

static std::mutex g_scratch_mu;
static std::map<int, char*> g_scratch_addr;   // device -> address of its `scratch`

// Device address of the current device's `scratch` (looked up once per device).
static int scratch_address(char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, WORLD_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it == g_scratch_addr.end()) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(nullptr, WORLD_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        it = g_scratch_addr.emplace(dev, static_cast<char*>(p)).first;
    }
    *out = it->second;
    return WORLD_OK;
}

int world_step_many_noalloc(world_t* const* ws, int32_t n, int32_t K) {
    TraceRange trace("world_step_many_noalloc n=%d K=%d", n, K);
    if (int rc = check_batch(ws, n, K)) return rc;
    if (n > kNoAllocMaxWorlds) return fail(nullptr, WORLD_E_INVALID_ARG, "more than 2048 worlds in one batch");
    char* table = nullptr;
    if (int rc = scratch_address(&table)) return rc;
    world* w0 = ws[0];
    hipStream_t s = w0->stream;
    std::vector<const world*> list(ws, ws + n);
    const std::vector<int> bp = batch_prefix(list, w0->act_waves, w0->tile);
    int slots = 0, streams = 0;
    for (const world* x : list) {
        slots += x->cfg.cap;
        streams |= may_stream(x);
    }
    for (int first = 0; first < n; first += kFillChunk) {
        TableChunk c;
        std::memset(&c, 0, sizeof(c));
        c.n_total = n;
        c.first = first;
        c.count = std::min(kFillChunk, n - first);
        for (int i = 0; i < c.count; ++i) c.w[i] = list[size_t(first + i)]->d_dev;
        for (int k = 0; k < kPreKinds; ++k)
            for (int i = 0; i <= c.count; ++i) c.pre[k][i] = bp[size_t(k) * (n + 1) + first + i];
        hipLaunchKernelGGL(k_fill_table, dim3(1), dim3(128), 0, s, table, c);
    }
    HIP_TRY(w0, hipGetLastError());
    const size_t ptr_bytes = align_up(sizeof(void*) * size_t(n), 16);
    Batch b{reinterpret_cast<const WorldDev* const*>(table), reinterpret_cast<const int*>(table + ptr_bytes), n,
            w0->act_rows, n == 1 ? static_cast<const WorldDev*>(w0->d_dev) : nullptr, w0->cfg.cap, w0->dev.ctrl,
            w0->dev.dyn, net_wide(slots), w0->act_waves, w0->tile, streams};
    for (int k = 0; k < K; ++k) HIP_TRY(w0, launch_step(b, bp.data(), n, s));
    return mark_launch(ws, n);
}

}  // extern "C"
