#!/usr/bin/env python
"""Benchmark of the fused world step on one MI355X.

Metric: agent-steps/s on the 200 x 400 world with ~4k agents (every agent of
the population acts once per step).  The workload (``m1_4k``): 200 x 400 grid,
4608 agent slots, 4096 initial agents, Bernoulli(0.3) resources, regrowth
rates x5, 7x7x2+1 observation, GRU hidden 32, seed 0.  W warm-up steps, then
exactly K timed steps (world_step in chunks of --chunk steps) between two
device synchronisations.  Inputs are resident in HBM before timing starts.

Also reported:
* ``roofline``: the dominant kernel (the act phase: observation + GRU) timed
  with HIP events on the world's stream in a separate per-phase pass, its
  algorithmic bytes per launch (live agents x bytes each agent must read and
  write + the grid) against the 8 TB/s HBM peak; ``traffic`` from the
  committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary when the kernel source
  still matches it.  The kernel durations come from a per-phase pass over
  the same steps (from the same state) whose launches carry start / end
  events stamped by their own dispatch; ``kernels`` lists all three.
* ``cpu_baseline``: the oracle (plain C, one thread) on a bounded sample of
  the same workload on the host cores.
* ``paper_dynamics``: the paper's own world (``paper1k``: its constants, its
  network and its rules -- stacking, walls, energy clip, offspring on the
  parent's cell) timed by the wall clock; the paper reports 1e6 steps of this
  world in 20 minutes on one GPU (App. B.4), quoted beside it as context.
* ``lab``: the lab environments of Sec. 2.2 -- agents evolved in the paper's
  network world (net1k) tested alone in 40 x 40 worlds without regrowth at
  three densities (greediness) and with reproduction (peer pressure): all
  lab worlds in shared launches, their rate against a sample of them stepped
  one at a time, and the greediness / efficiency statistics.
* ``paper_network``: the same 200 x 400 world with ~4k agents driven by the
  paper's controller (App. B.5: CNN + LSTM(4), 2445 parameters, sampled
  actions; workload ``net_m1_4k``): wall-clock agent-steps/s, per-kernel
  event times, and the act kernel (k_act_net_wide, the network act kernel
  compiled for five waves per SIMD) against the HBM roofline with its
  algorithmic bytes and flops per agent.
* ``cache_exceeding``: the dense start of cfg2 (12k-16k agents, beyond the
  last-level cache); ``batched``: 64 uneven worlds in shared launches,
  autotuned, against the same worlds stepped one at a time; ``served``: the
  continuous-batching server over a Poisson arrival trace, with p50/p99
  per-step latency; ``ecology_metrics``: the App. C metrics over the timed
  steps.
* ``--only net|paper|lab`` runs one of these legs alone and prints it (for
  profiling).

``--gpus N`` with N > 1 is refused: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "act_m1_4k_traffic.txt")
NET_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "act_net_m1_4k_traffic.txt")
KERNEL_SOURCES = ["rng.h", "world_dev.h", "phases.h", "kernels.h"]
NET_KERNEL_SOURCES = KERNEL_SOURCES + ["net.h"]
FP32_VECTOR_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(sources=None) -> str:
    h = hashlib.sha256()
    for f in sources or KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2302_09334_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def observed_inputs(snap: dict, cfg: dict) -> tuple[np.ndarray, np.ndarray]:
    """Per agent: the non-zero binary inputs (resource and occupancy windows;
    outside cells read as no resource and occupied) and the input rows the act
    kernel reads for them (per window the rows of its ones, or the rows of its
    zeros plus the window's column total when ones are the majority)."""
    H, W, rho = cfg["H"], cfg["W"], cfg["obs_radius"]
    w2 = (2 * rho + 1) ** 2
    R = np.zeros((H + 2 * rho, W + 2 * rho), np.int32)
    R[rho:rho + H, rho:rho + W] = snap["R"]
    O = np.ones((H + 2 * rho, W + 2 * rho), np.int32)
    O[rho:rho + H, rho:rho + W] = 0
    O[snap["row"] + rho, snap["col"] + rho] = 1
    nr = np.zeros(snap["n_live"], np.int64)
    no = np.zeros(snap["n_live"], np.int64)
    for dy in range(-rho, rho + 1):
        for dx in range(-rho, rho + 1):
            r = snap["row"] + rho + dy
            c = snap["col"] + rho + dx
            nr += R[r, c]
            no += O[r, c]
    rows = sum(np.where(2 * m > w2, w2 - m + 1, m) for m in (nr, no))
    return nr + no, rows


def act_bytes_per_agent(cfg: dict, rows_mean: float) -> float:
    """Bytes the act phase must move per agent: the precomputed recurrent
    projection (3*hidden floats), the input biases, the head, the energy row,
    one 3*hidden row per input row read (see observed_inputs), the hidden
    state in and out, and the agent's scalars (slot, cell, energy, uid in;
    action out)."""
    hd = cfg["hidden"]
    rw = 3 * hd * 4
    return (rw + rw + (5 * hd + 5) * 4 + rw + rows_mean * rw + 2 * hd * 4 + 21)


# Share of the live list whose recurrent projection runs in the move kernel
# (the library's build default, ECO_PROJ_MOVE_EIGHTHS = 4); the rest, minus
# the agents that died in the move phase, runs in the claim kernel.
PROJ_MOVE_SHARE = 4 / 8


def proj_bytes_per_agent(cfg: dict) -> float:
    """Bytes of the recurrent projection per agent: W_hh, b_hh and h in, the
    projection out."""
    hd = cfg["hidden"]
    return 3 * hd * hd * 4 + 3 * hd * 4 + hd * 4 + 3 * hd * 4


# Move phase, per agent: its 32-byte record in, the move-claim word and the
# two resource bytes of the source and target cell, the per-slot state out
# (energy, age, streak, cell, previous cell: 20 bytes, alive and ate: 2),
# both occupancy words, the post-move record and the next record (32 + 32),
# the live-list entry (4) and the eaten resource byte.
MOVE_BYTES_PER_AGENT = 32 + 8 + 2 + 22 + 8 + 64 + 4 + 1
# Claim phase, per agent: the post-move record (32), the move-claim clear (8),
# the claim word (4); per eligible agent the 24 occupancy words (96) and the
# 8 birth keys (64) of its neighbourhood.  Regrowth, per cell: the resource
# byte in and out.
CLAIM_BYTES_PER_AGENT = 32 + 8 + 4
CLAIM_BYTES_PER_ELIGIBLE = 96 + 64


def step_algorithmic_bytes(cfg: dict, P: int, acting, rows_read, births):
    """Bytes one step must move (per step of a window; numpy arrays in, an
    array out), counted as the benchmark definition's sparse-input form: per
    acting agent the recurrent weights W_hh, both bias vectors, the head (W_o,
    b_o), the hidden state in and out with about 40 bytes of scalars (8 hd +
    40) and the energy input's row; the input rows the act phase actually read
    (the device counts them: per binary window the rows of its ones, or its
    column total and the rows of its zeros); the parent's genome read and the
    child's written per birth; the grid (resource byte and occupancy word, in
    and out)."""
    hd = cfg["hidden"]
    rw = 3 * hd * 4
    per_agent = 3 * hd * hd * 4 + 2 * rw + (5 * hd + 5) * 4 + 8 * hd + 40 + rw
    return (np.asarray(acting, np.float64) * per_agent + np.asarray(rows_read, np.float64) * rw
            + np.asarray(births, np.float64) * 8 * P + cfg["H"] * cfg["W"] * 10)


def kernel_window_bytes(cfg: dict, P: int, acting, rows_read, births_prev, deaths, claim_wins) -> dict:
    """Algorithmic bytes per launch of each phase kernel, averaged over a
    window (arrays per step): act = the children of the previous step (parent
    genome in, child genome out) + per acting agent act_bytes_per_agent with
    the rows it read + the grid once; move = its per-agent records + its share
    of the recurrent projection; claim = the rest of the projection (the
    survivors among those positions), its per-agent records, the
    neighbourhood of each birth-claim winner, the grid's resource bytes."""
    acting = np.asarray(acting, np.float64)
    hd = cfg["hidden"]
    rw = 3 * hd * 4
    act = (acting * act_bytes_per_agent(cfg, 0.0) + np.asarray(rows_read, np.float64) * rw
           + np.asarray(births_prev, np.float64) * 8 * P + cfg["H"] * cfg["W"] * 5)
    pb = proj_bytes_per_agent(cfg)
    move = acting * (MOVE_BYTES_PER_AGENT + PROJ_MOVE_SHARE * pb)
    claim = ((1 - PROJ_MOVE_SHARE) * (acting - np.asarray(deaths, np.float64)) * pb + acting * CLAIM_BYTES_PER_AGENT
             + np.asarray(claim_wins, np.float64) * CLAIM_BYTES_PER_ELIGIBLE + 2 * cfg["H"] * cfg["W"])
    return {"act": float(act.mean()), "move": float(move.mean()), "claim": float(claim.mean())}


def read_traffic_per_agent(src_hash: str, rows, path: str = TRAFFIC_FILE):
    """HBM bytes per acting agent of the act kernel variant `rows` (input rows
    per round trip, or "rows_waves" with the agents per block), from the
    committed counter summary (measured on the same bench window), or None
    when the kernel sources changed since."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != src_hash:
        return None
    try:
        return float(kv[f"hbm_bytes_per_acting_agent_rows{rows}"])
    except (KeyError, ValueError):
        return None


def read_traffic(src_hash: str, rows, path: str = TRAFFIC_FILE):
    """HBM bytes per launch of the act kernel compiled for `rows` input rows
    per round trip (None: the network's act kernel), from the committed
    counter summary (None when the kernel sources changed since it was
    taken)."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != src_hash:
        return None
    try:
        return float(kv["hbm_bytes_per_launch" if rows is None else f"hbm_bytes_per_launch_rows{rows}"])
    except (KeyError, ValueError):
        return None


# The paper's network (App. B.5), per agent and act launch: every parameter
# read once (2445 floats), the LSTM state in and out (8 floats each way), the
# agent record in (32 B), the action out (record word and action byte) and the
# move-claim word (8 B); the grid (resource byte and occupancy word per cell)
# once per launch.  Multiply-adds: conv1 8x8 outputs x 4 x 27, conv2 4x4 x 8 x
# 36, LSTM 16 x (78 + 4), dense 8 x 82, head 5 x 8.
NET_PARAMS = 2445
NET_ACT_BYTES_PER_AGENT = 4 * NET_PARAMS + 2 * 32 + 32 + 5 + 8
NET_MACS_PER_AGENT = 64 * 4 * 27 + 16 * 8 * 36 + 16 * 82 + 8 * 82 + 5 * 8


def net_run(args) -> dict:
    """The ~4k-agent world with the paper's network: warm-up, then exactly
    --net-steps steps timed by the wall clock between two synchronisations
    (graph launches of --chunk steps), then a per-phase pass from the same
    state for the kernel durations."""
    import torch
    from paper_2302_09334_amd import workloads, world
    cfg = workloads.WORKLOADS["net_m1_4k"]
    stream = torch.cuda.Stream()
    w = world.World(cfg, args.seed, stream=stream, mode="graph")
    assert w.n_params == NET_PARAMS
    done = 0
    while done < args.net_warmup:
        k = min(args.chunk, args.net_warmup - done)
        w.step(k)
        done += k
    w.sync()
    start = w.snapshot(hidden=True, theta=True)
    t_first = start["t"]
    w.step(min(args.chunk, args.net_steps))   # graph capture outside the timed region
    w.sync()
    w.load(start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < args.net_steps:
        k = min(args.chunk, args.net_steps - done)
        w.step(k)
        done += k
    w.sync()
    wall = time.perf_counter() - t0
    ctr = w.counters(t_first, args.net_steps)
    acting = np.concatenate([[start["n_live"]], ctr["n_live"][:-1]])
    w.load(start)
    ph = w.phase_times(args.net_phase_steps)
    pc = w.counters(t_first, args.net_phase_steps)
    n_act = float(np.concatenate([[start["n_live"]], pc["n_live"][:-1]]).mean())
    grid_bytes = cfg["H"] * cfg["W"] * 5
    act_bytes = n_act * NET_ACT_BYTES_PER_AGENT + grid_bytes
    elig = float((start["streak"] >= cfg["T_repr"]).sum())
    kbytes = {"act": act_bytes, "move": n_act * MOVE_BYTES_PER_AGENT,
              "claim": n_act * CLAIM_BYTES_PER_AGENT + elig * CLAIM_BYTES_PER_ELIGIBLE + 2 * cfg["H"] * cfg["W"]}
    kms = {"act": float(ph[0]), "move": float(ph[1]), "claim": float(ph[2])}
    act_s = kms["act"] * 1e-3
    achieved = act_bytes / act_s / 1e9
    tflops = n_act * 2 * NET_MACS_PER_AGENT / act_s / 1e12
    src_hash = kernel_source_hash(NET_KERNEL_SOURCES)
    w.close()
    out = {
        "workload": "net_m1_4k: 200x400 grid, cap 4608, 4096 initial agents, resources Bernoulli(0.3), "
                    "regrowth x5.0, obs 15x15x3, CNN + LSTM(4) + dense 8 + 5 (2445 parameters), actions "
                    "sampled at temperature 1/50, seed %d, steps %d..%d" % (args.seed, t_first,
                                                                           t_first + args.net_steps - 1),
        "metric": "agent-steps/s", "value": float(acting.sum()) / wall, "ms_per_step": wall / args.net_steps * 1e3,
        "steps": args.net_steps, "warmup": args.net_warmup, "launch_mode": "graph",
        "n_live_mean": float(acting.mean()), "births": int(ctr["births"].sum()), "deaths": int(ctr["deaths"].sum()),
        "kernels": {k: {"ms_per_launch": kms[k], "algorithmic_bytes": kbytes[k],
                        "GBps": kbytes[k] / (kms[k] * 1e-3) / 1e9} for k in kms},
        "roofline": {
            "kernel": "k_act_net_wide (observation, CNN, LSTM, dense layers, sampling; one wave per agent; "
                      "the network act kernel compiled for five waves per SIMD, used when a launch has more "
                      "agent slots than four waves per SIMD hold)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": read_traffic(src_hash, None, NET_TRAFFIC_FILE),
            "algorithmic_bytes_per_launch": act_bytes, "launch_ms": kms["act"],
            "act_per_agent_bytes": NET_ACT_BYTES_PER_AGENT, "agents_per_launch": n_act,
            "flops_per_agent": 2 * NET_MACS_PER_AGENT, "achieved_TFLOPs": tflops,
            "fp32_vector_peak_TFLOPs": FP32_VECTOR_PEAK_TFLOPS,
            "kernel_source_sha256_16": src_hash,
        },
    }
    log(f"[bench] paper network: {out['value'] / 1e6:.1f} M agent-steps/s, {out['ms_per_step'] * 1e3:.1f} us/step, "
        f"{out['n_live_mean']:.0f} agents; k_act_net {kms['act'] * 1e3:.2f} us ({achieved:.0f} GB/s, "
        f"{tflops:.1f} TFLOP/s), move {kms['move'] * 1e3:.2f} us, claim {kms['claim'] * 1e3:.2f} us")
    return out


def cpu_baseline(cfg: dict, seed: int, seconds: float) -> dict:
    import oracle
    ow = oracle.OracleWorld(oracle.OracleConfig.from_dict(cfg), seed)
    acted = 0
    steps = 0
    t0 = time.perf_counter()
    while True:
        n = ow.n_live
        ow.step()
        acted += n
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds and steps >= 3:
            break
    ow.close()
    return {"value": acted / el, "unit": "agent-steps/s", "cores": 1, "kind": "oracle",
            "host_cores": len(os.sched_getaffinity(0)),
            "sample": f"steps 0..{steps - 1} of the same workload from its seed ({acted} agent-steps, "
                      f"{el:.1f} s, plain C oracle, one thread; initialisation excluded)"}


def hbm_honest_run(args, rows: int) -> dict:
    """The 200 x 400 world with 16384 slots and 12000 initial agents over its
    first --m2-steps steps, while 12k-16k agents are alive (the population
    later settles near 4k): a step then moves well over the 256 MB last-level
    cache, so the rate is not helped by cache hits the smaller workload may
    get.  One world is timed by the wall clock; a second one from the same
    seed (the same trajectory) gives the kernel durations."""
    import torch
    from paper_2302_09334_amd import workloads, world
    cfg = workloads.WORKLOADS["cfg2"]
    steps = args.m2_steps
    stream = torch.cuda.Stream()
    w = world.World(cfg, args.seed, stream=stream, mode="kernels")
    w.set_tuning(rows)
    s0 = w.snapshot()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w.step(steps)
    w.sync()
    wall = time.perf_counter() - t0
    c = w.counters(0, steps)
    P = w.n_params
    w.close()
    w2 = world.World(cfg, args.seed, stream=stream, mode="kernels")
    w2.set_tuning(rows)
    ph = w2.phase_times(steps)
    w2.close()
    # bytes from the window's own device counters, as for the headline (the
    # world starts from its seed: no children are pending at step 0)
    acting_v = np.concatenate([[int(s0["n_live"])], c["n_live"][:-1]]).astype(np.float64)
    acting = int(acting_v.sum())
    n = acting / steps
    births_prev = np.concatenate([[0], c["births"][:-1]])
    kb = kernel_window_bytes(cfg, P, acting_v, c["rows_read"], births_prev, c["deaths"], c["claim_wins"])
    step_b = step_algorithmic_bytes(cfg, P, acting_v, c["rows_read"], c["births"])
    out = {"workload": "cfg2: 200x400 grid, cap 16384, 12000 initial agents, resources Bernoulli(0.3), "
                       "regrowth x5.0, obs 7x7x2+1, GRU 32, seed %d, steps 0..%d" % (args.seed, steps - 1),
           "steps": steps, "agent_steps_per_s": acting / wall, "ms_per_step": wall / steps * 1e3,
           "n_live_mean": n, "births_mean": float(c["births"].mean()),
           "kernel_ms": {"act": float(ph[0]), "move": float(ph[1]), "claim": float(ph[2])},
           "act_GBps": kb["act"] / (float(ph[0]) * 1e-3) / 1e9, "move_GBps": kb["move"] / (float(ph[1]) * 1e-3) / 1e9,
           "claim_GBps": kb["claim"] / (float(ph[2]) * 1e-3) / 1e9,
           "act_frac": kb["act"] / (float(ph[0]) * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "act_input_rows_read_per_agent": float(np.sum(c["rows_read"])) / acting,
           "act_algorithmic_MB_per_launch": kb["act"] / 1e6,
           "step_algorithmic_MB": float(step_b.mean()) / 1e6,
           "step_frac": float(step_b.sum()) / wall / 1e9 / HBM_PEAK_GBS,
           "bytes_basis": "the headline's formulas (kernel bytes per launch, step bytes) over this window's device "
                          "counters; the rate and step_frac are per-phase launches timed by the wall clock"}
    log(f"[bench] cfg2 (cache-exceeding, {n:.0f} agents): {out['agent_steps_per_s'] / 1e6:.1f} M agent-steps/s, "
        f"{out['ms_per_step'] * 1e3:.1f} us/step, act {out['act_GBps']:.0f} GB/s, move {out['move_GBps']:.0f} GB/s, "
        f"claim {out['claim_GBps']:.0f} GB/s; step {out['step_algorithmic_MB']:.1f} MB, frac {out['step_frac']:.3f}")
    return out


# Act rows per round trip of the cache-exceeding leg when it runs alone (the
# calibration of the main leg picks this value at 200 x 400).
ONLY_M2_ROWS = 8


def batched_run(args) -> dict:
    """Uneven worlds (grid 64x128..200x400, caps 512..8192, 10% initial agents,
    rate scale U[0.5, 2]) in shared launches, autotuned, against the same
    worlds stepped one at a time on the same GPU."""
    from paper_2302_09334_amd import batch, tune, workloads
    entries = workloads.batch_manifest(args.batch_worlds, seed=0)
    log(f"[bench] batched: {len(entries)} worlds, warm-up {args.batch_warmup}, timed {args.batch_steps}")
    b = batch.WorldBatch(entries, mode="graph")
    if args.batch_warmup > 0:
        b.step(args.batch_warmup)
    b.sync()
    tuned = tune.autotune(b, trial_steps=100)   # restores the state it started from
    best = tuned["best"]
    log(f"[bench] batched autotune: {best}")
    K = best["K"]
    wall, chunk_ms = batch.time_chunks(b.step, args.batch_steps, K, b.stream)
    b.sync()
    agent_steps = b.acting_agents(args.batch_warmup, args.batch_steps)
    # the batched launch against the HBM roofline: every world's step bytes
    # over the window (its own counters), over the batch's wall time
    from paper_2302_09334_amd import world as wmod
    step_bytes = 0.0
    for wd in b.worlds:
        first = args.batch_warmup
        c = wd.counters(first, args.batch_steps)
        n0 = wd.counters(first - 1, 1)["n_live"][0] if first > 0 else wd.cfg["n_init"]
        acting = np.concatenate([[n0], c["n_live"][:-1]])
        step_bytes += float(step_algorithmic_bytes(wd.cfg, wmod.dims(wd.cfg)[1], acting, c["rows_read"],
                                                   c["births"]).sum())
    n_agents = sum(w.snapshot()["n_live"] for w in b.worlds)
    b.close()
    seq = batch.run_sequential(entries, args.batch_warmup, args.batch_steps, 100, mode="graph")
    gbps = step_bytes / wall / 1e9
    out = {"worlds": len(entries), "steps": args.batch_steps, "warmup": args.batch_warmup,
           "agent_steps_per_s": agent_steps / wall, "ms_per_step": wall / args.batch_steps * 1e3,
           "step_ms_p50": float(np.percentile(chunk_ms / K, 50)), "step_ms_p99": float(np.percentile(chunk_ms / K, 99)),
           "roofline": {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbps / HBM_PEAK_GBS,
                        "basis": "all worlds' step algorithmic bytes (same formula as the headline's step_frac, "
                                 "from each world's counters) over the batch's wall time"},
           "live_agents_end": int(n_agents), "tuned": best,
           "sequential_plain": {"agent_steps_per_s": seq["agent_steps_per_s"], "wall_s": seq["wall_s"]},
           "speedup_vs_sequential": (agent_steps / wall) / seq["agent_steps_per_s"]}
    log(f"[bench] batched {out['agent_steps_per_s'] / 1e6:.1f} M agent-steps/s vs sequential "
        f"{seq['agent_steps_per_s'] / 1e6:.1f} M")
    return out


def served_run(args) -> dict:
    """Poisson(20/s) simulation requests (grid from the uneven set, caps
    512..8192, steps U[500, 5000], GRU 16 or 32) admitted against the HBM
    budget and continuously batched."""
    from paper_2302_09334_amd import serve, workloads
    trace = workloads.serve_trace(duration_s=args.serve_seconds, rate_hz=20.0, seed=0)
    reqs = serve.requests_from_trace(trace)
    log(f"[bench] served: {len(reqs)} requests over {args.serve_seconds:.0f} s of arrivals")
    be = serve.HipBackend(mode="kernels")
    srv = serve.Server(be, budget_bytes=int(args.serve_budget_gb * 1e9), K=50)
    results, m = srv.run(reqs, duration=args.serve_seconds, realtime=True,
                         progress=lambda t, done, act, q: log(f"[bench] served t={t:.0f} s: {done} done, "
                                                              f"{act} active, {q} queued"))
    be.shutdown()
    m["fixture"] = ("M4: Poisson(20/s) arrivals for 600 s" if args.serve_seconds >= 600 else
                    f"M4 truncated to {args.serve_seconds:.0f} s of arrivals (the full 600 s run: "
                    "profiles/served_cfg4_600s.txt)")
    m["arrival_window_s"] = args.serve_seconds
    m["rate_hz"] = 20.0
    m["offered_steps_per_s"] = 20.0 * float(np.mean([r.steps for r in reqs])) if reqs else 0.0
    log(f"[bench] served {m['requests']} requests: {m['agent_steps_per_s'] / 1e6:.1f} M agent-steps/s, "
        f"p50 {m['step_ms_p50']:.3f} ms p99 {m['step_ms_p99']:.3f} ms per step")
    return m


# App. B.4: 1e6 steps of the paper's world (at most 1000 agents) in about 20
# minutes on one GPU (JAX; the GPU model is not named).
PAPER_STEPS_PER_S = 1e6 / (20 * 60)


def paper_run(args) -> dict:
    """The paper's world with its own dynamics and network (paper1k)."""
    import torch
    from paper_2302_09334_amd import workloads, world
    cfg = workloads.WORKLOADS["paper1k"]
    stream = torch.cuda.Stream()
    w = world.World(cfg, args.seed, stream=stream, mode="graph")
    done = 0
    while done < args.paper_warmup:
        k = min(args.chunk, args.paper_warmup - done)
        w.step(k)
        done += k
    w.sync()
    start = w.snapshot(hidden=True, theta=True)
    t_first = start["t"]
    w.step(min(args.chunk, args.paper_steps))
    w.sync()
    w.load(start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < args.paper_steps:
        k = min(args.chunk, args.paper_steps - done)
        w.step(k)
        done += k
    w.sync()
    wall = time.perf_counter() - t0
    ctr = w.counters(t_first, args.paper_steps)
    acting = np.concatenate([[start["n_live"]], ctr["n_live"][:-1]])
    w.load(start)
    ph = w.phase_times(args.net_phase_steps)
    w.close()
    steps_per_s = args.paper_steps / wall
    out = {
        "workload": "paper1k: the paper's world (App. B.4): 200x400 grid, at most 1000 agents, 330 initial, resources "
                    "Bernoulli(0.2), its network (15x15x3, CNN + LSTM(4), sampled at T = 1/50) and rules (stacking, "
                    "walls, energy in 1/40 units with E0 = E_max = 120, decay 1, gain 40, reproduction after 140 steps "
                    "above 0, death after 200 below or past age 650, regrowth 0.002 c(x) + 5e-5, alpha 200), seed %d, "
                    "steps %d..%d" % (args.seed, t_first, t_first + args.paper_steps - 1),
        "metric": "agent-steps/s", "value": float(acting.sum()) / wall, "steps_per_s": steps_per_s,
        "ms_per_step": wall / args.paper_steps * 1e3, "steps": args.paper_steps, "warmup": args.paper_warmup,
        "n_live_mean": float(acting.mean()), "births": int(ctr["births"].sum()), "deaths": int(ctr["deaths"].sum()),
        "kernel_ms": {"act": float(ph[0]), "move": float(ph[1]), "claim": float(ph[2])},
        "million_steps_s": 1e6 / steps_per_s,
        "paper_reported": {"steps_per_s": PAPER_STEPS_PER_S, "million_steps_s": 1200.0,
                           "hardware": "one GPU, JAX (App. B.4; model not named)"},
        "steps_per_s_vs_paper": steps_per_s / PAPER_STEPS_PER_S,
    }
    log(f"[bench] paper dynamics: {steps_per_s:.0f} steps/s ({out['value'] / 1e6:.1f} M agent-steps/s, "
        f"{out['n_live_mean']:.0f} agents): 1e6 steps in {out['million_steps_s']:.0f} s against ~1200 s reported")
    return out


def lab_run(args) -> dict:
    """Lab environments (Sec. 2.2) as a batched workload of many tiny worlds."""
    import torch
    from paper_2302_09334_amd import lab, workloads, world
    base = workloads.WORKLOADS["net1k"]
    t0 = time.perf_counter()
    snap = lab.evolve(base, args.seed, args.lab_evolve_steps)
    genomes = lab.sample_agents(snap, args.lab_agents, seed=0)
    evolve_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    run = lab.LabRun(genomes, base, lab.conditions(), trials=args.lab_trials)
    setup_s = time.perf_counter() - t0
    steps = lab.STEPS
    run.step(100)   # graph capture outside the timed region
    run.sync()
    for w, img in zip(run.worlds, run.images):
        w.load(img)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run.step(steps)
    run.sync()
    wall = time.perf_counter() - t0
    ctrs = run.counters(steps)
    acting = sum(int(np.concatenate([[1], c["n_live"][:-1]]).sum()) for c in ctrs)
    g = lab.greediness_study(run, ctrs, len(genomes))
    pp = lab.peer_pressure_study(run, ctrs)
    # a sample of the same worlds stepped one at a time (plain path, graph launches)
    n_seq = min(args.lab_seq_sample, len(run.worlds))
    seq_wall = 0.0
    for i in range(n_seq):
        w = run.worlds[i]
        w.load(run.images[i])
        w.step(100)
        w.sync()
        w.load(run.images[i])
        t1 = time.perf_counter()
        for _ in range(steps // 100):
            w.step(100)
        w.sync()
        seq_wall += time.perf_counter() - t1
    seq_rate = n_seq * steps / seq_wall
    n_worlds = len(run.worlds)
    run.close()
    out = {
        "workload": f"{len(genomes)} agents sampled from net1k after {args.lab_evolve_steps} steps (seed {args.seed}); "
                    f"40x40 lab worlds without regrowth, densities {lab.DENSITIES} without reproduction and the "
                    f"high density with reproduction (T_repr {lab.T_REPR_LAB}); {args.lab_trials} trials each; "
                    f"{steps} steps",
        "worlds": n_worlds, "steps": steps, "wall_s": wall,
        "world_steps_per_s": n_worlds * steps / wall, "agent_steps_per_s": acting / wall,
        "sequential_sample": {"worlds": n_seq, "world_steps_per_s": seq_rate},
        "speedup_vs_sequential": (n_worlds * steps / wall) / seq_rate,
        "evolve_s": evolve_s, "setup_s": setup_s,
        "greediness": {"G_mean_by_density": g["G_mean_by_density"], "sustainable_foragers": g["sustainable_foragers"],
                       "agents": len(genomes)},
        "peer_pressure": pp,
    }
    log(f"[bench] lab: {n_worlds} worlds x {steps} steps in {wall * 1e3:.1f} ms = {out['world_steps_per_s'] / 1e6:.2f} M "
        f"world-steps/s ({out['speedup_vs_sequential']:.0f}x one at a time); G {g['G_mean_by_density']}, "
        f"sustainable {g['sustainable_foragers']}/{len(genomes)}; E off {pp['E_mean_off']:.2f} on {pp['E_mean_on']:.2f}")
    return out


def copy_calibration(torch, world):
    """Three launches of the plain copy kernel over 1 GiB (the known-size
    reference for the memory counters)."""
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    s = torch.cuda.Stream()
    for _ in range(3):
        world.test_copy(src, dst, s)
    torch.cuda.synchronize()
    log("[bench] copy calibration: 3 x 1 GiB device copies done")


# Steps from the seed that prepare the headline fixture's state (the M1-4k
# workload: steps 0..999 are its warm-up, so that the population has turned
# over, with births and deaths every step) before --warmup and --steps.
FIXTURE_STEPS = 1000
# The committed GPU parity tests compare m1_4k with the oracle over steps
# 0..PARITY_STEPS_M1_4K - 1 in the timed launch configuration.
PARITY_STEPS_M1_4K = 2200


class OneWorld:
    """One world seen through the batch interface the autotuner drives."""

    def __init__(self, w):
        self.w = w

    def snapshots(self):
        return self.w.snapshot(hidden=True, theta=True)

    def load(self, s):
        self.w.load(s)

    def set_mode(self, m):
        self.w.set_mode(m)

    def set_tuning(self, rows, waves, tile):
        self.w.set_tuning(rows, waves, tile)

    def step(self, k):
        self.w.step(k)

    def sync(self):
        self.w.sync()


def headline_run(args) -> dict:
    """The headline: m1_4k prepared by its 1000 fixture steps, --warmup more
    untimed steps, then exactly --steps timed steps (graph launches of
    --chunk steps, or per-phase kernels, whichever the calibration picked)
    between two synchronisations; then the same steps again from the same
    state as per-phase kernels with dispatch-stamped events (kernel times);
    bytes from the window's own device counters."""
    import torch
    from paper_2302_09334_amd import workloads, world
    cfg = workloads.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    w = world.World(cfg, args.seed, stream=stream, mode="graph")
    P = w.n_params
    log(f"[bench] {args.workload}: H={cfg['H']} W={cfg['W']} cap={cfg['cap']} n_init={cfg['n_init']} "
        f"hidden={cfg['hidden']} P={P}")

    def run(nsteps, mode):
        w.set_mode(mode)
        done = 0
        while done < nsteps:
            k = min(args.chunk, nsteps - done)
            w.step(k)
            done += k

    run(args.fixture_steps, "graph")
    w.sync()
    prep = w.snapshot(hidden=True, theta=True)
    # pick the launch mode and shape (act rows per round trip, agents per act
    # block, regrowth tile edge; none changes any result) with the project's
    # autotuner: a coordinate descent, each trial 200 steps from the prepared
    # state
    from paper_2302_09334_amd import tune
    one = OneWorld(w)
    if args.shape:
        r_, wv_, tl_ = (int(x) for x in args.shape.split(","))
        sp = dict(modes=[args.mode if args.mode != "auto" else "graph"], rows=(r_,), waves=(wv_,), tiles=(tl_,))
    else:
        sp = dict(modes=["graph", "kernels"] if args.mode == "auto" else [args.mode])
    tuned = tune.autotune(one, trial_steps=200, ks=(args.chunk,), **sp)
    calib = {f"{t['mode']}/rows{t['act_rows']}/waves{t['act_waves']}/tile{t['regrow_tile']}": t["us_per_step"] / 1e3
             for t in tuned["trials"]}
    for k, v in calib.items():
        log(f"[bench] {k}: {v * 1e3:.1f} us/step")
    bt = tuned["best"]
    best, best_rows, best_waves, best_tile = bt["mode"], bt["act_rows"], bt["act_waves"], bt["regrow_tile"]
    w.set_tuning(best_rows, best_waves, best_tile)
    w.load(prep)
    run(args.warmup, "graph")
    w.sync()
    start = w.snapshot(hidden=True, theta=True)
    t_first = start["t"]
    log(f"[bench] fixture {args.fixture_steps} + warm-up {args.warmup} steps done: t={t_first} "
        f"n_live={start['n_live']}")

    # the timed region: exactly K steps from the warmed-up state
    run(min(args.chunk, args.steps), best)   # graph capture outside the timed region
    w.sync()
    w.load(start)
    w.set_mode(best)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range((args.steps + args.chunk - 1) // args.chunk + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        ev[0].record(stream)
        done = 0
        i = 0
        while done < args.steps:
            k = min(args.chunk, args.steps - done)
            w.step(k)
            done += k
            i += 1
            ev[i].record(stream)
    w.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    chunk_ms = np.array([ev[j].elapsed_time(ev[j + 1]) for j in range(i)])
    chunk_steps = np.array([min(args.chunk, args.steps - j * args.chunk) for j in range(i)])
    per_step_ms = chunk_ms / chunk_steps
    prev = w.counters(t_first - 1, 1) if t_first > 0 else None
    ctr = w.counters(t_first, args.steps)
    n0 = int(prev["n_live"][0]) if prev is not None else int(start["n_live"])
    acting = np.concatenate([[n0], ctr["n_live"][:-1]])
    births_prev = np.concatenate([[int(prev["births"][0]) if prev is not None else 0], ctr["births"][:-1]])
    agent_steps = int(acting.sum())
    end = w.snapshot(hidden=True, theta=True)
    deaths = int(ctr["deaths"].sum())
    win0 = (t_first + 49) // 50
    win1 = (t_first + args.steps) // 50
    mh = w.move_hist(win1 - 1, 1)[0] if win1 > win0 else None
    metrics = {
        "life_expectancy": float(ctr["dead_age"].sum()) / deaths if deaths else None,
        "resources_mean": float(ctr["resources"].mean()),
        "population_mean": float(ctr["n_live"].mean()),
        "movement_window": None if mh is None else {
            "window": int(win1 - 1), "counted": int(mh[-1]),
            "percent_by_bin": [round(100.0 * float(x) / max(int(mh[-1]), 1), 2) for x in mh[:-1]]},
    }
    log(f"[bench] timed steps {t_first}..{t_first + args.steps - 1} in {wall * 1e3:.2f} ms ({best}); agent-steps "
        f"{agent_steps}; N_live mean {acting.mean():.1f} min {acting.min()} max {acting.max()}; births "
        f"{int(ctr['births'].sum())} deaths {deaths}")

    # nnz(x), the binary inputs that are 1, of every timed step (GRU worlds
    # with the benchmark's rules): the same steps once more, one launch each,
    # recounted on the host from each step's starting state.  The rows the act
    # kernel reads and the acting agents, recounted from the same states, must
    # equal the device counters at every step, else the recount is not reported.
    recount_ok, nnz_host = False, None
    if not cfg.get("controller", 0) and not cfg.get("dynamics", 0):
        w.load(start)
        w.set_mode("kernels")
        nnz_host = np.zeros(args.steps, np.float64)
        rows_host = np.zeros(args.steps, np.int64)
        live_host = np.zeros(args.steps, np.int64)
        for j in range(args.steps):
            s = w.snapshot()
            on, rd = observed_inputs(s, cfg)
            nnz_host[j], rows_host[j], live_host[j] = float(on.sum()), int(rd.sum()), s["n_live"]
            w.step(1)
        w.sync()
        recount_ok = bool(np.array_equal(rows_host, np.asarray(ctr["rows_read"], np.int64))
                          and np.array_equal(live_host, np.asarray(acting, np.int64)))
        log(f"[bench] host recount of the timed steps' inputs: nnz per agent {nnz_host.sum() / agent_steps:.2f}, "
            f"rows per agent {rows_host.sum() / agent_steps:.2f}; equal to the device counters: {recount_ok}")

    # the same steps again from the same state as per-phase kernels, each
    # launch between events its own dispatch stamps (kernel execution time)
    w.load(start)
    ph_ms = w.phase_times(args.steps)
    again = w.snapshot(hidden=True, theta=True)
    same_state = all(np.array_equal(end[k], again[k]) for k in ("uid", "row", "col", "energy", "age", "streak", "R"))
    kms = {"act": float(ph_ms[0]), "move": float(ph_ms[1]), "claim": float(ph_ms[2])}
    rows_read = ctr["rows_read"]
    kbytes = kernel_window_bytes(cfg, P, acting, rows_read, births_prev, ctr["deaths"], ctr["claim_wins"])
    step_b = step_algorithmic_bytes(cfg, P, acting, rows_read, ctr["births"])
    step_b_nnz = step_algorithmic_bytes(cfg, P, acting, nnz_host, ctr["births"]) if recount_ok else None
    kbytes_nnz = (kernel_window_bytes(cfg, P, acting, nnz_host, births_prev, ctr["deaths"], ctr["claim_wins"])
                  if recount_ok else None)
    dominant = max(kms, key=kms.get)
    achieved = kbytes[dominant] / (kms[dominant] * 1e-3) / 1e9
    step_gbps = float(step_b.sum()) / wall / 1e9
    src_hash = kernel_source_hash()
    per_agent_traffic = (read_traffic_per_agent(src_hash, f"{best_rows}_{best_waves}") if dominant == "act"
                         else None)
    n_act = float(acting.mean())
    traffic = per_agent_traffic * n_act if per_agent_traffic is not None else None
    # the plain path's per-step latency distribution: 200 steps from the same
    # state as single-step launches of the chosen mode, an event after each
    w.load(start)
    w.set_mode(best)
    w.step(1)   # graph capture outside the measured launches
    w.sync()
    w.load(start)
    sev = [torch.cuda.Event(enable_timing=True) for _ in range(201)]
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        sev[0].record(stream)
        for j in range(200):
            w.step(1)
            sev[j + 1].record(stream)
    w.sync()
    torch.cuda.synchronize()
    single_ms = np.array([sev[j].elapsed_time(sev[j + 1]) for j in range(200)])
    w.close()
    log(f"[bench] kernel us act {kms['act'] * 1e3:.2f} move {kms['move'] * 1e3:.2f} claim {kms['claim'] * 1e3:.2f}; "
        f"rows read per agent {float(rows_read.sum()) / agent_steps:.2f}; MB act {kbytes['act'] / 1e6:.2f} move "
        f"{kbytes['move'] / 1e6:.2f} claim {kbytes['claim'] / 1e6:.2f}; step {float(step_b.mean()) / 1e6:.1f} MB at "
        f"{step_gbps:.0f} GB/s; dominant {dominant}")
    return {
        "value": agent_steps / wall, "wall": wall, "ms_per_step": wall / args.steps * 1e3,
        "config": {
            "workload": f"{args.workload}: {cfg['H']}x{cfg['W']} grid, cap {cfg['cap']}, {cfg['n_init']} initial "
                        f"agents, resources Bernoulli({cfg['res_init_p']}), regrowth x{cfg['rate_scale']}, "
                        f"obs {2 * cfg['obs_radius'] + 1}x{2 * cfg['obs_radius'] + 1}x2+1, GRU {cfg['hidden']}, "
                        f"seed {args.seed}; timed steps {t_first}..{t_first + args.steps - 1} after "
                        f"{args.fixture_steps} fixture steps and {args.warmup} warm-up steps",
            "launch_mode": best,
            "act_rows_per_round_trip": best_rows,
            "act_agents_per_block": best_waves,
            "regrow_tile_edge": best_tile,
            "steps_per_launch": args.chunk,
            "first_timed_step": t_first,
            "n_live_mean": n_act,
            "n_live_min": int(acting.min()),
            "n_live_max": int(acting.max()),
            "births": int(ctr["births"].sum()),
            "deaths": deaths,
            "oracle_parity_tested_steps": f"0..{PARITY_STEPS_M1_4K - 1}"
                                          + ("" if t_first + args.steps <= PARITY_STEPS_M1_4K
                                             else " (this window goes beyond them)"),
            "parallelism": "single GPU",
        },
        "latency_ms_per_step": {"p50": float(np.percentile(per_step_ms, 50)),
                                "p99": float(np.percentile(per_step_ms, 99)),
                                "samples": int(len(per_step_ms)),
                                "window": f"per {args.chunk}-step launch of the timed steps",
                                "single_step_launches": {
                                    "p50": float(np.percentile(single_ms, 50)),
                                    "p99": float(np.percentile(single_ms, 99)), "samples": 200,
                                    "window": f"steps {t_first}..{t_first + 199} again, one launch per step "
                                              f"({best})"}},
        "calibration_us_per_step": {m: v * 1e3 for m, v in calib.items()},
        "kernels": {k: {"ms_per_launch": kms[k], "algorithmic_bytes": kbytes[k],
                        "GBps": kbytes[k] / (kms[k] * 1e-3) / 1e9} for k in kms},
        "roofline": {
            "kernel": {"act": "k_act (observation + sparse input rows + GRU + head, one wave per agent)",
                       "move": "k_move (moves, energy, death, survivor scan; half of the recurrent projection)",
                       "claim": "k_claim (birth claims, birth scan, regrowth; the other half of the recurrent projection)"}[dominant],
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_basis": None if traffic is None else
                "rocprofv3 FETCH_SIZE + WRITE_SIZE of this kernel per acting agent on the same bench window "
                "(profiles/act_m1_4k_traffic.txt), times this window's mean acting agents",
            "algorithmic_bytes_per_launch": kbytes[dominant],
            "launch_ms": kms[dominant],
            "kernel_pass_same_steps": same_state,
            "agents_per_launch": n_act,
            "act_input_rows_read_per_agent": float(rows_read.sum()) / agent_steps,
            "step_algorithmic_bytes": float(step_b.mean()),
            "step_achieved_GBps": step_gbps,
            "step_frac": step_gbps / HBM_PEAK_GBS,
            "step_bytes_formula": "per acting agent 4*(3hd*hd + 6hd + 5hd + 5) + 8hd + 40 + 12hd (energy row); "
                                  "+ 12hd per input row read (device counter); + 8P per birth; + 10 H W",
            "frac_nnz": (kbytes_nnz[dominant] / (kms[dominant] * 1e-3) / 1e9 / HBM_PEAK_GBS
                         if recount_ok else None),
            "nnz_inputs_per_agent": float(nnz_host.sum()) / agent_steps if recount_ok else None,
            "step_algorithmic_bytes_nnz": float(step_b_nnz.mean()) if recount_ok else None,
            "step_frac_nnz": float(step_b_nnz.sum()) / wall / 1e9 / HBM_PEAK_GBS if recount_ok else None,
            "step_nnz_basis": "frac_nnz and step_frac_nnz: the same kernel and step bytes with the input term "
                              "counted as nnz(x) rows of 12hd bytes (the binary inputs that are 1, recounted on the "
                              "host from every timed step's starting state; the rows read and the acting agents "
                              "recounted from the same states equal the device counters at every step); the act "
                              "kernel reads fewer rows than nnz (a window with more ones than zeros is read as its "
                              "column total and the rows of its zeros), so frac and step_frac, counting the rows "
                              "read, are the figures of the bytes moved (frac_nnz exceeds the measured traffic)",
            "kernel_source_sha256_16": src_hash,
        },
        "ecology_metrics": metrics,
        "_cfg": cfg,
        "_start_t": t_first,
    }


def m0_run(args) -> dict:
    """M0: the 32 x 64 world (cfg0) for its 1000 steps from the seed: one
    launch per step (per-phase kernels, the launch-bound latency of a tiny
    world) with an event per step, then the same 1000 steps as graphs of 100;
    the oracle's rate on the same steps beside it."""
    import torch
    from paper_2302_09334_amd import batch, workloads, world
    cfg = workloads.WORKLOADS["cfg0"]
    steps = workloads.STEPS["cfg0"]
    out = {"workload": "cfg0: 32x64 grid, cap 256, 32 initial agents, Bernoulli(0.1), obs 5x5x2+1, GRU 16, "
                       f"seed {args.seed}, steps 0..{steps - 1}"}
    for mode, K in (("kernels", 1), ("graph", 100)):
        w = world.World(cfg, args.seed, mode=mode)
        s0 = w.snapshot(hidden=True, theta=True)
        w.step(K)    # graph capture / first launch, outside the timed region
        w.sync()
        w.load(s0)
        wall, ms = batch.time_chunks(w.step, steps, K, w.stream)
        c = w.counters(0, steps)
        acting = int(cfg["n_init"]) + int(c["n_live"][:-1].sum())
        out[f"{mode}_K{K}"] = {"steps_per_s": steps / wall, "agent_steps_per_s": acting / wall,
                               "step_ms_p50": float(np.percentile(ms / K, 50)),
                               "step_ms_p99": float(np.percentile(ms / K, 99))}
        out["n_live_mean"] = float(np.concatenate([[cfg["n_init"]], c["n_live"][:-1]]).mean())
        w.close()
    import oracle
    ow = oracle.OracleWorld(oracle.OracleConfig.from_dict(cfg), args.seed)
    t0 = time.perf_counter()
    acted = 0
    for _ in range(steps):
        acted += ow.n_live
        ow.step()
    el = time.perf_counter() - t0
    ow.close()
    out["oracle"] = {"steps_per_s": steps / el, "agent_steps_per_s": acted / el, "cores": 1}
    out["gpu_vs_oracle_steps"] = out["graph_K100"]["steps_per_s"] / out["oracle"]["steps_per_s"]
    log(f"[bench] M0 cfg0: {out['kernels_K1']['steps_per_s']:.0f} steps/s one launch per step (p50 "
        f"{out['kernels_K1']['step_ms_p50'] * 1e3:.1f} us), {out['graph_K100']['steps_per_s']:.0f} steps/s in graphs; "
        f"oracle {out['oracle']['steps_per_s']:.0f} steps/s")
    return out


def m1_run(args) -> dict:
    """M1: the paper-scale world (cfg1: 200 x 400, 8192 slots, 1000 initial
    agents, Bernoulli(0.05)) for its 10,000 steps from the seed as 100
    graphs of 100 steps, with the mean live population."""
    import torch
    from paper_2302_09334_amd import batch, workloads, world
    cfg = workloads.WORKLOADS["cfg1"]
    steps = workloads.STEPS["cfg1"]
    w2 = world.World(cfg, args.seed, mode="graph")
    s0 = w2.snapshot(hidden=True, theta=True)
    w2.step(100)    # graph capture, outside the timed region
    w2.sync()
    w2.load(s0)
    # two timed halves (the counter ring holds 8192 steps: each half's
    # counters are read between them, outside the timed regions)
    wall = 0.0
    ms_all, n_live = [], []
    for h0 in range(0, steps, steps // 2):
        wh, ms = batch.time_chunks(w2.step, steps // 2, 100, w2.stream)
        wall += wh
        ms_all.append(ms)
        n_live.append(w2.counters(h0, steps // 2)["n_live"])
    ms = np.concatenate(ms_all)
    n_live = np.concatenate(n_live)
    acting = np.concatenate([[cfg["n_init"]], n_live[:-1]])
    w2.close()
    out = {"workload": "cfg1: 200x400 grid, cap 8192, 1000 initial agents, Bernoulli(0.05), obs 7x7x2+1, GRU 32, "
                       f"seed {args.seed}, steps 0..{steps - 1} as {steps // 100} graphs of 100 steps (timed in "
                       "two halves; the counters are read between them)",
           "agent_steps_per_s": float(acting.sum()) / wall, "steps_per_s": steps / wall,
           "ms_per_step": wall / steps * 1e3, "n_live_mean": float(acting.mean()), "n_live_min": int(acting.min()),
           "n_live_max": int(acting.max()), "step_ms_p50": float(np.percentile(ms / 100, 50)),
           "step_ms_p99": float(np.percentile(ms / 100, 99))}
    log(f"[bench] M1 cfg1: {out['agent_steps_per_s'] / 1e6:.1f} M agent-steps/s, {out['steps_per_s']:.0f} steps/s, "
        f"mean N_live {out['n_live_mean']:.0f}")
    return out


def m2_run(args) -> dict:
    """M2: the dense-population stress world (cfg2) for its 5000 steps from
    the seed as graphs of 100 steps."""
    from paper_2302_09334_amd import batch, workloads, world
    cfg = workloads.WORKLOADS["cfg2"]
    steps = workloads.STEPS["cfg2"]
    w2 = world.World(cfg, args.seed, mode="graph")
    s0 = w2.snapshot(hidden=True, theta=True)
    w2.step(100)    # graph capture, outside the timed region
    w2.sync()
    w2.load(s0)
    wall, ms = batch.time_chunks(w2.step, steps, 100, w2.stream)
    c = w2.counters(0, steps)
    acting = np.concatenate([[cfg["n_init"]], c["n_live"][:-1]])
    w2.close()
    out = {"workload": "cfg2: 200x400 grid, cap 16384, 12000 initial agents, Bernoulli(0.3), regrowth x5, obs "
                       f"7x7x2+1, GRU 32, seed {args.seed}, steps 0..{steps - 1} as graphs of 100 steps",
           "agent_steps_per_s": float(acting.sum()) / wall, "steps_per_s": steps / wall,
           "ms_per_step": wall / steps * 1e3, "n_live_mean": float(acting.mean()), "n_live_min": int(acting.min()),
           "n_live_max": int(acting.max()), "births": int(c["births"].sum()), "deaths": int(c["deaths"].sum()),
           "step_ms_p50": float(np.percentile(ms / 100, 50)), "step_ms_p99": float(np.percentile(ms / 100, 99))}
    log(f"[bench] M2 cfg2 5000 steps: {out['agent_steps_per_s'] / 1e6:.1f} M agent-steps/s, mean N_live "
        f"{out['n_live_mean']:.0f}, births {out['births']}, deaths {out['deaths']}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--fixture-steps", type=int, default=FIXTURE_STEPS,
                    help="steps from the seed that prepare the workload before --warmup (the M1-4k fixture: 1000)")
    ap.add_argument("--workload", default="m1_4k")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", default="auto", choices=["auto", "kernels", "graph"])
    ap.add_argument("--chunk", type=int, default=100, help="steps per world_step call")
    ap.add_argument("--shape", default="",
                    help="rows,waves,tile: fix the launch shape of the headline (default: autotuned)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run the plain copy kernel on 1 GiB (memory-counter calibration)")
    ap.add_argument("--m2-steps", type=int, default=60, help="steps of the cache-exceeding cfg2 run (0 = skip)")
    ap.add_argument("--fixtures", type=int, default=1, help="run the M0, M1 and M2 fixtures (0 = skip)")
    ap.add_argument("--batch-worlds", type=int, default=64, help="uneven worlds of the batched run (0 = skip)")
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--batch-warmup", type=int, default=0)
    ap.add_argument("--serve-seconds", type=float, default=20.0, help="arrival window of the served run (0 = skip)")
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--net-steps", type=int, default=500, help="timed steps of the paper-network world (0 = skip)")
    ap.add_argument("--net-warmup", type=int, default=300)
    ap.add_argument("--net-phase-steps", type=int, default=100)
    ap.add_argument("--only", choices=["net", "paper", "lab", "m2", "headline", "served", "batched", "fixtures"],
                    help="run only this leg and print it")
    ap.add_argument("--paper-steps", type=int, default=2000, help="timed steps of the paper-dynamics world (0 = skip)")
    ap.add_argument("--paper-warmup", type=int, default=1000)
    ap.add_argument("--lab-agents", type=int, default=50, help="evolved agents of the lab leg (0 = skip)")
    ap.add_argument("--lab-trials", type=int, default=10)
    ap.add_argument("--lab-evolve-steps", type=int, default=20000)
    ap.add_argument("--lab-seq-sample", type=int, default=20)
    args = ap.parse_args()

    world_size = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world_size != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.steps < 1 or args.steps > 8000:
        sys.exit("--steps must be in 1..8000 (the per-step counter ring holds 8192 steps)")

    import torch
    from paper_2302_09334_amd import world

    if args.only and args.only != "headline":
        leg = {"net": ("paper_network", net_run), "paper": ("paper_dynamics", paper_run), "lab": ("lab", lab_run),
               "m2": ("cache_exceeding", lambda a: hbm_honest_run(a, ONLY_M2_ROWS)),
               "served": ("served", served_run), "batched": ("batched", batched_run),
               "fixtures": ("fixtures", lambda a: {"M0": m0_run(a), "M1": m1_run(a), "M2": m2_run(a)})}
        name, fn = leg[args.only]
        out = fn(args)
        if args.calib_copy:
            copy_calibration(torch, world)
        print(json.dumps({name: out}))
        return

    head = headline_run(args)
    cfg = head.pop("_cfg")
    head.pop("_start_t")
    if args.calib_copy:
        copy_calibration(torch, world)
    if args.only == "headline":
        print(json.dumps({"headline": head}))
        return

    net = net_run(args) if args.net_steps > 0 else None
    paper = paper_run(args) if args.paper_steps > 0 else None
    labs = lab_run(args) if args.lab_agents > 0 else None
    m2 = hbm_honest_run(args, head["config"]["act_rows_per_round_trip"]) if args.m2_steps > 0 else None
    fixtures = None
    if args.fixtures:
        fixtures = {"M0": m0_run(args), "M1": m1_run(args), "M2": m2_run(args)}
    batched = batched_run(args) if args.batch_worlds > 0 else None
    served = served_run(args) if args.serve_seconds > 0 else None
    cpu = None
    if not args.no_cpu:
        log("[bench] oracle CPU baseline ...")
        cpu = cpu_baseline(cfg, args.seed, args.cpu_seconds)
        log(f"[bench] oracle: {cpu['value']:.0f} agent-steps/s")

    out = {
        "metric": "agent-steps/s @200x400, ~4k agents; batched/served p50/p99 step latency",
        "value": head["value"],
        "unit": "agent-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded counter-based generator: resources, placement, genomes)",
        "config": head["config"],
        "latency_ms_per_step": head["latency_ms_per_step"],
        "calibration_us_per_step": head["calibration_us_per_step"],
        "kernels": head["kernels"],
        "roofline": head["roofline"],
        "ecology_metrics": head["ecology_metrics"],
        "fixtures": fixtures,
        "paper_network": net,
        "paper_dynamics": paper,
        "lab": labs,
        "cache_exceeding": m2,
        "cpu_baseline": cpu,
        "batched": batched,
        "served": served,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
