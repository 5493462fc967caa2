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
# (the library's build default, ECO_PROJ_MOVE_EIGHTHS = 3); the rest, minus
# the agents that died in the move phase, runs in the claim kernel.
PROJ_MOVE_SHARE = 3 / 8


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
    acting = int(s0["n_live"]) + int(c["n_live"][:-1].sum())
    s1 = w.snapshot()
    w.close()
    w2 = world.World(cfg, args.seed, stream=stream, mode="kernels")
    w2.set_tuning(rows)
    ph = w2.phase_times(steps)
    w2.close()
    rows_read = float(np.concatenate([observed_inputs(s, cfg)[1] for s in (s0, s1)]).mean())
    n = acting / steps
    act_b = n * act_bytes_per_agent(cfg, rows_read) + cfg["H"] * cfg["W"] * 5
    pb = proj_bytes_per_agent(cfg)
    move_b = n * (MOVE_BYTES_PER_AGENT + PROJ_MOVE_SHARE * pb)
    claim_b = ((1 - PROJ_MOVE_SHARE) * (n - float(c["deaths"].mean())) * pb + n * CLAIM_BYTES_PER_AGENT
               + 2 * cfg["H"] * cfg["W"])
    out = {"workload": "cfg2: 200x400 grid, cap 16384, 12000 initial agents, resources Bernoulli(0.3), "
                       "regrowth x5.0, obs 7x7x2+1, GRU 32, seed %d, steps 0..%d" % (args.seed, steps - 1),
           "steps": steps, "agent_steps_per_s": acting / wall, "ms_per_step": wall / steps * 1e3,
           "n_live_mean": n, "births_mean": float(c["births"].mean()),
           "kernel_ms": {"act": float(ph[0]), "move": float(ph[1]), "claim": float(ph[2])},
           "act_GBps": act_b / (float(ph[0]) * 1e-3) / 1e9, "move_GBps": move_b / (float(ph[1]) * 1e-3) / 1e9,
           "claim_GBps": claim_b / (float(ph[2]) * 1e-3) / 1e9,
           "act_algorithmic_MB_per_launch": act_b / 1e6, "step_algorithmic_MB": (act_b + move_b + claim_b) / 1e6}
    log(f"[bench] cfg2 (cache-exceeding, {n:.0f} agents): {out['agent_steps_per_s'] / 1e6:.1f} M agent-steps/s, "
        f"{out['ms_per_step'] * 1e3:.1f} us/step, act {out['act_GBps']:.0f} GB/s, move {out['move_GBps']:.0f} GB/s, "
        f"claim {out['claim_GBps']:.0f} GB/s")
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
    b.step(args.batch_warmup)
    b.sync()
    tuned = tune.autotune(b, trial_steps=100)
    best = tuned["best"]
    log(f"[bench] batched autotune: {best}")
    K = best["K"]
    wall, chunk_ms = batch.time_chunks(b.step, args.batch_steps, K, b.stream)
    b.sync()
    agent_steps = b.acting_agents(args.batch_warmup, args.batch_steps)
    n_agents = sum(w.snapshot()["n_live"] for w in b.worlds)
    b.close()
    seq = batch.run_sequential(entries, args.batch_warmup, args.batch_steps, 100, mode="graph")
    out = {"worlds": len(entries), "steps": args.batch_steps, "warmup": args.batch_warmup,
           "agent_steps_per_s": agent_steps / wall, "ms_per_step": wall / args.batch_steps * 1e3,
           "step_ms_p50": float(np.percentile(chunk_ms / K, 50)), "step_ms_p99": float(np.percentile(chunk_ms / K, 99)),
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
    results, m = srv.run(reqs, duration=args.serve_seconds, realtime=True)
    m["arrival_window_s"] = args.serve_seconds
    m["rate_hz"] = 20.0
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


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--workload", default="m1_4k")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", default="auto", choices=["auto", "kernels", "graph"])
    ap.add_argument("--chunk", type=int, default=100, help="steps per world_step call")
    ap.add_argument("--phase-steps", type=int, default=200, help="steps of the per-phase event pass")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run the plain copy kernel on 1 GiB (memory-counter calibration)")
    ap.add_argument("--m2-steps", type=int, default=60, help="steps of the cache-exceeding cfg2 run (0 = skip)")
    ap.add_argument("--batch-worlds", type=int, default=64, help="uneven worlds of the batched run (0 = skip)")
    ap.add_argument("--batch-steps", type=int, default=400)
    ap.add_argument("--batch-warmup", type=int, default=100)
    ap.add_argument("--serve-seconds", type=float, default=20.0, help="arrival window of the served run (0 = skip)")
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--net-steps", type=int, default=500, help="timed steps of the paper-network world (0 = skip)")
    ap.add_argument("--net-warmup", type=int, default=300)
    ap.add_argument("--net-phase-steps", type=int, default=100)
    ap.add_argument("--only", choices=["net", "paper", "lab", "m2"], help="run only this leg and print it")
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
    from paper_2302_09334_amd import workloads, world

    if args.only:
        leg = {"net": ("paper_network", net_run), "paper": ("paper_dynamics", paper_run), "lab": ("lab", lab_run),
               "m2": ("cache_exceeding", lambda a: hbm_honest_run(a, ONLY_M2_ROWS))}
        name, fn = leg[args.only]
        out = fn(args)
        if args.calib_copy:
            copy_calibration(torch, world)
        print(json.dumps({name: out}))
        return

    cfg = workloads.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    w = world.World(cfg, args.seed, stream=stream, mode="graph")
    log(f"[bench] {args.workload}: H={cfg['H']} W={cfg['W']} cap={cfg['cap']} n_init={cfg['n_init']} "
        f"hidden={cfg['hidden']} P={w.n_params}")

    def run(nsteps, mode):
        w.set_mode(mode)
        done = 0
        while done < nsteps:
            k = min(args.chunk, nsteps - done)
            w.step(k)
            done += k

    # warm-up (graph mode; every mode reaches the same state)
    run(args.warmup, "graph")
    w.sync()
    start = w.snapshot(hidden=True, theta=True)
    log(f"[bench] warm-up done: t={start['t']} n_live={start['n_live']}")

    # pick the launch mode and the act kernel's rows per round trip (both
    # leave every result unchanged) on a short calibration from the same state
    modes = ["graph", "kernels"] if args.mode == "auto" else [args.mode]
    calib = {}
    for m in modes:
        for rows in (8, 16, 32):
            w.set_tuning(rows)
            w.load(start)
            run(min(args.chunk, args.steps), m)   # capture / first launch
            w.sync()
            w.load(start)
            n_cal = min(2 * args.chunk, args.steps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run(n_cal, m)
            w.sync()
            calib[f"{m}/rows{rows}"] = (time.perf_counter() - t0) / n_cal * 1e3
            log(f"[bench] {m} rows {rows}: {calib[f'{m}/rows{rows}'] * 1e3:.1f} us/step")
    best_key = min(calib, key=calib.get)
    best, best_rows = best_key.split("/rows")[0], int(best_key.split("/rows")[1])
    w.set_tuning(best_rows)

    # the timed region: exactly K steps from the warmed-up state
    w.load(start)
    run(min(args.chunk, args.steps), best)
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
    t_first = start["t"]
    ctr_prev = w.counters(t_first - 1, 1)["n_live"][0] if t_first > 0 else start["n_live"]
    ctr = w.counters(t_first, args.steps)
    acting = np.concatenate([[ctr_prev], ctr["n_live"][:-1]])
    agent_steps = int(acting.sum())
    value = agent_steps / wall
    end = w.snapshot()
    # ecology metrics of App. C over the timed steps (computed inside them)
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
    log(f"[bench] timed {args.steps} steps in {wall * 1e3:.2f} ms ({best}); agent-steps {agent_steps}; "
        f"N_live mean {acting.mean():.1f} min {acting.min()} max {acting.max()}; births {int(ctr['births'].sum())} "
        f"deaths {int(ctr['deaths'].sum())}")

    # roofline of the dominant kernel: act phase in per-phase mode with events
    w.load(start)
    nnz0, rows0 = observed_inputs(start, cfg)
    ph_ms = w.phase_times(args.phase_steps)
    mid = w.snapshot()
    nnz1, rows1 = observed_inputs(mid, cfg)
    nnz_mean = float(np.concatenate([nnz0, nnz1]).mean())
    rows_mean = float(np.concatenate([rows0, rows1]).mean())
    pc = w.counters(t_first, args.phase_steps)
    n_act = float(np.concatenate([[start["n_live"]], pc["n_live"][:-1]]).mean())
    per_agent = act_bytes_per_agent(cfg, rows_mean)
    grid_bytes = cfg["H"] * cfg["W"] * 5
    elig = float(np.mean([(s["streak"] >= cfg["T_repr"]).sum() for s in (start, mid)]))
    kbytes = {
        "act": n_act * per_agent + grid_bytes,
        "move": n_act * (MOVE_BYTES_PER_AGENT + PROJ_MOVE_SHARE * proj_bytes_per_agent(cfg)),
        "claim": (1 - PROJ_MOVE_SHARE) * (n_act - float(pc["deaths"].mean())) * proj_bytes_per_agent(cfg)
                 + n_act * CLAIM_BYTES_PER_AGENT + elig * CLAIM_BYTES_PER_ELIGIBLE + 2 * cfg["H"] * cfg["W"],
    }
    kms = {"act": float(ph_ms[0]), "move": float(ph_ms[1]), "claim": float(ph_ms[2])}
    dominant = max(kms, key=kms.get)
    act_bytes = kbytes["act"]
    step_bytes = sum(kbytes.values())
    achieved = kbytes[dominant] / (kms[dominant] * 1e-3) / 1e9
    src_hash = kernel_source_hash()
    traffic = read_traffic(src_hash, best_rows) if dominant == "act" else None
    dense_per_agent = 4 * w.n_params + 2 * cfg["hidden"] * 4 + 21
    log(f"[bench] kernel us act {kms['act'] * 1e3:.2f} move {kms['move'] * 1e3:.2f} claim {kms['claim'] * 1e3:.2f}; "
        f"nnz mean {nnz_mean:.2f} rows read {rows_mean:.2f}; MB act {kbytes['act'] / 1e6:.2f} move {kbytes['move'] / 1e6:.2f} "
        f"claim {kbytes['claim'] / 1e6:.2f}; dominant {dominant}")

    if args.calib_copy:
        copy_calibration(torch, world)

    net = None
    if args.net_steps > 0:
        net = net_run(args)
    paper = None
    if args.paper_steps > 0:
        paper = paper_run(args)
    labs = None
    if args.lab_agents > 0:
        labs = lab_run(args)

    m2 = None
    if args.m2_steps > 0:
        m2 = hbm_honest_run(args, best_rows)

    batched = None
    if args.batch_worlds > 0:
        batched = batched_run(args)
    served = None
    if args.serve_seconds > 0:
        served = served_run(args)

    cpu = None
    if not args.no_cpu:
        log("[bench] oracle CPU baseline ...")
        cpu = cpu_baseline(cfg, args.seed, args.cpu_seconds)
        log(f"[bench] oracle: {cpu['value']:.0f} agent-steps/s")

    # every weight read once per acting agent, h in and out, ~20 B of scalars in
    # and out, parent genome in and child genome out per birth, grid as u8 +
    # i32 in and out: what a step would move with no input skipped
    P = w.n_params
    dense_step = (acting.mean() * (4 * P + 8 * cfg["hidden"] + 40) + ctr["births"].mean() * 8 * P
                  + cfg["H"] * cfg["W"] * (2 * 1 + 2 * 4))
    ms_per_step = wall / args.steps * 1e3
    out = {
        "metric": "agent-steps/s @200x400, ~4k agents; batched/served p50/p99 step latency",
        "value": value,
        "unit": "agent-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded counter-based generator: resources, placement, genomes)",
        "config": {
            "workload": f"{args.workload}: {cfg['H']}x{cfg['W']} grid, cap {cfg['cap']}, {cfg['n_init']} initial "
                        f"agents, resources Bernoulli({cfg['res_init_p']}), regrowth x{cfg['rate_scale']}, "
                        f"obs {2 * cfg['obs_radius'] + 1}x{2 * cfg['obs_radius'] + 1}x2+1, GRU {cfg['hidden']}, "
                        f"seed {args.seed}",
            "launch_mode": best,
            "act_rows_per_round_trip": best_rows,
            "steps_per_launch": args.chunk,
            "n_live_mean": float(acting.mean()),
            "n_live_min": int(acting.min()),
            "n_live_max": int(acting.max()),
            "births": int(ctr["births"].sum()),
            "deaths": int(ctr["deaths"].sum()),
            "parallelism": "single GPU",
        },
        "latency_ms_per_step": {"p50": float(np.percentile(per_step_ms, 50)),
                                "p99": float(np.percentile(per_step_ms, 99)),
                                "window": f"per {args.chunk}-step launch"},
        "calibration_us_per_step": {m: v * 1e3 for m, v in calib.items()},
        "kernels": {k: {"ms_per_launch": kms[k], "algorithmic_bytes": kbytes[k],
                        "GBps": kbytes[k] / (kms[k] * 1e-3) / 1e9} for k in kms},
        "roofline": {
            "kernel": {"act": "k_act (observation + sparse input rows + GRU + head, one wave per agent)",
                       "move": "k_move (moves, energy, death, survivor scan; 3/8 of the recurrent projection)",
                       "claim": "k_claim (birth claims, birth scan, regrowth; 5/8 of the recurrent projection)"}[dominant],
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": kbytes[dominant],
            "launch_ms": kms[dominant],
            "act_per_agent_bytes": per_agent,
            "agents_per_launch": n_act,
            "nnz_binary_inputs_mean": nnz_mean,
            "act_input_rows_read_mean": rows_mean,
            "act_dense_equivalent_bytes_per_launch": n_act * dense_per_agent + grid_bytes,
            "step_algorithmic_bytes": step_bytes,
            "step_achieved_GBps": step_bytes / (wall / args.steps) / 1e9,
            "step_dense_equivalent_bytes": dense_step,
            "step_dense_equivalent_GBps": dense_step / (wall / args.steps) / 1e9,
            "kernel_source_sha256_16": src_hash,
        },
        "ecology_metrics": metrics,
        "paper_network": net,
        "paper_dynamics": paper,
        "lab": labs,
        "cache_exceeding": m2,
        "cpu_baseline": cpu,
        "batched": batched,
        "served": served,
    }
    w.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
