"""Seeded synthetic workloads (world parameters only; no arithmetic of the method).

The paper (arXiv 2302.09334) runs one synthetic world: a grid with latitude-
dependent resource regrowth (App. B.1), randomly placed agents with random
initial genomes (App. B.2, B.4).  The workloads below keep that structure with
the sizes of the benchmark configurations:

* ``cfg0``      32 x 64 grid, 256 slots, 32 agents, 5x5x2+1 inputs, GRU 16.
* ``cfg1``      200 x 400 grid, 8192 slots, 1000 agents, 7x7x2+1, GRU 32.
* ``m1_4k``     200 x 400 grid, 4608 slots, 4096 agents, dense resources
                (Bernoulli 0.3) and regrowth x5 so the population stays near 4k.
* ``cfg2``      200 x 400 grid, 16384 slots, 12000 agents, Bernoulli 0.3, x5.
* ``batch64``   64 uneven worlds (grid sizes from a fixed set, caps 512..8192).
* ``net1k``     the paper's own scale with its network (App. B.4, B.5): a
                200 x 400 grid, at most 1000 agents (1024 slots), 330 placed
                at the start, 16,000 resources on average (Bernoulli 0.2),
                15 x 15 x 3 observation, CNN + LSTM(4).
* ``net_m1_4k`` the m1_4k world (about 4k agents) with the paper's network.
* ``paper1k``   the paper's own world (App. B.4): 200 x 400, at most 1000
                agents, 330 at the start, 16,000 resources on average, the
                paper's network and dynamics (stacking, walls, energy in units
                of 1/40 with E0 = E_max = 3, decay 0.025, +1 per resource,
                reproduction after 140 steps above 0, death after 200 steps
                below 0 or past age 650, regrowth 0.002 c(x) + 5e-5 with
                alpha = 200).

Every random choice of a workload (the uneven-world manifest, the serving
arrival trace) comes from ``numpy.random.default_rng`` with a fixed seed; the
simulation's own randomness comes from its counter-based generator.
"""
from __future__ import annotations

import numpy as np

BASE = dict(
    obs_radius=3, hidden=32, res_init_p=0.05, rate_bottom=0.02, rate_top=0.002,
    rate_scale=1.0, spont=1e-5, E0=50, decay=1, gain=10, E_repr=40, T_repr=20,
    L_max=2000, sigma_mut=0.02, w_init_gain=0.5,
)


def make(**over) -> dict:
    d = dict(BASE)
    d.update(over)
    return d


WORKLOADS = {
    "cfg0": make(H=32, W=64, cap=256, n_init=32, obs_radius=2, hidden=16, res_init_p=0.1),
    "cfg1": make(H=200, W=400, cap=8192, n_init=1000, res_init_p=0.05),
    "m1_4k": make(H=200, W=400, cap=4608, n_init=4096, res_init_p=0.3, rate_scale=5.0),
    "cfg2": make(H=200, W=400, cap=16384, n_init=12000, res_init_p=0.3, rate_scale=5.0),
    "net1k": make(H=200, W=400, cap=1024, n_init=330, res_init_p=0.2, obs_radius=7, hidden=4, controller=1),
    "net_m1_4k": make(H=200, W=400, cap=4608, n_init=4096, res_init_p=0.3, rate_scale=5.0, obs_radius=7, hidden=4,
                      controller=1),
    "paper1k": make(H=200, W=400, cap=1000, n_init=330, res_init_p=0.2, obs_radius=7, hidden=4, controller=1,
                    dynamics=1, E0=120, E_max=120, decay=1, gain=40, E_repr=0, T_repr=140, T_death=200, L_max=650,
                    sigma_mut=0.02, spont=5e-5, regrow_pI=0.002, regrow_alpha=200.0, rate_top=0.0, rate_bottom=0.0),
}

# Steps each workload is run for in the benchmark configurations.
STEPS = {"cfg0": 1000, "cfg1": 10000, "m1_4k": 2000, "cfg2": 5000, "net1k": 2000, "net_m1_4k": 2000, "paper1k": 5000}

GRID_SET = [(64, 128), (100, 200), (128, 256), (200, 400)]


def batch_manifest(n_worlds: int = 64, seed: int = 0) -> list[dict]:
    """Uneven worlds: grid uniform over GRID_SET, cap uniform over multiples of
    64 in [512, 8192], 10% initial agents, latitude rates scaled by U[0.5, 2]."""
    rng = np.random.default_rng(seed)
    out = []
    caps = np.arange(512, 8192 + 1, 64)
    for i in range(n_worlds):
        H, W = GRID_SET[int(rng.integers(len(GRID_SET)))]
        cap = int(caps[int(rng.integers(len(caps)))])
        scale = float(rng.uniform(0.5, 2.0))
        out.append(dict(cfg=make(H=H, W=W, cap=cap, n_init=max(1, cap // 10), rate_scale=scale),
                        seed=i))
    return out


def serve_trace(duration_s: float = 600.0, rate_hz: float = 20.0, seed: int = 0) -> list[dict]:
    """Poisson arrivals of simulation requests: grid from GRID_SET, cap as in
    the batch manifest, steps U[500, 5000], GRU hidden 16 or 32."""
    rng = np.random.default_rng(seed)
    caps = np.arange(512, 8192 + 1, 64)
    t = 0.0
    out = []
    i = 0
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s:
            break
        H, W = GRID_SET[int(rng.integers(len(GRID_SET)))]
        cap = int(caps[int(rng.integers(len(caps)))])
        hidden = 16 if rng.integers(2) == 0 else 32
        steps = int(rng.integers(500, 5001))
        out.append(dict(arrival=t, steps=steps, seed=1000 + i,
                        cfg=make(H=H, W=W, cap=cap, n_init=max(1, cap // 10), hidden=hidden)))
        i += 1
    return out
