"""Autotuner for batched launches.

Only knobs that cannot change any result are searched: the launch mode
(per-phase kernels or a captured graph), the number of steps per launch, the
act kernel's input rows per round trip, its agents per block, and the edge of
the regrowth tiles (each is shown result-invariant by the batched-equals-alone
tests).  The search is a coordinate descent: starting from the library's
defaults, each knob in turn is set to its fastest value with the others held
(if that gains more than 1%), and the sweep repeats until a full pass changes nothing (at most `rounds`
passes).  Every trial runs the same number of steps from the same saved state
(after one untimed launch that captures its graph), and the state is restored
exactly afterwards, so tuning leaves the simulation where it was.
"""
from __future__ import annotations

import time

MODES = ("graph", "kernels")
KS = (25, 50, 100)
ROWS = (8, 16, 32)
WAVES = (2, 4, 8)
TILES = (8, 16, 32)
DEFAULT = {"mode": "graph", "K": 100, "act_rows": 16, "act_waves": 4, "regrow_tile": 16}
MIN_GAIN = 0.01


def autotune(batch, trial_steps: int = 100, modes=MODES, rows=ROWS, ks=KS, waves=WAVES, tiles=TILES,
             rounds: int = 3) -> dict:
    import torch
    space = (("mode", tuple(modes)), ("K", tuple(ks)), ("act_rows", tuple(rows)), ("act_waves", tuple(waves)),
             ("regrow_tile", tuple(tiles)))
    names = [n for n, _ in space]
    saved = batch.snapshots()
    timed: dict = {}

    def trial(p: dict) -> float:
        key = tuple(p[n] for n in names)
        if key in timed:
            return timed[key]
        batch.set_mode(p["mode"])
        batch.set_tuning(p["act_rows"], p["act_waves"], p["regrow_tile"])
        K = p["K"]
        batch.load(saved)
        batch.step(min(K, trial_steps))      # capture / first launch
        batch.sync()
        batch.load(saved)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < trial_steps:
            k = min(K, trial_steps - done)
            batch.step(k)
            done += k
        batch.sync()
        timed[key] = (time.perf_counter() - t0) / trial_steps * 1e6
        return timed[key]

    cur = {n: (DEFAULT[n] if DEFAULT[n] in vals else vals[0]) for n, vals in space}
    trial(cur)
    for _ in range(rounds):
        changed = False
        for name, values in space:
            best = min(values, key=lambda v: trial(dict(cur, **{name: v})))
            # a change must gain more than 1% (timing noise and ties keep the
            # current value)
            if best != cur[name] and trial(dict(cur, **{name: best})) < (1.0 - MIN_GAIN) * trial(cur):
                cur[name] = best
                changed = True
        if not changed:
            break
    batch.load(saved)
    batch.set_mode(cur["mode"])
    batch.set_tuning(cur["act_rows"], cur["act_waves"], cur["regrow_tile"])
    trials = [dict(zip(names, k), us_per_step=v) for k, v in timed.items()]
    return {"best": dict(cur, us_per_step=timed[tuple(cur[n] for n in names)]), "trials": trials}
