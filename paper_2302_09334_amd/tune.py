"""Autotuner for batched launches.

Only knobs that cannot change any result are searched: the launch mode
(per-phase kernels or a captured graph), the number of
steps per launch, and the act kernel's rows per round trip.  Every trial runs
from the same saved state and the state is restored exactly afterwards, so
tuning leaves the simulation where it was.
"""
from __future__ import annotations

import time

from .batch import WorldBatch

MODES = ("graph", "kernels")
ROWS = (8, 16, 32)
KS = (25, 50, 100)


def autotune(batch: WorldBatch, trial_steps: int = 100, modes=MODES, rows=ROWS, ks=KS) -> dict:
    import torch
    saved = batch.snapshots()
    results = []
    for mode in modes:
        for r in rows:
            for K in ks:
                batch.set_mode(mode)
                batch.set_tuning(r)
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
                results.append({"mode": mode, "act_rows": r, "K": K,
                                "us_per_step": (time.perf_counter() - t0) / trial_steps * 1e6})
    best = min(results, key=lambda x: x["us_per_step"])
    batch.load(saved)
    batch.set_mode(best["mode"])
    batch.set_tuning(best["act_rows"])
    return {"best": best, "trials": results}
