"""Many independent worlds of uneven size advanced in shared launches.

Every launch covers all worlds of the batch (one grid per phase, worlds found
by a block-prefix search), and each world's result is bit-identical to
stepping it alone: an agent is always processed by the same code with the
same reduction order, whatever else is in the launch.
"""
from __future__ import annotations

import time

import numpy as np

from . import world


class WorldBatch:
    """Worlds sharing one stream, stepped together with world_step_many."""

    def __init__(self, entries: list[dict], stream=None, mode: str = "graph", act_rows: int = 16):
        import torch
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.worlds = [world.World(e["cfg"], e["seed"], stream=self.stream, mode=mode) for e in entries]
        self.set_mode(mode)
        self.set_tuning(act_rows)

    def set_mode(self, mode: str):
        self.mode = mode
        for w in self.worlds:
            w.set_mode(mode)

    def set_tuning(self, act_rows: int = 16, act_waves: int = 4, regrow_tile: int = 16):
        self.act_rows, self.act_waves, self.regrow_tile = act_rows, act_waves, regrow_tile
        for w in self.worlds:
            w.set_tuning(act_rows, act_waves, regrow_tile)

    def step(self, K: int):
        world.step_many(self.worlds, K)

    def sync(self):
        self.stream.synchronize()
        for w in self.worlds:
            w.sync()

    def snapshots(self, hidden: bool = True, theta: bool = True) -> list[dict]:
        return [w.snapshot(hidden=hidden, theta=theta) for w in self.worlds]

    def load(self, snaps: list[dict]):
        for w, s in zip(self.worlds, snaps):
            w.load(s)

    def acting_agents(self, first: int, n: int) -> int:
        """Agent-steps of steps [first, first + n) summed over the worlds."""
        total = 0
        for w in self.worlds:
            prev = w.counters(first - 1, 1)["n_live"][0] if first > 0 else w.cfg["n_init"]
            c = w.counters(first, n)["n_live"]
            total += int(prev) + int(c[:-1].sum())
        return total

    def close(self):
        for w in self.worlds:
            w.close()
        self.worlds = []


def time_chunks(step_fn, steps: int, K: int, stream) -> tuple[float, np.ndarray]:
    """Run `steps` steps as launches of K, timing each launch with events.
    Returns (wall seconds, per-launch milliseconds)."""
    import torch
    n = (steps + K - 1) // K
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    done = 0
    for i in range(n):
        k = min(K, steps - done)
        step_fn(k)
        done += k
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(n)])


def run_batched(entries: list[dict], warmup: int, steps: int, K: int, mode: str = "graph",
                act_rows: int = 16) -> dict:
    b = WorldBatch(entries, mode=mode, act_rows=act_rows)
    done = 0
    while done < warmup:
        k = min(K, warmup - done)
        b.step(k)
        done += k
    b.sync()
    wall, chunk_ms = time_chunks(b.step, steps, K, b.stream)
    b.sync()
    agent_steps = b.acting_agents(warmup, steps)
    out = {"wall_s": wall, "agent_steps": agent_steps, "agent_steps_per_s": agent_steps / wall,
           "chunk_ms": chunk_ms, "step_ms_p50": float(np.percentile(chunk_ms / K, 50)),
           "step_ms_p99": float(np.percentile(chunk_ms / K, 99))}
    b.close()
    return out


def run_sequential(entries: list[dict], warmup: int, steps: int, K: int, mode: str = "graph") -> dict:
    """The plain path: each world stepped alone with world_step, one after another."""
    import torch
    stream = torch.cuda.Stream()
    total_wall = 0.0
    agent_steps = 0
    for e in entries:
        w = world.World(e["cfg"], e["seed"], stream=stream, mode=mode)
        done = 0
        while done < warmup:
            k = min(K, warmup - done)
            w.step(k)
            done += k
        w.sync()
        s0 = w.snapshot(hidden=True, theta=True)
        w.step(min(K, steps))   # graph capture / first launch, outside the timed region
        w.sync()
        w.load(s0)
        wall, _ = time_chunks(w.step, steps, K, stream)
        total_wall += wall
        prev = w.counters(warmup - 1, 1)["n_live"][0] if warmup > 0 else e["cfg"]["n_init"]
        agent_steps += int(prev) + int(w.counters(warmup, steps)["n_live"][:-1].sum())
        w.close()
    return {"wall_s": total_wall, "agent_steps": agent_steps, "agent_steps_per_s": agent_steps / total_wall}
