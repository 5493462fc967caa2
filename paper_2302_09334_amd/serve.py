"""Continuous-batching serving loop for simulation requests.

A request is (world parameters, seed, number of steps).  Requests arrive over
time; one is admitted as soon as its device state fits in the HBM budget
(FIFO), its world is created on a separate admission stream while the
current batch runs, and it joins the next shared launch.  All admitted worlds
advance together in launches of up to K steps (world_step_many); a world
leaves when its steps are done, its final canonical state is recorded and its
memory returns to the budget.  Each world's result is bit-identical to
running it alone (the batched launch processes every agent exactly as the
single-world launch does).

Reported: per-step latency samples (wall time between consecutive launch
completions of a world divided by the steps of that launch), aggregate
agent-steps/s, admission wait and time to first step.
"""
from __future__ import annotations

import hashlib
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


def state_digest(s: dict) -> str:
    """Digest of a canonical world image (integer state, recurrent state and
    inputs, genomes)."""
    h = hashlib.sha256()
    for k in ("t", "n_live", "next_uid"):
        h.update(str(int(s[k])).encode())
    for k in ("R", "uid", "row", "col", "energy", "age", "streak", "h", "theta", "last_action", "ate"):
        if k in s:
            h.update(np.ascontiguousarray(s[k]).tobytes())
    return h.hexdigest()


class HipBackend:
    """Worlds on the GPU through libworld.so; one shared stream for launches
    and one admission stream for world creation."""

    def __init__(self, mode: str = "kernels", act_rows: int = 16, device: str = "cuda:0"):
        import torch

        from . import world
        self.world = world
        self.torch = torch
        self.mode = mode
        self.act_rows = act_rows
        self.device = device
        self.stream = torch.cuda.Stream(device=device)
        self.admit_stream = torch.cuda.Stream(device=device)

    def required_bytes(self, cfg: dict) -> int:
        return self.world.required_bytes(cfg)

    def create(self, cfg: dict, seed: int):
        w = self.world.World(cfg, seed, device=self.device, stream=self.admit_stream, mode=self.mode)
        w.set_tuning(self.act_rows)
        w.set_stream(self.stream)
        return w

    def step_many(self, worlds: list, k: int):
        self.world.step_many(worlds, k)

    def mark(self):
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        return ev

    def wait(self, mark):
        mark.synchronize()

    def agent_steps(self, w, steps: int) -> int:
        c = w.counters(0, steps)["n_live"]
        return int(w.cfg["n_init"]) + int(c[:-1].sum())

    def result(self, w) -> dict:
        s = w.snapshot(hidden=True, theta=True)
        return {"digest": state_digest(s), "n_live": s["n_live"], "t": s["t"]}

    def close(self, w):
        w.close()


@dataclass
class Request:
    rid: int
    arrival: float
    cfg: dict
    seed: int
    steps: int


@dataclass
class Active:
    req: Request
    world: object
    nbytes: int
    admitted: float
    done: int = 0
    first_step: float | None = None
    last_done: float | None = None
    latencies: list = field(default_factory=list)


class Server:
    def __init__(self, backend, budget_bytes: int, K: int = 50, max_batch: int | None = None):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.K = int(K)
        self.max_batch = max_batch

    def run(self, requests: list[Request], duration: float | None = None, realtime: bool = True,
            clock=time.perf_counter) -> tuple[dict, dict]:
        """Serve `requests` (sorted by arrival time, seconds from start).  With
        `duration`, arrivals after it are dropped and the active set drains."""
        t0 = clock()
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        if duration is not None:
            pending = deque(r for r in pending if r.arrival <= duration)
        queue: deque[Request] = deque()
        active: list[Active] = []
        used = 0
        peak_used = 0
        results: dict[int, dict] = {}
        samples: list[float] = []
        waits: list[float] = []
        ttfs: list[float] = []
        agent_steps = 0
        launches = 0
        sim_time = 0.0   # virtual clock when not real time

        def now():
            return (clock() - t0) if realtime else sim_time

        def admit():
            nonlocal used, peak_used
            while queue and (self.max_batch is None or len(active) < self.max_batch):
                need = self.backend.required_bytes(queue[0].cfg)
                if need > self.budget:
                    r = queue.popleft()
                    results[r.rid] = {"error": "request larger than the budget"}
                    continue
                if used + need > self.budget:
                    break
                r = queue.popleft()
                w = self.backend.create(r.cfg, r.seed)
                used += need
                peak_used = max(peak_used, used)
                a = Active(r, w, need, admitted=now())
                waits.append(a.admitted - r.arrival)
                active.append(a)

        while pending or queue or active:
            t = now()
            while pending and pending[0].arrival <= t:
                queue.append(pending.popleft())
            admit()
            if not active:
                if pending:
                    if realtime:
                        time.sleep(max(0.0, min(0.05, pending[0].arrival - now())))
                    else:
                        sim_time = max(sim_time, pending[0].arrival)
                continue
            k = min(self.K, min(a.req.steps - a.done for a in active))
            batch = list(active)
            # one shared launch per kind of world (a launch covers worlds of one
            # controller and one rule set); the launches queue on one stream
            for group in world_kinds(batch).values():
                self.backend.step_many([a.world for a in group], k)
            end = self.backend.mark()
            launches += 1
            # overlap: admit requests that arrived meanwhile while the launch runs
            t = now()
            while pending and pending[0].arrival <= t:
                queue.append(pending.popleft())
            admit()
            self.backend.wait(end)
            if not realtime:
                sim_time += 1e-3
            t_done = now()
            for a in batch:
                a.done += k
                prev = a.last_done if a.last_done is not None else a.admitted
                lat = (t_done - prev) / k * 1e3
                a.latencies.append(lat)
                samples.append(lat)
                if a.first_step is None:
                    a.first_step = t_done
                    ttfs.append(t_done - a.req.arrival)
                a.last_done = t_done
            finished = [a for a in active if a.done >= a.req.steps]
            for a in finished:
                res = self.backend.result(a.world)
                steps_run = self.backend.agent_steps(a.world, a.req.steps)
                agent_steps += steps_run
                res.update(steps=a.done, agent_steps=steps_run, admitted=a.admitted,
                           first_step=a.first_step, finished=now())
                results[a.req.rid] = res
                self.backend.close(a.world)
                used -= a.nbytes
                active.remove(a)
        wall = now()
        lat = np.array(samples) if samples else np.zeros(1)
        metrics = {
            "requests": len(results), "wall_s": wall, "launches": launches,
            "agent_steps": agent_steps, "agent_steps_per_s": agent_steps / wall if wall > 0 else 0.0,
            "step_ms_p50": float(np.percentile(lat, 50)), "step_ms_p99": float(np.percentile(lat, 99)),
            "admission_wait_s_p50": float(np.percentile(waits, 50)) if waits else 0.0,
            "admission_wait_s_p99": float(np.percentile(waits, 99)) if waits else 0.0,
            "time_to_first_step_s_p50": float(np.percentile(ttfs, 50)) if ttfs else 0.0,
            "peak_budget_used_bytes": peak_used, "budget_bytes": self.budget,
        }
        return results, metrics


def world_kind(cfg: dict) -> tuple:
    """Worlds of one kind (controller, dynamics) can share a launch."""
    return (int(cfg.get("controller", 0)), int(cfg.get("dynamics", 0)))


def world_kinds(active: list) -> dict:
    groups: dict = {}
    for a in active:
        groups.setdefault(world_kind(a.req.cfg), []).append(a)
    return groups


def requests_from_trace(trace: list[dict]) -> list[Request]:
    return [Request(i, float(e["arrival"]), e["cfg"], int(e["seed"]), int(e["steps"])) for i, e in enumerate(trace)]
