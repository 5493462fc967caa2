"""Continuous-batching serving loop for simulation requests.

A request is (world parameters, seed, number of steps).  Requests arrive over
time; one is admitted as soon as its device state fits in the HBM budget
(FIFO, the budget reserved at once).  With a backend that can create worlds
in the background (HipBackend: a creator thread, world_create on its own
stream), the serving loop never waits for a creation: a new world joins the
first launch after it is ready.  All admitted worlds advance together in
launches of K steps (world_step_many, one launch per kind of world); worlds
with fewer than K steps left run their remaining steps in a launch of their
own on the same stream, so one world's end never shortens the others'
launch.  A world that is done leaves the active set at once; its final
canonical state is recorded in the background (a finisher thread) and its
memory returns to the budget when that is done.  Each world's result is
bit-identical to running it alone (a batched launch processes every agent
exactly as the single-world launch does).

Reported: per-step latency samples -- the device time of each launch a world
was in (events on the launch stream) divided by its steps, and separately the
wall time between consecutive launch completions of a world from its first
launch on, divided by the steps; aggregate agent-steps/s; admission wait
(arrival to admission) and time to first step.
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
    """Worlds on the GPU through libworld.so: one shared stream for the
    launches; worlds are created by a creator thread (each creation on its
    own stream, then moved to the launch stream) and finished -- final image,
    counters, release -- by a finisher thread, so the serving loop only
    enqueues launches and waits for them."""

    def __init__(self, mode: str = "kernels", act_rows: int = 16, device: str = "cuda:0", background: bool = True):
        import concurrent.futures as cf
        import threading

        import torch

        from . import world
        self.world = world
        self.torch = torch
        self.mode = mode
        self.act_rows = act_rows
        self.device = device
        self.stream = torch.cuda.Stream(device=device)
        self._local = threading.local()
        self.background = background
        if background:
            self._creator = cf.ThreadPoolExecutor(max_workers=1, thread_name_prefix="create")
            self._finisher = cf.ThreadPoolExecutor(max_workers=1, thread_name_prefix="finish")

    def required_bytes(self, cfg: dict) -> int:
        return self.world.required_bytes(cfg)

    def _side_stream(self):
        s = getattr(self._local, "stream", None)
        if s is None:
            s = self._local.stream = self.torch.cuda.Stream(device=self.device)
        return s

    def create(self, cfg: dict, seed: int):
        w = self.world.World(cfg, seed, device=self.device, stream=self._side_stream(), mode=self.mode)
        w.set_tuning(self.act_rows)
        w.set_stream(self.stream)
        return w

    def create_async(self, cfg: dict, seed: int):
        """A future of create(cfg, seed), run by the creator thread."""
        return self._creator.submit(self.create, cfg, seed)

    def step_many(self, worlds: list, k: int):
        self.world.step_many_noalloc(worlds, k) if self.mode == "kernels" else self.world.step_many(worlds, k)

    def mark(self):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(self.stream)
        return ev

    def wait(self, mark):
        mark.synchronize()

    def elapsed_ms(self, a, b) -> float:
        """Device time between two marks (both completed)."""
        return float(a.elapsed_time(b))

    def agent_steps(self, w, steps: int) -> int:
        c = w.counters(0, steps)["n_live"]
        return int(w.cfg["n_init"]) + int(c[:-1].sum())

    def result(self, w) -> dict:
        s = w.snapshot(hidden=True, theta=True)
        return {"digest": state_digest(s), "n_live": s["n_live"], "t": s["t"]}

    def close(self, w):
        w.close()

    def _finish(self, w, steps: int):
        w.set_stream(self._side_stream())   # waits for the launches it was in
        res = self.result(w)
        res["agent_steps"] = self.agent_steps(w, steps)
        self.close(w)
        return res

    def finish_async(self, w, steps: int):
        """A future of (result with agent_steps), run by the finisher thread;
        the world is released when it completes."""
        return self._finisher.submit(self._finish, w, steps)

    def shutdown(self):
        if self.background:
            self._creator.shutdown(wait=True)
            self._finisher.shutdown(wait=True)


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
            clock=time.perf_counter, progress=None, progress_every: float = 30.0) -> tuple[dict, dict]:
        """Serve `requests` (sorted by arrival time, seconds from start).  With
        `duration`, arrivals after it are dropped and the active set drains.
        `progress(t, done, active, queued)` is called every `progress_every`
        seconds of the run (queued: arrived and not yet admitted)."""
        be = self.backend
        async_create = realtime and hasattr(be, "create_async")
        async_finish = realtime and hasattr(be, "finish_async")
        t0 = clock()
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        if duration is not None:
            pending = deque(r for r in pending if r.arrival <= duration)
        queue: deque[Request] = deque()
        creating: list = []      # (request, future, bytes)
        finishing: list = []     # (Active, future)
        active: list[Active] = []
        used = 0
        peak_used = 0
        results: dict[int, dict] = {}
        dev_samples: list[float] = []
        wall_samples: list[float] = []
        waits: list[float] = []
        ttfs: list[float] = []
        agent_steps = 0
        launches = 0
        sim_time = 0.0   # virtual clock when not real time

        def now():
            return (clock() - t0) if realtime else sim_time

        def admit():
            nonlocal used, peak_used
            while queue and (self.max_batch is None or len(active) + len(creating) < self.max_batch):
                need = be.required_bytes(queue[0].cfg)
                if need > self.budget:
                    r = queue.popleft()
                    results[r.rid] = {"error": "request larger than the budget"}
                    continue
                if used + need > self.budget:
                    break
                r = queue.popleft()
                used += need
                peak_used = max(peak_used, used)
                waits.append(now() - r.arrival)
                if async_create:
                    creating.append((r, be.create_async(r.cfg, r.seed), need))
                else:
                    active.append(Active(r, be.create(r.cfg, r.seed), need, admitted=now()))

        def join_created(block: bool):
            still = []
            for r, fut, need in creating:
                if fut.done() or block:
                    active.append(Active(r, fut.result(), need, admitted=now()))
                else:
                    still.append((r, fut, need))
            creating[:] = still

        def reap_finished(block: bool):
            nonlocal used, agent_steps
            still = []
            for a, fut in finishing:
                if fut.done() or block:
                    res = fut.result()
                    agent_steps += res["agent_steps"]
                    res.update(steps=a.done, admitted=a.admitted, first_step=a.first_step, finished=now())
                    results[a.req.rid] = res
                    used -= a.nbytes
                else:
                    still.append((a, fut))
            finishing[:] = still

        next_report = progress_every
        while pending or queue or active or creating or finishing:
            t = now()
            if progress is not None and t >= next_report:
                progress(t, len(results), len(active) + len(creating), len(queue))
                next_report += progress_every
            while pending and pending[0].arrival <= t:
                queue.append(pending.popleft())
            reap_finished(block=False)
            admit()
            join_created(block=not active and not pending and not queue)
            if not active:
                if finishing and not creating:
                    reap_finished(block=not pending and not queue)
                if pending and not creating and not queue:
                    if realtime:
                        time.sleep(max(0.0, min(0.005, pending[0].arrival - now())))
                    else:
                        sim_time = max(sim_time, pending[0].arrival)
                elif creating and realtime:
                    time.sleep(0.0005)
                continue
            # launches: worlds with at least K steps left together (one launch
            # per kind), the others by their remaining steps
            groups: dict = {}
            for a in active:
                k = min(self.K, a.req.steps - a.done)
                groups.setdefault((k, world_kind(a.req.cfg)), []).append(a)
            marks = []
            for (k, _), group in sorted(groups.items(), key=lambda kv: -kv[0][0]):
                m0 = be.mark()
                be.step_many([a.world for a in group], k)
                marks.append((k, group, m0, be.mark()))
                launches += 1
            # overlap: admit requests that arrived meanwhile while the launches run
            t = now()
            while pending and pending[0].arrival <= t:
                queue.append(pending.popleft())
            admit()
            be.wait(marks[-1][3])
            if not realtime:
                sim_time += 1e-3
            t_done = now()
            for k, group, m0, m1 in marks:
                dev_ms = be.elapsed_ms(m0, m1) if hasattr(be, "elapsed_ms") else None
                for a in group:
                    a.done += k
                    if dev_ms is not None:
                        dev_samples.append(dev_ms / k)
                    if a.last_done is not None:
                        lat = (t_done - a.last_done) / k * 1e3
                        a.latencies.append(lat)
                        wall_samples.append(lat)
                    if a.first_step is None:
                        a.first_step = t_done
                        ttfs.append(t_done - a.req.arrival)
                    a.last_done = t_done
            finished = [a for a in active if a.done >= a.req.steps]
            for a in finished:
                active.remove(a)
                if async_finish:
                    finishing.append((a, be.finish_async(a.world, a.req.steps)))
                else:
                    res = be.result(a.world)
                    steps_run = be.agent_steps(a.world, a.req.steps)
                    agent_steps += steps_run
                    res.update(steps=a.done, agent_steps=steps_run, admitted=a.admitted,
                               first_step=a.first_step, finished=now())
                    results[a.req.rid] = res
                    be.close(a.world)
                    used -= a.nbytes
        wall = now()

        def pct(x, q):
            return float(np.percentile(x, q)) if len(x) else 0.0

        lat = dev_samples if dev_samples else wall_samples
        metrics = {
            "requests": len(results), "wall_s": wall, "launches": launches,
            "agent_steps": agent_steps, "agent_steps_per_s": agent_steps / wall if wall > 0 else 0.0,
            "step_ms_p50": pct(lat, 50), "step_ms_p99": pct(lat, 99),
            "step_ms_basis": "device time of each launch a world was in / its steps" if dev_samples else
                             "wall time between consecutive launch completions of a world / steps",
            "step_wall_ms_p50": pct(wall_samples, 50), "step_wall_ms_p99": pct(wall_samples, 99),
            "admission_wait_s_p50": pct(waits, 50), "admission_wait_s_p99": pct(waits, 99),
            "time_to_first_step_s_p50": pct(ttfs, 50), "time_to_first_step_s_p99": pct(ttfs, 99),
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
