"""Serving and batching on the GPU: each served result equals the same
request run alone; autotuning leaves the simulation state untouched."""
import numpy as np
import pytest

from parity_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_09334_amd import batch, serve, tune, workloads, world
    return world, serve, batch, tune, workloads


@pytest.mark.parametrize("mode", ["kernels", "graph"])
def test_served_equals_alone(env, mode):
    world, serve, batch, tune, wl = env
    reqs = []
    for i in range(8):
        cfg = wl.make(H=[64, 100, 128][i % 3], W=[128, 200, 256][i % 3], cap=512 + 64 * i, n_init=51 + 6 * i,
                      hidden=16 if i % 2 else 32, rate_scale=1.0 + 0.25 * i, res_init_p=0.3)
        reqs.append(serve.Request(i, arrival=0.02 * i, cfg=cfg, seed=50 + i, steps=60 + 35 * (i % 4)))
    be = serve.HipBackend(mode=mode)
    budget = 3 * max(world.required_bytes(r.cfg) for r in reqs)
    say(f"[serve] mode={mode} budget={budget}")
    results, m = serve.Server(be, budget_bytes=budget, K=25).run(reqs, realtime=True)
    say(f"[serve] {m}")
    assert len(results) == len(reqs) and m["peak_budget_used_bytes"] <= budget
    for r in reqs:
        w = world.World(r.cfg, r.seed, mode="graph")
        w.step(r.steps)
        alone = serve.state_digest(w.snapshot(hidden=True, theta=True))
        w.close()
        assert results[r.rid]["digest"] == alone, r.rid


def test_autotune_preserves_state(env):
    world, serve, batch, tune, wl = env
    entries = [e for e in wl.batch_manifest(6, seed=4)]
    for e in entries:
        e["cfg"] = dict(e["cfg"], cap=min(e["cfg"]["cap"], 1024), n_init=min(e["cfg"]["n_init"], 100))
    a = batch.WorldBatch(entries, mode="graph")
    a.step(20)
    before = a.snapshots()
    res = tune.autotune(a, trial_steps=20, ks=(10, 20))
    say(f"[tune] best {res['best']}")
    after = a.snapshots()
    for x, y in zip(before, after):
        for k in ("uid", "row", "col", "energy", "age", "streak", "R", "h", "theta"):
            assert np.array_equal(np.asarray(x[k]), np.asarray(y[k])), k
    a.step(30)
    b = batch.WorldBatch(entries, mode="kernels")
    b.step(20)
    b.step(30)
    for x, y in zip(a.snapshots(), b.snapshots()):
        assert serve.state_digest(x) == serve.state_digest(y)
    a.close()
    b.close()


def test_served_mixed_kinds_equal_alone(env):
    """Requests with both controllers and both rule sets served together (one
    shared launch per kind): every result equals the same request run alone."""
    world, serve, batch, tune, wl = env
    reqs = []
    for i in range(8):
        kw = dict(H=[64, 100][i % 2], W=[128, 200][i % 2], cap=256 + 64 * i, n_init=40 + 5 * i, res_init_p=0.3,
                  rate_scale=2.0, T_repr=10, L_max=300)
        if i % 2:
            kw.update(obs_radius=7, hidden=4, controller=1, w_init_gain=1.0)
        if i % 4 >= 2:
            kw.update(dynamics=1, E0=120, E_max=120, decay=1, gain=40, E_repr=0, T_repr=20, T_death=25,
                      regrow_pI=0.2, regrow_alpha=200.0, spont=0.002)
        reqs.append(serve.Request(i, arrival=0.01 * i, cfg=wl.make(**kw), seed=70 + i, steps=40 + 20 * (i % 3)))
    be = serve.HipBackend(mode="graph")
    budget = 4 * max(world.required_bytes(r.cfg) for r in reqs)
    results, m = serve.Server(be, budget_bytes=budget, K=20).run(reqs, realtime=True)
    say(f"[serve mixed] {m}")
    assert len(results) == len(reqs)
    for r in reqs:
        w = world.World(r.cfg, r.seed, mode="graph")
        w.step(r.steps)
        alone = serve.state_digest(w.snapshot(hidden=True, theta=True))
        w.close()
        assert results[r.rid]["digest"] == alone, r.rid


def test_finish_while_loop_captures(env):
    """What the serving loop's helper threads do while the loop launches on
    the shared stream, capturing a new graph for every launch: create a world
    on a side stream, move finished worlds off the shared stream, read their
    images and counters, and release them (with the batch launch tables that
    list them).  None of these calls may synchronise with the shared stream
    or the legacy default stream (HIP makes that one depend on it) while a
    capture is in progress there; every result must equal the same world
    stepped alone."""
    import threading

    import torch
    world, serve, batch, tune, wl = env
    cfg = wl.make(H=64, W=128, cap=512, n_init=51, hidden=16, rate_scale=1.0, res_init_p=0.3)
    S, side = torch.cuda.Stream(), torch.cuda.Stream()
    runners = [world.World(cfg, 20 + i, stream=S, mode="graph") for i in range(2)]
    leaving = [world.World(cfg, 30 + i, stream=S, mode="graph") for i in range(6)]
    world.step_many(leaving[:3], 4)   # batch tables listing the leaving worlds
    world.step_many(leaving[3:], 4)
    for w in leaving:
        w.step(2)
    errors, images, created = [], {}, []

    def finisher():
        try:
            for i, w in enumerate(leaving):
                created.append(world.World(cfg, 90 + i, stream=side, mode="graph"))
                w.set_stream(side)
                img = w.snapshot(hidden=True, theta=True)
                ctr = w.counters(0, 6)
                w.close()
                images[i] = (serve.state_digest(img), int(ctr["n_live"][-1]) == img["n_live"])
        except Exception as e:
            errors.append(repr(e))

    say("[serve] a helper thread finishes worlds while the loop captures a graph per launch")
    th = threading.Thread(target=finisher)
    th.start()
    steps, K = 0, 1
    while (th.is_alive() or K <= 8) and K <= 40:
        world.step_many(runners, K)   # a new K: a new capture
        steps += K
        K += 1
    th.join()
    torch.cuda.synchronize()
    assert not errors, errors
    assert len(created) == len(leaving)
    for i in range(len(leaving)):
        alone = world.World(cfg, 30 + i, mode="graph")
        alone.step(6)
        assert images[i][0] == serve.state_digest(alone.snapshot(hidden=True, theta=True)), i
        assert images[i][1], i
        alone.close()
    for i, w in enumerate(runners):
        w.sync()
        alone = world.World(cfg, 20 + i, mode="graph")
        alone.step(steps)
        assert serve.state_digest(w.snapshot(hidden=True, theta=True)) == \
            serve.state_digest(alone.snapshot(hidden=True, theta=True)), i
