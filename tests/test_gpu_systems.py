"""GPU path properties that need no oracle: determinism across launch modes,
batched stepping bit-identical to stepping alone, and exact resume from a
snapshot (through the C-ABI)."""
import numpy as np
import pytest

from parity_util import say

pytestmark = pytest.mark.gpu

KEYS = ("uid", "row", "col", "energy", "age", "streak", "R")


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_09334_amd import workloads, world
    return world, workloads


def dense(wl, **kw):
    d = dict(H=40, W=72, cap=300, n_init=200, obs_radius=2, hidden=16, res_init_p=0.4, rate_scale=5.0,
             T_repr=8, L_max=150)
    d.update(kw)
    return wl.make(**d)


def same(a, b, where):
    assert a["t"] == b["t"] and a["n_live"] == b["n_live"] and a["next_uid"] == b["next_uid"], where
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), (where, k)
    assert np.array_equal(a["h"].view(np.uint32), b["h"].view(np.uint32)), (where, "h")
    assert np.array_equal(a["theta"].view(np.uint32), b["theta"].view(np.uint32)), (where, "theta")


def test_modes_bit_identical(env):
    world, wl = env
    cfg = dense(wl, obs_radius=3, hidden=32)
    snaps = {}
    for mode in ("kernels", "graph"):
        say(f"[systems] mode {mode}")
        w = world.World(cfg, 11, mode=mode)
        for _ in range(4):
            w.step(30)
        snaps[mode] = w.snapshot(hidden=True, theta=True)
        w.close()
    same(snaps["kernels"], snaps["graph"], "graph")
    # and the same run again
    w = world.World(cfg, 11, mode="kernels")
    for _ in range(4):
        w.step(30)
    same(snaps["kernels"], w.snapshot(hidden=True, theta=True), "rerun")


@pytest.mark.parametrize("mode", ["kernels", "graph"])
def test_batched_equals_alone(env, mode):
    world, wl = env
    import torch
    cfgs = [
        (dense(wl), 1),
        (dense(wl, H=50, W=90, cap=400, n_init=300, obs_radius=3, hidden=32), 2),
        (wl.WORKLOADS["cfg0"], 3),
        (dense(wl, obs_radius=1, H=33, W=17, cap=250, n_init=150), 4),
        (dense(wl, H=64, W=128, cap=512, n_init=51, obs_radius=3, hidden=32, rate_scale=1.3), 5),
    ]
    say(f"[systems] batched vs alone, mode {mode}")
    stream = torch.cuda.Stream()
    alone = []
    for cfg, seed in cfgs:
        w = world.World(cfg, seed, mode=mode)
        for _ in range(3):
            w.step(40)
        alone.append(w.snapshot(hidden=True, theta=True))
        w.close()
    ws = [world.World(cfg, seed, stream=stream, mode=mode) for cfg, seed in cfgs]
    for _ in range(3):
        world.step_many(ws, 40)
    for i, w in enumerate(ws):
        same(alone[i], w.snapshot(hidden=True, theta=True), f"world {i}")
    # a sub-batch keeps going consistently
    world.step_many(ws[1:3], 10)
    for w in ws:
        w.close()


def test_snapshot_load_resume(env):
    world, wl = env
    cfg = dense(wl, obs_radius=3, hidden=32)
    a = world.World(cfg, 7, mode="graph")
    a.step(60)
    mid = a.snapshot(hidden=True, theta=True)
    a.step(60)
    ref = a.snapshot(hidden=True, theta=True)
    b = world.World(cfg, 7, mode="kernels")
    b.step(5)   # any other state
    b.load(mid)
    assert b.snapshot(hidden=True, theta=True)["t"] == mid["t"]
    b.set_mode("graph")
    b.step(60)
    same(ref, b.snapshot(hidden=True, theta=True), "resumed")
    # counters of the resumed steps match the uninterrupted run
    ca, cb = a.counters(mid["t"], 60), b.counters(mid["t"], 60)
    for k in ca:
        assert np.array_equal(ca[k], cb[k]), k


def test_load_rejects_bad_images(env):
    world, wl = env
    cfg = dense(wl)
    w = world.World(cfg, 1)
    s = w.snapshot(hidden=True, theta=True)
    bad = dict(s)
    bad["row"] = s["row"].copy()
    bad["col"] = s["col"].copy()
    bad["row"][1], bad["col"][1] = s["row"][0], s["col"][0]
    with pytest.raises(world.WorldError):
        w.load(bad)
    bad = dict(s)
    bad["uid"] = s["uid"][::-1].copy()
    with pytest.raises(world.WorldError):
        w.load(bad)
    # the world is still usable after a rejected load
    w.step(3)
    w.sync()
