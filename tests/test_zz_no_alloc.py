"""world_step_many_noalloc (the batched step that allocates nothing: its
launch table lives in a fixed device array) against world_step_many on
identical worlds, through the C-ABI: two calls in a row, the second with a
smaller batch, then a single world; every world's complete state bit-exact
after each call.  Also recorded into a caller's own HIP graph and replayed."""
import ctypes as C

import numpy as np
import pytest

from parity_util import say

pytestmark = pytest.mark.gpu

KEYS = ("uid", "row", "col", "energy", "age", "streak", "R", "last_action", "ate")


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_09334_amd import workloads, world
    return world, workloads, torch


def step_noalloc(world, ws, K):
    """world_step_many_noalloc through the C-ABI."""
    L = world.lib()
    arr = (C.c_void_p * len(ws))(*[w.handle for w in ws])
    rc = L.world_step_many_noalloc(arr, len(ws), int(K))
    assert rc == 0, (rc, L.world_last_error(None))


def same(a, b, where):
    assert a["t"] == b["t"] and a["n_live"] == b["n_live"] and a["next_uid"] == b["next_uid"], where
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), (where, k)
    assert np.array_equal(a["h"].view(np.uint32), b["h"].view(np.uint32)), (where, "h")
    assert np.array_equal(a["theta"].view(np.uint32), b["theta"].view(np.uint32)), (where, "theta")


def test_noalloc_equals_step_many(env):
    world, wl, torch = env
    entries = wl.batch_manifest(5, seed=3)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    A = [world.World(e["cfg"], e["seed"], stream=sa) for e in entries]
    B = [world.World(e["cfg"], e["seed"], stream=sb) for e in entries]
    for sub, K in ((slice(0, 5), 7), (slice(0, 2), 5), (slice(3, 4), 3)):
        say(f"[noalloc] worlds {sub.start}..{sub.stop - 1}, K={K}")
        step_noalloc(world, A[sub], K)
        world.step_many(B[sub], K)
        for i, (a, b) in enumerate(zip(A, B)):
            same(a.snapshot(hidden=True, theta=True), b.snapshot(hidden=True, theta=True), (sub.start, K, i))
    for w in A + B:
        w.close()


def test_noalloc_replayed_from_a_captured_graph(env):
    """A caller that cannot allocate records world_step_many_noalloc into a
    HIP graph of its own (torch.cuda.graph) and replays it: each of three
    replays advances the worlds exactly as the same call made eagerly on
    twin worlds, with the program's own reads (complete images) between the
    replays; afterwards the worlds can be moved to another stream and
    released."""
    world, wl, torch = env
    entries = wl.batch_manifest(3, seed=5)
    S, T = torch.cuda.Stream(), torch.cuda.Stream()
    A = [world.World(e["cfg"], e["seed"], stream=S) for e in entries]
    B = [world.World(e["cfg"], e["seed"], stream=T) for e in entries]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    say("[noalloc] capture into a caller's graph")
    with torch.cuda.graph(g, stream=S, capture_error_mode="thread_local"):
        step_noalloc(world, A, 4)
    for r in range(3):
        say(f"[noalloc] replay {r}")
        g.replay()
        torch.cuda.synchronize()
        step_noalloc(world, B, 4)
        for i, (a, b) in enumerate(zip(A, B)):
            same(a.snapshot(hidden=True, theta=True), b.snapshot(hidden=True, theta=True), ("replay", r, i))
    side = torch.cuda.Stream()
    for w in A:
        w.set_stream(side)
        w.sync()
    for w in A + B:
        w.close()
    del g
