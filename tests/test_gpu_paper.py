"""The paper's own dynamics (App. B: stacking, walls, energy clip, offspring on
the parent's cell, death below E_repr for T_death steps, 4-neighbour
regrowth with the climate c(x)) on the GPU, through the C-ABI: parity with the
oracle (integer state bit-exact every step) with both controllers and at the
paper's scale, and launch modes / batches / resume bit-identical."""
import numpy as np
import pytest

from parity_util import run_parity, say
from test_gpu_systems import same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_2302_09334_amd import workloads, world
    return world, oracle, workloads


def paper(wl, **kw):
    # short reproduction / starvation times and a fast regrowth, so that
    # births, deaths at walls and by starvation, and stacking all happen
    d = dict(H=40, W=72, cap=400, n_init=200, obs_radius=2, hidden=16, res_init_p=0.2, E0=120, E_max=120, decay=1,
             gain=40, E_repr=0, T_repr=25, T_death=30, L_max=650, spont=0.002, regrow_pI=0.2, regrow_alpha=200.0,
             rate_top=0.0, rate_bottom=0.0, dynamics=1)
    d.update(kw)
    return wl.make(**d)


CASES = {
    "gru": lambda wl: (paper(wl), 1, 300, 50),
    "net": lambda wl: (paper(wl, obs_radius=7, hidden=4, controller=1, w_init_gain=1.0), 2, 300, 50),
    "paper1k": lambda wl: (wl.WORKLOADS["paper1k"], 3, 200, 50),
}


@pytest.mark.parametrize("case", list(CASES))
def test_paper_parity(env, case):
    world, oracle, wl = env
    cfg, seed, steps, K = CASES[case](wl)
    say(f"[paper parity] {case} seed={seed} steps={steps}")
    st = run_parity(world.World, oracle.OracleWorld, oracle.OracleConfig, cfg, seed, steps, K, theta_every=2)
    say(f"[paper parity] {case} ok {st}")
    assert st["agent_steps"] > 0 and st["births"] > 0 and st["deaths"] > 0


NET = dict(obs_radius=7, hidden=4, controller=1, w_init_gain=1.0)
EDGES = {
    # no agents: the paper's regrowth alone
    "empty": lambda wl: (paper(wl, H=30, W=50, cap=64, n_init=0, **NET), 60, 20),
    # a grid smaller than the field of view with one agent: walls everywhere
    "tiny": lambda wl: (paper(wl, H=2, W=1, cap=4, n_init=1, res_init_p=1.0, spont=1.0, T_repr=3, **NET), 40, 7),
    # 20 cells, up to 64 agents stacked on them: the slot table binds every step
    "crowded": lambda wl: (paper(wl, H=4, W=5, cap=64, n_init=20, res_init_p=1.0, spont=1.0, regrow_pI=1.0,
                                 T_repr=3, L_max=40, **NET), 100, 25),
    "crowded_gru": lambda wl: (paper(wl, H=4, W=5, cap=64, n_init=20, res_init_p=1.0, spont=1.0, regrow_pI=1.0,
                                     T_repr=3, L_max=40), 100, 25),
    # no food at all: every agent starves, then the world stays empty
    "extinct": lambda wl: (paper(wl, H=12, W=20, cap=100, n_init=80, res_init_p=0.0, spont=0.0, regrow_pI=0.0,
                                 T_death=4, E0=4, E_max=4, **NET), 60, 20),
}


@pytest.mark.parametrize("case", list(EDGES))
def test_paper_edges(env, case):
    world, oracle, wl = env
    cfg, steps, K = EDGES[case](wl)
    say(f"[paper edge] {case} steps={steps} K={K}")
    st = run_parity(world.World, oracle.OracleWorld, oracle.OracleConfig, cfg, 5, steps, K, theta_every=1)
    say(f"[paper edge] {case} ok {st}")


def test_paper_stacks(env):
    world, oracle, wl = env
    w = world.World(paper(wl, obs_radius=7, hidden=4, controller=1, w_init_gain=1.0), 2)
    most = 1
    for _ in range(12):
        w.step(25)
        s = w.snapshot()
        cells = s["row"] * 72 + s["col"]
        most = max(most, int(np.bincount(cells).max()))
    assert most >= 2
    w.close()


def test_paper_modes_batch_resume(env):
    world, oracle, wl = env
    import torch
    cfgs = [(paper(wl), 4), (paper(wl, obs_radius=7, hidden=4, controller=1), 5)]
    for cfg, seed in cfgs:
        snaps = {}
        for mode in ("kernels", "graph"):
            w = world.World(cfg, seed, mode=mode)
            w.step(60)
            snaps[mode] = w.snapshot(hidden=True, theta=True)
            w.step(60)
            snaps[mode + "_end"] = w.snapshot(hidden=True, theta=True)
            w.close()
        same(snaps["kernels"], snaps["graph"], "graph")
        same(snaps["kernels_end"], snaps["graph_end"], "graph end")
        b = world.World(cfg, seed)
        b.step(7)
        b.load(snaps["kernels"])
        b.step(60)
        same(snaps["kernels_end"], b.snapshot(hidden=True, theta=True), "resumed")
        b.close()
        stream = torch.cuda.Stream()
        ws = [world.World(cfg, seed + k, stream=stream) for k in range(3)]
        world.step_many(ws, 60)
        for k, wk in enumerate(ws):
            a = world.World(cfg, seed + k)
            a.step(60)
            same(a.snapshot(hidden=True, theta=True), wk.snapshot(hidden=True, theta=True), f"batched {k}")
            a.close()
            wk.close()


def test_mixed_dynamics_rejected(env):
    world, oracle, wl = env
    import torch
    stream = torch.cuda.Stream()
    a = world.World(paper(wl), 1, stream=stream)
    b = world.World(wl.make(H=40, W=72, cap=400, n_init=200, obs_radius=2, hidden=16), 1, stream=stream)
    with pytest.raises(world.WorldError) as ei:
        world.step_many([a, b], 1)
    assert ei.value.code == -1
    a.close()
    b.close()
