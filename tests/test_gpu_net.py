"""The paper's controller (App. B.5) on the GPU, through the C-ABI: the Gumbel
transform of its action sampling bit for bit, parity with the oracle (integer
state bit-exact every step, logits within 1e-5 relative, sampled actions equal
except inside the near-tie band of the sampling scores), and the systems
properties (launch modes, batches, resume) bit-exact."""
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


def net(wl, **kw):
    d = dict(H=40, W=72, cap=300, n_init=200, obs_radius=7, hidden=4, res_init_p=0.4, rate_scale=5.0,
             T_repr=8, L_max=150, w_init_gain=1.0, controller=1)
    d.update(kw)
    return wl.make(**d)


def test_gumbel_bit_exact(env):
    world, oracle, wl = env
    rng = np.random.default_rng(1)
    w = rng.integers(0, 2**32, size=1 << 20, dtype=np.uint64).astype(np.uint32)
    w[:512] = np.arange(512, dtype=np.uint32) << 9            # smallest u
    w[512:1024] = 0xFFFFFFFF - (np.arange(512, dtype=np.uint32) << 9)   # largest u
    g = world.test_gumbel(w)
    o = oracle.gumbel(w)
    assert np.array_equal(g.view(np.uint32), o.view(np.uint32))


CASES = {
    # a crowded world: many collisions, births and deaths
    "dense": lambda wl: (net(wl), 1, 300, 50),
    # a grid smaller than the field of view: walls on every side
    "walls": lambda wl: (net(wl, H=9, W=6, cap=40, n_init=20), 2, 200, 50),
    # the paper's own scale (330 agents at the start, at most 1000)
    "net1k": lambda wl: (wl.WORKLOADS["net1k"], 3, 100, 50),
}


@pytest.mark.parametrize("case", list(CASES))
def test_net_parity(env, case):
    world, oracle, wl = env
    cfg, seed, steps, K = CASES[case](wl)
    say(f"[net parity] {case} seed={seed} steps={steps} K={K}")
    st = run_parity(world.World, oracle.OracleWorld, oracle.OracleConfig, cfg, seed, steps, K, theta_every=2)
    say(f"[net parity] {case} ok {st}")
    assert st["agent_steps"] > 0


def test_net_parity_fullsize(env):
    """The net_m1_4k world (about 4k agents, the configuration the benchmark
    times), every agent of 20 steps against the oracle."""
    world, oracle, wl = env
    say("[net parity] net_m1_4k 20 steps")
    st = run_parity(world.World, oracle.OracleWorld, oracle.OracleConfig, wl.WORKLOADS["net_m1_4k"], 0, 20, 10)
    say(f"[net parity] net_m1_4k ok {st}")
    assert st["agent_steps"] > 40000


def test_net_graph_batch_resume(env):
    # Each world alone has at most 16 agent slots per CU, so it runs the act
    # kernel compiled for four waves per SIMD; together they exceed that and
    # the batched launch runs the five-wave kernel: the results must not change.
    world, oracle, wl = env
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    cfgs = [(net(wl), 5), (net(wl, H=64, W=128, cap=512, n_init=300), 6), (wl.WORKLOADS["net1k"], 7),
            (net(wl, H=100, W=200, cap=16 * cus, n_init=1500), 8)]
    assert all(c["cap"] <= 16 * cus for c, _ in cfgs) and sum(c["cap"] for c, _ in cfgs) > 16 * cus
    say("[net systems] alone (kernels), alone (graph), batched")
    alone = {}
    for mode in ("kernels", "graph"):
        for i, (cfg, seed) in enumerate(cfgs):
            w = world.World(cfg, seed, mode=mode)
            for _ in range(3):
                w.step(40)
            alone[(mode, i)] = w.snapshot(hidden=True, theta=True)
            w.close()
    for i in range(len(cfgs)):
        same(alone[("kernels", i)], alone[("graph", i)], f"graph {i}")
    stream = torch.cuda.Stream()
    ws = [world.World(cfg, seed, stream=stream, mode="graph") for cfg, seed in cfgs]
    for _ in range(3):
        world.step_many(ws, 40)
    for i, w in enumerate(ws):
        same(alone[("kernels", i)], w.snapshot(hidden=True, theta=True), f"batched {i}")
    for w in ws:
        w.close()
    # resume from a snapshot taken mid-run
    cfg, seed = cfgs[0]
    a = world.World(cfg, seed)
    a.step(70)
    mid = a.snapshot(hidden=True, theta=True)
    a.step(50)
    ref = a.snapshot(hidden=True, theta=True)
    b = world.World(cfg, seed)   # the seed keys the generator: it is configuration, not state
    b.step(3)                    # any other state
    b.load(mid)
    b.step(50)
    same(ref, b.snapshot(hidden=True, theta=True), "resumed")
    a.close()
    b.close()


def test_mixed_controllers_rejected(env):
    world, oracle, wl = env
    import torch
    stream = torch.cuda.Stream()
    a = world.World(net(wl), 1, stream=stream)
    b = world.World(wl.WORKLOADS["cfg0"], 1, stream=stream)
    with pytest.raises(world.WorldError) as ei:
        world.step_many([a, b], 1)
    assert ei.value.code == -1
    a.close()
    b.close()
