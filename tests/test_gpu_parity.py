"""GPU path vs the oracle, through the C-ABI (bit-exact integer state every
step, logits within 1e-5 relative, near-tie resync only)."""
import numpy as np
import pytest

from parity_util import run_parity, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_2302_09334_amd import workloads, world
    return world, oracle, workloads


def test_primitives_bit_exact(env):
    world, oracle, wl = env
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**32, size=(50000, 4), dtype=np.uint64).astype(np.uint32)
    for key in ([0, 0], [123456789, 42], [0xFFFFFFFF, 0xFFFFFFFF]):
        assert np.array_equal(world.test_philox(ctr, key), oracle.philox(ctr, key))
    a = rng.integers(0, 2**32, size=1 << 20, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 2**32, size=1 << 20, dtype=np.uint64).astype(np.uint32)
    a[:256] = np.arange(256) << 8   # smallest and largest u1
    b[:256] = (np.arange(256) * 0x40000) & 0xFFFFFFFF
    g0, g1 = world.test_gauss(a, b)
    o0, o1 = oracle.gauss_pair(a, b)
    assert np.array_equal(g0.view(np.uint32), o0.view(np.uint32))
    assert np.array_equal(g1.view(np.uint32), o1.view(np.uint32))


def dense(workloads, **kw):
    d = dict(H=40, W=72, cap=300, n_init=200, obs_radius=2, hidden=16, res_init_p=0.4, rate_scale=5.0,
             T_repr=8, L_max=150)
    d.update(kw)
    return workloads.make(**d)


CASES = {
    "cfg0": lambda wl: (wl.WORKLOADS["cfg0"], 0, 1000, 100),
    "dense_h16_r2": lambda wl: (dense(wl), 1, 300, 50),
    "dense_h32_r3": lambda wl: (dense(wl, H=50, W=90, cap=400, n_init=300, obs_radius=3, hidden=32), 2, 150, 50),
    "dense_h16_r1": lambda wl: (dense(wl, obs_radius=1, H=33, W=17, cap=250, n_init=150), 3, 200, 40),
}


@pytest.mark.parametrize("case", list(CASES))
def test_parity_kernels(env, case):
    world, oracle, wl = env
    cfg, seed, steps, K = CASES[case](wl)
    say(f"[parity] {case} seed={seed} steps={steps} K={K}")
    st = run_parity(world.World, oracle.OracleWorld, oracle.OracleConfig, cfg, seed, steps, K,
                    theta_every=2)
    say(f"[parity] {case} ok {st}")
    assert st["agent_steps"] > 0


@pytest.mark.parametrize("mode", ["graph", "kernels"])
def test_parity_modes(env, mode):
    world, oracle, wl = env
    cfg, seed, steps, K = CASES["dense_h16_r2"](wl)
    say(f"[parity] mode={mode}")
    st = run_parity(world.World, oracle.OracleWorld, oracle.OracleConfig, cfg, seed, 200, K, mode=mode)
    say(f"[parity] mode={mode} ok {st}")
