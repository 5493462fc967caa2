"""The largest worlds the library accepts, on the GPU against the oracle:
2^20 agent slots (the limit of world_config.cap) on a 1024 x 1024 grid, half
full at the start, with births from the third step and the whole first
generation dying at age 6; and a 2^26-cell grid (8192 x 8192, the grid's
limit) with 1000 agents.  Each world is stepped on the GPU (a graph of 7
steps) and checked by its counters' invariants; then the oracle is started
from the GPU's complete image and both take one more step: acting uids,
logits and counters of that step, and the complete next state (genomes
included), must agree.  The movement windows are not compared (a world
loaded mid-window counts no agent in it, R22)."""
import numpy as np
import pytest

from parity_util import check_chunk, compare_state, new_stats, say

pytestmark = pytest.mark.gpu

CASES = {
    "cap_2^20": (dict(H=1024, W=1024, cap=1 << 20, n_init=1 << 19, obs_radius=1, hidden=16, res_init_p=0.3,
                      rate_scale=4.0, T_repr=3, L_max=6), 7),
    "grid_2^26": (dict(H=8192, W=8192, cap=4096, n_init=1000, obs_radius=2, hidden=16, res_init_p=0.05,
                       T_repr=3, L_max=6), 7),
}


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_2302_09334_amd import workloads, world
    return world, oracle, workloads


@pytest.mark.timeout(900)
@pytest.mark.parametrize("case", list(CASES))
def test_largest_world(env, case):
    world, oracle, wl = env
    kw, steps = CASES[case]
    cfg = wl.make(**kw)
    say(f"[limits] {case}: {kw}, {world.required_bytes(cfg) / 1e9:.2f} GB on the device")
    g = world.World(cfg, 7, mode="graph", log_steps=1)
    g.step(steps)
    g.sync()
    ctr = g.counters(0, steps)
    n = kw["n_init"]
    for s in range(steps):
        n += int(ctr["births"][s]) - int(ctr["deaths"][s])
        assert int(ctr["n_live"][s]) == n and 0 <= n <= kw["cap"], (s, int(ctr["n_live"][s]), n)
    assert ctr["births"].sum() > 0 and ctr["deaths"].sum() > 0
    say(f"[limits] {case}: {steps} steps, n_live {n}, births {int(ctr['births'].sum())}, "
        f"deaths {int(ctr['deaths'].sum())}")
    img = g.snapshot(hidden=True, theta=True)
    o = oracle.OracleWorld(oracle.OracleConfig.from_dict(dict(cfg, n_init=0)), 7)
    o.load(img)
    del img
    g.step(1)
    g.sync()
    stats = new_stats()
    check_chunk(g, o, steps, 1, stats)
    compare_state(g.snapshot(hidden=True, theta=True), o.state(with_hidden=True, with_theta=True),
                  f"{case} t={steps + 1}", theta=True)
    say(f"[limits] {case}: step {steps} equal to the oracle's ({stats['agent_steps']} agents, "
        f"max logit error {stats['max_logit_err']:.2e}, {stats['resyncs']} near-tie resyncs)")
    g.close()
    o.close()
