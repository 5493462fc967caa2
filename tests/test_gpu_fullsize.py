"""Full-size workloads against the oracle, in the launch configuration the
benchmark times (a captured graph of 100 steps for 200 x 400 with ~4.6k
agents); every step's counters and acting agents, logits within 1e-5, and the
complete state (including every genome) bit-exact at the end."""
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


@pytest.mark.parametrize("name,steps,K", [("m1_4k", 100, 100), ("cfg1", 40, 40), ("cfg2", 12, 12)])
def test_fullsize(env, name, steps, K):
    world, oracle, wl = env
    cfg = wl.WORKLOADS[name]
    say(f"[full] {name} steps={steps} K={K}")
    st = run_parity(world.World, oracle.OracleWorld, oracle.OracleConfig, cfg, 0, steps, K, mode="graph",
                    theta_every=1)
    say(f"[full] {name} ok {st}")
