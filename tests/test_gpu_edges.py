"""Edge cases against the oracle (bit-exact integer state every step)."""
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


def edge_cases(wl):
    m = wl.make
    return {
        # no agents: regrowth only
        "empty": (m(H=30, W=50, cap=64, n_init=0, obs_radius=2, hidden=16, res_init_p=0.02, rate_scale=8.0), 60, 20),
        # every slot used from the start: births only through deaths
        "full": (m(H=24, W=24, cap=200, n_init=200, obs_radius=2, hidden=16, res_init_p=0.5, rate_scale=5.0,
                   T_repr=5, L_max=60), 120, 30),
        # every cell occupied: no move can succeed, no child can be placed
        "packed": (m(H=6, W=7, cap=42, n_init=42, obs_radius=1, hidden=16, res_init_p=0.5, spont=0.3), 40, 10),
        # the smallest grid, a single slot
        "tiny": (m(H=2, W=1, cap=1, n_init=1, obs_radius=1, hidden=32, res_init_p=1.0, spont=1.0, T_repr=3,
                   L_max=30), 40, 7),
        # regrowth certain everywhere; the cap binds every step
        "saturated": (m(H=20, W=33, cap=90, n_init=30, obs_radius=3, hidden=32, res_init_p=1.0, spont=1.0,
                        T_repr=4, L_max=40), 120, 25),
        # a ragged world larger than several tiles, long-lived agents
        "ragged": (m(H=37, W=101, cap=700, n_init=350, obs_radius=3, hidden=16, res_init_p=0.3, rate_scale=4.0,
                     T_repr=10, L_max=500), 80, 40),
    }


@pytest.mark.parametrize("case", ["empty", "full", "packed", "tiny", "saturated", "ragged"])
def test_edge_parity(env, case):
    world, oracle, wl = env
    cfg, steps, K = edge_cases(wl)[case]
    say(f"[edge] {case}")
    st = run_parity(world.World, oracle.OracleWorld, oracle.OracleConfig, cfg, 5, steps, K, theta_every=1)
    say(f"[edge] {case} ok {st}")


@pytest.mark.parametrize("action", [0, 1, 2, 3, 4])
def test_forced_actions(env, action):
    """Everyone pushes the same way: maximal collisions at the boundary."""
    world, oracle, wl = env
    cfg = wl.make(H=16, W=20, cap=200, n_init=150, obs_radius=2, hidden=16, res_init_p=0.4, rate_scale=5.0,
                  T_repr=6, L_max=80)
    say(f"[edge] forced {action}")
    run_parity(world.World, oracle.OracleWorld, oracle.OracleConfig, cfg, 9, 60, 20, forced=action,
               theta_every=1)
