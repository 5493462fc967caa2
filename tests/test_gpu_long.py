"""Oracle parity over every window the benchmark times, in the launch
configuration it times (captured graphs of K steps).  The device runs the
whole window; the oracle checks it segment by segment in worker processes
(tests/parity_util.py: every step's counters, acting agents and logits, and
at every segment boundary the complete state with every genome bit-exact).

Windows covered (steps from the seed):
* m1_4k 0..2199     the headline (1000 fixture steps, then warm-up and timed steps)
* cfg2 0..4999      the dense start beyond the last-level cache (steps 0..59)
                    and the whole 5000-step stress fixture
* cfg1 0..9999      the paper-scale fixture, 100 graphs of 100 steps
* net_m1_4k 0..799  the paper's network at ~4k agents (timed steps 300..799)
* paper1k 0..2999   the paper's world and dynamics (timed steps 1000..2999)
"""
import pytest

from parity_util import run_parity_segmented, say

pytestmark = pytest.mark.gpu

WINDOWS = {
    "m1_4k": (2200, 100, 200),
    "cfg2": (5000, 100, 500),
    "cfg1": (10000, 100, 1000),
    "net_m1_4k": (800, 100, 100),
    "paper1k": (3000, 100, 500),
}


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_09334_amd import workloads, world
    return world, workloads


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", list(WINDOWS))
def test_window(env, name):
    world, wl = env
    steps, K, seg = WINDOWS[name]
    cfg = wl.WORKLOADS[name]
    say(f"[long] {name} steps=0..{steps - 1} K={K} segment={seg}")
    gw = world.World(cfg, 0, mode="graph", log_steps=K)
    st = run_parity_segmented(gw, cfg, 0, steps, K, seg,
                              on_segment=lambda a, b: say(f"[long] {name} device steps {a}..{b - 1} queued"))
    gw.close()
    say(f"[long] {name} ok {st}")
    assert st["steps"] == steps and st["agent_steps"] > 0
