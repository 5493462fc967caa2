"""Lab environments (Sec. 2.2) on the GPU: evolved agents from a natural run of
the paper's network placed alone in lab worlds, all conditions stepped in one
batch; every world of one agent (and a peer-pressure world of another) against
the oracle from the same starting state, bit-exact every step (resources seen,
eaten, births included); a lab world stepped alone equals its batched result;
the greediness and peer-pressure studies run on the counters."""
import numpy as np
import pytest

from parity_util import compare_state, say
from test_gpu_systems import same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_2302_09334_amd import lab, workloads, world
    return world, oracle, workloads, lab


def test_lab_batch_parity(env):
    world, oracle, wl, lab = env
    base = wl.make(H=40, W=72, cap=300, n_init=200, obs_radius=7, hidden=4, res_init_p=0.4, rate_scale=5.0,
                   T_repr=8, L_max=300, w_init_gain=1.0, controller=1)
    steps = 200
    say("[lab] evolving 300 steps")
    snap = lab.evolve(base, 3, 300)
    genomes = lab.sample_agents(snap, 3, seed=0)
    run = lab.LabRun(genomes, base, lab.conditions(), trials=2, log_steps=steps)
    say(f"[lab] {len(run.worlds)} lab worlds, {steps} steps in one batch")
    run.step(steps)
    run.sync()
    ctrs = run.counters(steps)
    checked = 0
    keys = ("n_live", "births", "deaths", "eaten", "resources", "claim_wins", "dead_age", "seen")
    for i, (key, w) in enumerate(zip(run.keys, run.worlds)):
        if key[0] != 0 and key != (1, "high_repro", 0):
            continue
        ow = oracle.OracleWorld(oracle.OracleConfig.from_dict(run.cfgs[i]), run.seeds[i])
        ow.load(run.images[i])
        for s in range(steps):
            log = w.action_log(s)
            info = ow.step(log["uid"], log["action"])
            assert info["mismatches"] == 0, (key, s)
            for k in keys:
                assert ctrs[i][k][s] == info[k], (key, s, k)
        compare_state(w.snapshot(hidden=True, theta=True), ow.state(with_hidden=True, with_theta=True),
                      f"lab {key}", theta=True)
        checked += 1
    assert checked >= 9
    # one lab world stepped alone equals its batched result
    k = run.keys.index((1, "high_repro", 1))
    alone = world.World(run.cfgs[k], run.seeds[k])
    alone.load(run.images[k])
    alone.step(steps)
    same(alone.snapshot(hidden=True, theta=True), run.worlds[k].snapshot(hidden=True, theta=True), "alone")
    alone.close()
    g = lab.greediness_study(run, ctrs, len(genomes))
    p = lab.peer_pressure_study(run, ctrs)
    say(f"[lab] G by density {g['G_mean_by_density']}, sustainable {g['sustainable_foragers']}; "
        f"E off {p['E_mean_off']:.2f} on {p['E_mean_on']:.2f}")
    assert sum(c["births"].sum() for key, c in zip(run.keys, ctrs) if key[1] != "high_repro") == 0
    run.close()
