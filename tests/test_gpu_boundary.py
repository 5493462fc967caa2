"""The boundary's test hooks and counters against the oracle and against
recomputation from the state (through the C-ABI):

* a scripted walk: a forced action per agent (by uid), changed mid-run,
  with the controller deciding for every uid outside the script -- the GPU
  and the oracle under the same script agree step by step;
* the action log's top-2 margin equals the margin of the logged logits
  (GRU) or of the sampling scores the oracle computes from them (the paper's
  network);
* the per-step count of input rows the act phase read equals the count
  recomputed from each step's start state;
* the full integer state of cfg0 compared with the oracle after every step;
* world_step_many refuses a world listed twice; destroying a world releases
  the batches that list it.
"""
import numpy as np
import pytest

from parity_util import check_chunk, compare_state, new_stats, run_parity, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_2302_09334_amd import workloads, world
    return world, oracle, workloads


def dense(wl, **kw):
    d = dict(H=40, W=72, cap=300, n_init=200, obs_radius=3, hidden=32, res_init_p=0.4, rate_scale=5.0,
             T_repr=8, L_max=150)
    d.update(kw)
    return wl.make(**d)


@pytest.mark.parametrize("ctrl", ["gru", "net"])
def test_scripted_walk(env, ctrl):
    world, oracle, wl = env
    cfg = dense(wl) if ctrl == "gru" else dense(wl, obs_radius=7, hidden=4, controller=1, w_init_gain=1.0)
    rng = np.random.default_rng(5)
    K = 25
    gw = world.World(cfg, 21, log_steps=K)
    ow = oracle.OracleWorld(oracle.OracleConfig.from_dict(cfg), 21)
    stats = new_stats()
    t = 0
    for phase in range(4):
        # uids below n_script follow the script (-1 = the controller decides
        # for this uid); the rest (later children) follow `default`
        n_script = int(cfg["n_init"]) + 40 * phase
        table = rng.integers(-1, 5, n_script).astype(np.int32)
        default = [-1, 4, -1, 1][phase]
        gw.set_forced_actions(table, default)
        ow.set_forced(table, default=default)
        say(f"[boundary] {ctrl} script phase {phase}: {n_script} uids, default {default}")
        for _ in range(2):
            gw.step(K)
            gw.sync()
            check_chunk(gw, ow, t, K, stats)
            t += K
            compare_state(gw.snapshot(hidden=True, theta=True), ow.state(with_hidden=True, with_theta=True),
                          f"t={t}", theta=True)
            # every scripted agent took its scripted action
            log = gw.action_log(t - 1)
            u = log["uid"]
            inside = u < n_script
            entry = table[np.minimum(u, n_script - 1)]
            want = np.where(inside & (entry >= 0), entry, default)
            forced = want >= 0
            assert np.array_equal(log["action"][forced], want[forced]), ("scripted actions", t - 1)
    gw.set_forced_actions(None, -1)
    ow.set_forced(None, default=-1)
    gw.step(K)
    gw.sync()
    check_chunk(gw, ow, t, K, stats)
    say(f"[boundary] {ctrl} scripted walk ok {stats}")
    assert stats["births"] > 0 and stats["deaths"] > 0
    gw.close()
    ow.close()


@pytest.mark.parametrize("ctrl", ["gru", "net"])
def test_action_log_margin(env, ctrl):
    world, oracle, wl = env
    cfg = dense(wl) if ctrl == "gru" else dense(wl, obs_radius=7, hidden=4, controller=1, w_init_gain=1.0)
    gw = world.World(cfg, 3, log_steps=10)
    gw.step(10)
    gw.sync()
    checked = 0
    for t in range(10):
        log = gw.action_log(t)
        for i in range(len(log["uid"])):
            lg = log["logits"][i]
            if ctrl == "gru":
                sc = lg
            else:
                _, sc = oracle.sample_action(3, int(log["uid"][i]), t, lg)
            order = np.argsort(-sc, kind="stable")
            want = np.float32(sc[order[0]]) - np.float32(sc[order[1]])
            assert log["margin"][i] == want, (t, i, log["margin"][i], want)
            assert log["margin"][i] >= 0
            checked += 1
    gw.close()
    say(f"[boundary] {ctrl} margins checked: {checked}")
    assert checked > 100


def rows_read_from_state(s, cfg):
    """Input rows the act phase reads for the state at a step start: per
    binary window the rows of its ones, or its total and the rows of its zeros
    when ones are the majority (outside cells: no resource, occupied)."""
    H, W, rho = cfg["H"], cfg["W"], cfg["obs_radius"]
    w2 = (2 * rho + 1) ** 2
    R = np.zeros((H + 2 * rho, W + 2 * rho), np.int64)
    R[rho:rho + H, rho:rho + W] = s["R"]
    O = np.ones((H + 2 * rho, W + 2 * rho), np.int64)
    O[rho:rho + H, rho:rho + W] = 0
    O[s["row"] + rho, s["col"] + rho] = 1
    total = 0
    for grid in (R, O):
        m = np.zeros(s["n_live"], np.int64)
        for dy in range(-rho, rho + 1):
            for dx in range(-rho, rho + 1):
                m += grid[s["row"] + rho + dy, s["col"] + rho + dx]
        total += int(np.where(2 * m > w2, w2 - m + 1, m).sum())
    return total


@pytest.mark.parametrize("rho,hidden", [(3, 32), (2, 16), (1, 16)])
def test_rows_read_counter(env, rho, hidden):
    world, oracle, wl = env
    cfg = dense(wl, obs_radius=rho, hidden=hidden)
    gw = world.World(cfg, 8)
    for t in range(60):
        s = gw.snapshot()
        want = rows_read_from_state(s, cfg)
        gw.step(1)
        got = int(gw.counters(t, 1)["rows_read"][0])
        assert got == want, (t, got, want)
    gw.close()


def test_cfg0_state_every_step(env):
    world, oracle, wl = env
    say("[boundary] cfg0 1000 steps, full state after every step")
    st = run_parity(world.World, oracle.OracleWorld, oracle.OracleConfig, wl.WORKLOADS["cfg0"], 0, 1000, 1,
                    theta_every=50)
    say(f"[boundary] cfg0 every step ok {st}")
    assert st["agent_steps"] > 0


def test_step_many_duplicates_and_destroy(env):
    world, oracle, wl = env
    import torch
    s = torch.cuda.Stream()
    a = world.World(dense(wl), 1, stream=s)
    b = world.World(dense(wl, H=30), 2, stream=s)
    with pytest.raises(world.WorldError) as ei:
        world.step_many([a, b, a], 1)
    assert ei.value.code == -1
    world.step_many([a, b], 5)
    a.sync()
    ref = b.snapshot(hidden=True, theta=True)
    a.close()   # releases the batch [a, b]
    c = world.World(dense(wl), 1, stream=s)
    world.step_many([b, c], 5)
    b.sync()
    # b continued from ref: the same as stepping it alone from ref
    d = world.World(dense(wl, H=30), 2, stream=s)
    d.load(ref)
    d.step(5)
    sb, sd = b.snapshot(hidden=True, theta=True), d.snapshot(hidden=True, theta=True)
    for k in ("uid", "row", "col", "energy", "age", "streak", "R"):
        assert np.array_equal(sb[k], sd[k]), k
    assert np.array_equal(sb["theta"].view(np.uint32), sd["theta"].view(np.uint32))
    for w in (b, c, d):
        w.close()
