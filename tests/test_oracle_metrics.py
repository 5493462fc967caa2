"""Pins of the oracle's ecology metrics (App. C): life expectancy (ages of the
agents that died) and the movement histogram over 50-step windows.

* Age at death: every step's sum recomputed from two consecutive canonical
  snapshots (the uids that disappeared, with their age before the step + 1),
  and the closed form of a well-fed world whose initial agents all die at
  exactly L_max.
* Movement: every window's histogram recomputed from the snapshots at the
  window's boundaries (agents present at both, matched by uid, Manhattan
  distance, bin = distance // 3); closed forms with forced actions: agents
  that always stay all land in bin 0, and a lone fed agent that always moves
  north travels exactly min(start row, 50).
"""
import numpy as np

BIG = 10**9
WIN = 50
BINS = 17


def dense_cfg(oracle_lib, **kw):
    d = dict(H=40, W=64, cap=600, n_init=300, obs_radius=2, hidden=16, res_init_p=0.4, rate_scale=5.0,
             T_repr=8, L_max=90)
    d.update(kw)
    return oracle_lib.OracleConfig(**d)


def by_uid(a):
    return {int(u): i for i, u in enumerate(a["uid"])}


def hist_from_snapshots(a0, a1):
    """Histogram of the agents present in both snapshots (matched by uid)."""
    i0, i1 = by_uid(a0), by_uid(a1)
    h = np.zeros(BINS + 1, np.int64)
    for u, j in i1.items():
        if u not in i0:
            continue
        i = i0[u]
        d = abs(int(a1["row"][j]) - int(a0["row"][i])) + abs(int(a1["col"][j]) - int(a0["col"][i]))
        assert 0 <= d <= WIN
        h[d // 3] += 1
        h[BINS] += 1
    return h


def test_dead_age_from_snapshots(oracle_lib):
    ow = oracle_lib.OracleWorld(dense_cfg(oracle_lib), 3)
    total_deaths = 0
    for _ in range(160):
        before = ow.agents()
        info = ow.step()
        after = ow.agents()
        alive_after = set(int(u) for u in after["uid"])
        gone = [i for i, u in enumerate(before["uid"]) if int(u) not in alive_after]
        assert info["deaths"] == len(gone)
        assert info["dead_age"] == sum(int(before["age"][i]) + 1 for i in gone)
        total_deaths += len(gone)
    assert total_deaths > 50   # the run exercised deaths


def test_dead_age_closed_form(oracle_lib):
    # every cell holds a resource and regrows at once; no births: the initial
    # agents eat every step and all die of age at step L_max - 1
    L = 30
    cfg = dense_cfg(oracle_lib, res_init_p=1.0, rate_top=1.0, rate_bottom=1.0, rate_scale=1.0, spont=1.0,
                    T_repr=BIG, L_max=L, n_init=120, cap=120)
    ow = oracle_lib.OracleWorld(cfg, 5)
    for s in range(L):
        info = ow.step()
        if s < L - 1:
            assert info["deaths"] == 0 and info["dead_age"] == 0, s
    assert info["deaths"] == 120 and info["dead_age"] == 120 * L
    assert ow.n_live == 0


def test_move_hist_from_snapshots(oracle_lib):
    ow = oracle_lib.OracleWorld(dense_cfg(oracle_lib), 7)
    snaps = {}
    for s in range(4 * WIN):
        if s % WIN == 0:
            snaps[s] = ow.agents()
        ow.step()
    snaps[4 * WIN] = ow.agents()
    hist = ow.move_hist()
    assert hist.shape == (4, BINS + 1)
    for k in range(4):
        ref = hist_from_snapshots(snaps[k * WIN], snaps[(k + 1) * WIN])
        assert np.array_equal(hist[k], ref), (k, hist[k], ref)
    assert hist[:, BINS].min() > 10
    assert (hist[:, 1:BINS].sum() > 0)   # agents moved


def test_move_hist_all_stay(oracle_lib):
    ow = oracle_lib.OracleWorld(dense_cfg(oracle_lib, L_max=BIG), 11)
    ow.set_forced(None, default=4)
    s0 = ow.agents()
    for _ in range(WIN):
        ow.step()
    h = ow.move_hist()[0]
    present = len(set(map(int, s0["uid"])) & set(map(int, ow.agents()["uid"])))
    assert h[0] == present and h[BINS] == present and h[1:BINS].sum() == 0


def test_move_hist_lone_agent_north(oracle_lib):
    for seed in range(6):
        cfg = dense_cfg(oracle_lib, H=120, W=30, n_init=1, cap=4, res_init_p=1.0, rate_top=1.0, rate_bottom=1.0,
                        rate_scale=1.0, spont=1.0, T_repr=BIG, L_max=BIG)
        ow = oracle_lib.OracleWorld(cfg, seed)
        ow.set_forced(None, default=0)   # always north (row - 1); the top edge stops it
        r0 = int(ow.agents()["row"][0])
        for _ in range(WIN):
            ow.step()
        h = ow.move_hist()[0]
        d = min(r0, WIN)
        assert h[BINS] == 1 and h[d // 3] == 1, (seed, r0, h)
        assert int(ow.agents()["row"][0]) == r0 - d


def window_sees(R, row, col, rho):
    H, W = R.shape
    r0, r1 = max(row - rho, 0), min(row + rho + 1, H)
    c0, c1 = max(col - rho, 0), min(col + rho + 1, W)
    return bool(R[r0:r1, c0:c1].any())


def test_seen_from_snapshots(oracle_lib):
    # agents with a resource in their field of view at the step start (the
    # greediness of the lab environments, Sec. 2.2), recomputed from the state
    for cfg in (dense_cfg(oracle_lib, res_init_p=0.05, rate_scale=0.5),
                dense_cfg(oracle_lib, res_init_p=0.02, rate_scale=0.2, obs_radius=7, hidden=4,
                          controller=oracle_lib.CTRL_CNN_LSTM)):
        ow = oracle_lib.OracleWorld(cfg, 5)
        partial = 0
        for _ in range(60):
            R = ow.grid()
            a = ow.agents()
            ref = sum(window_sees(R, int(r), int(c), cfg.obs_radius) for r, c in zip(a["row"], a["col"]))
            info = ow.step()
            assert info["seen"] == ref
            partial += 0 < ref < len(a["uid"])
        assert partial > 10   # the runs exercised both outcomes


def test_seen_closed_forms(oracle_lib):
    full = oracle_lib.OracleWorld(dense_cfg(oracle_lib, res_init_p=1.0, n_init=50), 1)
    assert full.step()["seen"] == 50
    bare = oracle_lib.OracleWorld(dense_cfg(oracle_lib, res_init_p=0.0, rate_top=0.0, rate_bottom=0.0, spont=0.0,
                                            n_init=50), 1)
    for _ in range(5):
        assert bare.step()["seen"] == 0


def test_load_resumes_exactly(oracle_lib):
    for cfg in (dense_cfg(oracle_lib),
                dense_cfg(oracle_lib, obs_radius=7, hidden=4, controller=oracle_lib.CTRL_CNN_LSTM)):
        a = oracle_lib.OracleWorld(cfg, 8)
        for _ in range(37):
            a.step()
        mid = a.state(with_hidden=True, with_theta=True)
        b = oracle_lib.OracleWorld(cfg, 8)
        b.step()   # any other state
        b.load(mid)
        for _ in range(40):
            ia, ib = a.step(), b.step()
            assert ia == ib
        sa, sb = a.state(with_hidden=True, with_theta=True), b.state(with_hidden=True, with_theta=True)
        for k in sa:
            assert np.array_equal(np.asarray(sa[k]), np.asarray(sb[k])), k
        # a window in progress at the load counts no agent
        assert b.move_hist().shape[0] == 1 and b.move_hist()[0, BINS] == 0
        assert a.move_hist()[-1, BINS] > 0
