"""Pins of the oracle's agent dynamics (App. B.2, B.3 in the benchmark
parameterisation): moves and collisions, eating, energy, death, the minimal
criterion, births with mutation, and slot limits.

* Moves: every joint action of up to 4 agents on 3x3 / 4x4 grids against the
  rule restated as a greedy pass in priority order.
* Closed forms under forced actions: starvation at age E0/decay, death at
  exactly L_max when fed, first birth after exactly T_repr fed steps, a full
  world keeping its eligible parent's streak.
* Conservation with frozen dynamics, energy bookkeeping, invariants on dense
  random runs, and the mutation recomputed from the pinned primitives.
"""
import itertools

import numpy as np
import pytest
from scipy import stats

from oracle_ref import moves_by_priority

BIG = 10**9


def tiny_cfg(oracle_lib, **kw):
    d = dict(H=4, W=4, cap=8, n_init=3, obs_radius=1, hidden=16, res_init_p=0.0,
             rate_bottom=0.0, rate_top=0.0, spont=0.0, decay=0, gain=0,
             T_repr=BIG, L_max=BIG)
    d.update(kw)
    return oracle_lib.OracleConfig(**d)


@pytest.mark.parametrize("H,W,n,seed", [(3, 3, 3, 1), (3, 3, 4, 2), (4, 4, 4, 3), (4, 4, 2, 4),
                                        (3, 3, 2, 5), (2, 3, 4, 6)])
def test_moves_bruteforce(oracle_lib, H, W, n, seed):
    cfg = tiny_cfg(oracle_lib, H=H, W=W, n_init=n, cap=n)
    base = oracle_lib.OracleWorld(cfg, seed)
    s0 = base.agents()
    pos = [(int(r), int(c)) for r, c in zip(s0["row"], s0["col"])]
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = s0["uid"]
    ctr[:, 2] = 4  # MOVE stream, step 0
    draws = oracle_lib.philox(ctr, [seed, 0])[:, 0].astype(np.uint64)
    keys = (draws << np.uint64(32)) | s0["uid"].astype(np.uint64)
    for acts in itertools.product(range(5), repeat=n):
        w = oracle_lib.OracleWorld(cfg, seed)
        w.set_forced(np.array(acts, np.int32))
        w.step()
        s = w.agents()
        got = [(int(r), int(c)) for r, c in zip(s["row"], s["col"])]
        assert got == moves_by_priority(H, W, pos, acts, keys), acts
        assert len(set(got)) == n
        for (r0, c0), (r1, c1) in zip(pos, got):
            assert abs(r1 - r0) + abs(c1 - c0) <= 1


def test_starvation_age(oracle_lib):
    cfg = tiny_cfg(oracle_lib, H=5, W=5, n_init=1, cap=1, decay=1, E0=50)
    w = oracle_lib.OracleWorld(cfg, 0)
    w.set_forced(None, default=4)
    for t in range(49):
        w.step()
    a = w.agents()
    assert w.n_live == 1 and a["energy"][0] == 1 and a["age"][0] == 49
    info = w.step()
    assert w.n_live == 0 and info["deaths"] == 1


def test_fed_agent_reaches_lmax(oracle_lib):
    cfg = tiny_cfg(oracle_lib, H=5, W=5, n_init=1, cap=1, decay=1, gain=10, res_init_p=1.0,
                   spont=1.0, L_max=2000)
    w = oracle_lib.OracleWorld(cfg, 0)
    w.set_forced(None, default=4)
    for t in range(1999):
        info = w.step()
        assert info["eaten"] == 1
    a = w.agents()
    assert a["age"][0] == 1999 and a["energy"][0] == 50 + 9 * 1999
    info = w.step()
    assert w.n_live == 0 and info["deaths"] == 1


def test_first_birth_after_t_repr(oracle_lib):
    cfg = tiny_cfg(oracle_lib, H=7, W=7, n_init=1, cap=10, decay=1, gain=10, res_init_p=1.0,
                   spont=1.0, E_repr=40, T_repr=20)
    w = oracle_lib.OracleWorld(cfg, 5)
    w.set_forced(None, default=4)
    for t in range(19):
        info = w.step()
        assert info["births"] == 0
    p = w.agents()
    assert p["streak"][0] == 19
    info = w.step()
    assert info["births"] == 1
    a = w.agents()
    assert list(a["uid"]) == [0, 1]
    assert abs(a["row"][1] - a["row"][0]) + abs(a["col"][1] - a["col"][0]) == 1
    assert a["energy"][1] == 50 and a["age"][1] == 0 and a["streak"][1] == 0
    assert a["streak"][0] == 0
    assert not w.hidden()[1].any()
    assert w.next_uid == 2


def test_streak_counts_energy_at_the_threshold(oracle_lib):
    """The minimal criterion counts steps with energy at or above E_repr: an
    agent held exactly at E_repr has its first child after T_repr steps, one
    held a unit below never has one."""
    for e0, first in ((40, 4), (39, None)):
        cfg = tiny_cfg(oracle_lib, H=7, W=7, n_init=1, cap=4, E0=e0, E_repr=40, T_repr=5)
        w = oracle_lib.OracleWorld(cfg, 2)
        w.set_forced(None, default=4)
        births = [w.step()["births"] for _ in range(12)]
        assert w.agents()["energy"][0] == e0
        if first is None:
            assert not any(births)
        else:
            assert births.index(1) == first and not any(births[:first])


@pytest.mark.parametrize("seed", [0, 11, 2**33 + 7])
def test_initial_world_recomputed(oracle_lib, seed):
    """The initial world from the pinned generator (streams as the simulator
    numbers them: 1 initial resources, 2 placement): cell i holds a resource iff
    its stream-1 word is below floor(p 2^32); the agents take the n_init cells of
    smallest (stream-2 word, cell index), uids in that order."""
    from oracle_ref import exact_threshold
    H, W, n = 9, 13, 20
    cfg = tiny_cfg(oracle_lib, H=H, W=W, n_init=n, cap=n, res_init_p=0.3)
    w = oracle_lib.OracleWorld(cfg, seed)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    ctr = np.zeros((H * W, 4), np.uint32)
    ctr[:, 0] = np.arange(H * W)
    ctr[:, 2] = 1
    res = oracle_lib.philox(ctr, key)[:, 0]
    thr = exact_threshold(dict(rate_bottom=0.0, rate_top=0.0, rate_scale=1.0, spont=0.3, H=2), 0, 0)
    assert np.array_equal(w.grid().ravel(), (res.astype(np.uint64) < thr).astype(np.uint8))
    ctr[:, 2] = 2
    place = oracle_lib.philox(ctr, key)[:, 0]
    order = sorted(range(H * W), key=lambda i: (int(place[i]), i))[:n]
    a = w.agents()
    assert list(a["uid"]) == list(range(n))
    assert [int(r) * W + int(c) for r, c in zip(a["row"], a["col"])] == order


def test_birth_claim_resolution(oracle_lib):
    """Two eligible parents whose only free neighbour is the same cell: the
    smaller (second word of the birth draw, uid) wins it (birth draw = stream 5
    of the pinned generator at counter (uid, step, 5, 0)); the other keeps its
    streak."""
    wins = set()
    for seed in range(30):
        cfg = tiny_cfg(oracle_lib, H=3, W=3, n_init=8, cap=9, E_repr=40, T_repr=1)
        w = oracle_lib.OracleWorld(cfg, seed)
        w.set_forced(None, default=4)
        s = w.state(with_hidden=True, with_theta=True)
        cells = [(1, 0), (1, 2), (0, 0), (0, 1), (0, 2), (2, 0), (2, 1), (2, 2)]   # parents first
        s["row"] = np.array([r for r, _ in cells], np.int32)
        s["col"] = np.array([c for _, c in cells], np.int32)
        s["energy"] = np.array([50, 50] + [10] * 6, np.int32)
        s["streak"] = np.zeros(8, np.int32)
        w.load(s)
        info = w.step()
        ctr = np.array([[0, 0, 5, 0], [1, 0, 5, 0]], np.uint32)
        words = oracle_lib.philox(ctr, [seed, 0])[:, 1]
        winner = int(np.argmin([(int(words[u]) << 32) | u for u in range(2)]))
        wins.add(winner)
        a = w.agents()
        assert info["births"] == 1 and info["claim_wins"] == 1
        assert (int(a["row"][8]), int(a["col"][8])) == (1, 1)
        assert a["streak"][winner] == 0 and a["streak"][1 - winner] == 1
        w.close()
    assert wins == {0, 1}


def test_child_direction_uniform(oracle_lib):
    """A lone interior parent's child lands on each of its four neighbours
    equally often over seeds (the start of the neighbour scan is random)."""
    counts = {(-1, 0): 0, (1, 0): 0, (0, 1): 0, (0, -1): 0}
    for seed in range(800):
        cfg = tiny_cfg(oracle_lib, H=9, W=9, n_init=1, cap=2, E_repr=0, T_repr=1)
        w = oracle_lib.OracleWorld(cfg, seed)
        w.set_forced(None, default=4)
        p = w.agents()
        info = w.step()
        assert info["births"] == 1
        if 1 <= p["row"][0] <= 7 and 1 <= p["col"][0] <= 7:
            a = w.agents()
            counts[(int(a["row"][1] - a["row"][0]), int(a["col"][1] - a["col"][0]))] += 1
        w.close()
    obs = np.array(list(counts.values()))
    assert obs.sum() > 400
    assert stats.chisquare(obs).pvalue > 1e-4, counts


@pytest.mark.parametrize("free", range(4))
def test_child_takes_the_only_free_neighbour(oracle_lib, free):
    """Three neighbours held by agents that cannot reproduce (energy below
    E_repr): over many seeds the child always takes the fourth."""
    nbr = [(-1, 0), (1, 0), (0, 1), (0, -1)]
    for seed in range(40):
        cfg = tiny_cfg(oracle_lib, H=5, W=5, n_init=4, cap=5, E_repr=40, T_repr=1)
        w = oracle_lib.OracleWorld(cfg, seed)
        w.set_forced(None, default=4)
        s = w.state(with_hidden=True, with_theta=True)
        rows, cols = [2], [2]
        for k, (dr, dc) in enumerate(nbr):
            if k != free:
                rows.append(2 + dr)
                cols.append(2 + dc)
        s["row"] = np.array(rows, np.int32)
        s["col"] = np.array(cols, np.int32)
        s["energy"] = np.array([50, 10, 10, 10], np.int32)
        s["streak"] = np.zeros(4, np.int32)
        w.load(s)
        info = w.step()
        assert info["births"] == 1 and info["deaths"] == 0
        a = w.agents()
        assert (int(a["row"][4]), int(a["col"][4])) == (2 + nbr[free][0], 2 + nbr[free][1]), seed
        w.close()


def test_full_world_keeps_streak(oracle_lib):
    cfg = tiny_cfg(oracle_lib, H=5, W=5, n_init=1, cap=1, decay=1, gain=10, res_init_p=1.0,
                   spont=1.0, E_repr=40, T_repr=20)
    w = oracle_lib.OracleWorld(cfg, 5)
    w.set_forced(None, default=4)
    for t in range(30):
        info = w.step()
        assert info["births"] == 0 and w.n_live == 1
    assert w.agents()["streak"][0] == 30
    # with no free slot no birth claim is resolved or counted
    assert info["claim_wins"] == 0


def test_frozen_dynamics_conserve(oracle_lib):
    cfg = tiny_cfg(oracle_lib, H=24, W=30, n_init=60, cap=80, obs_radius=2, res_init_p=0.3)
    w = oracle_lib.OracleWorld(cfg, 3)
    r0 = int(w.grid().sum())
    a0 = w.agents()
    eaten = 0
    for t in range(40):
        info = w.step()
        eaten += info["eaten"]
        a = w.agents()
        assert w.n_live == 60 and np.array_equal(a["uid"], a0["uid"])
        assert (a["energy"] == 50).all()
        assert int(w.grid().sum()) == r0 - eaten == info["resources"]
        assert len(set(zip(a["row"], a["col"]))) == 60


def test_energy_bookkeeping(oracle_lib):
    cfg = tiny_cfg(oracle_lib, H=20, W=20, n_init=50, cap=60, obs_radius=2, res_init_p=0.4,
                   rate_bottom=0.2, rate_top=0.1, E0=10**6, decay=1, gain=10)
    w = oracle_lib.OracleWorld(cfg, 8)
    for t in range(30):
        e0 = int(w.agents()["energy"].astype(np.int64).sum())
        info = w.step()
        e1 = int(w.agents()["energy"].astype(np.int64).sum())
        assert e1 == e0 + 10 * info["eaten"] - 50


def dense_cfg(oracle_lib, **kw):
    d = dict(H=24, W=40, cap=200, n_init=150, obs_radius=2, hidden=16, res_init_p=0.4,
             rate_scale=5.0, T_repr=8, L_max=120)
    d.update(kw)
    return oracle_lib.OracleConfig(**d)


def test_invariants_dense(oracle_lib):
    cfg = dense_cfg(oracle_lib)
    w = oracle_lib.OracleWorld(cfg, 21)
    prev = w.agents()
    births = deaths = 0
    for t in range(150):
        nu = w.next_uid
        info = w.step()
        a = w.agents()
        births += info["births"]
        deaths += info["deaths"]
        assert w.n_live == len(a["uid"]) <= cfg.cap
        assert (np.diff(a["uid"].astype(np.int64)) > 0).all()
        assert ((a["row"] >= 0) & (a["row"] < cfg.H) & (a["col"] >= 0) & (a["col"] < cfg.W)).all()
        assert len(set(zip(a["row"], a["col"]))) == w.n_live
        old = dict(zip(prev["uid"], zip(prev["row"], prev["col"])))
        born = a["uid"] >= nu
        assert born.sum() == info["births"] and w.next_uid == nu + info["births"]
        assert (a["energy"][born] == cfg.E0).all() and (a["age"][born] == 0).all()
        for u, r, c in zip(a["uid"][~born], a["row"][~born], a["col"][~born]):
            r0, c0 = old[u]
            assert abs(r - r0) + abs(c - c0) <= 1
        assert len(prev["uid"]) - info["deaths"] + info["births"] == w.n_live
        prev = a
    assert births > 50 and deaths > 50


@pytest.mark.parametrize("sigma", [0.0, 0.02])
def test_mutation(oracle_lib, sigma):
    cfg = dense_cfg(oracle_lib, sigma_mut=sigma, cap=400, n_init=100)
    seed = 77
    w = oracle_lib.OracleWorld(cfg, seed)
    checked = 0
    deltas = []
    for t in range(60):
        th_prev = w.theta()
        uid_prev = w.agents()["uid"]
        nu = w.next_uid
        info = w.step()
        if not info["births"]:
            continue
        a = w.agents()
        th = w.theta()
        pos = {u: (r, c) for u, r, c in zip(a["uid"], a["row"], a["col"])}
        prev_idx = {u: i for i, u in enumerate(uid_prev)}
        for ci in np.nonzero(a["uid"] >= nu)[0]:
            cu = int(a["uid"][ci])
            r, c = pos[cu]
            cands = [u for u, (pr, pc) in pos.items() if u < nu and abs(pr - r) + abs(pc - c) == 1]
            P = th.shape[1]
            blocks = (P + 3) // 4
            ctr = np.zeros((blocks, 4), np.uint32)
            ctr[:, 0] = cu
            ctr[:, 1] = t
            ctr[:, 2] = 6
            ctr[:, 3] = np.arange(blocks)
            rr = oracle_lib.philox(ctr, [seed, 0])
            z0, z1 = oracle_lib.gauss_pair(rr[:, 0], rr[:, 1])
            z2, z3 = oracle_lib.gauss_pair(rr[:, 2], rr[:, 3])
            z = np.stack([z0, z1, z2, z3], 1).ravel()[:P].astype(np.float64)
            matches = []
            for u in cands:
                tp = th_prev[prev_idx[u]]
                ref = (np.float64(np.float32(sigma)) * z + tp.astype(np.float64)).astype(np.float32)
                ulp = np.spacing(np.abs(ref))
                if (np.abs(th[ci] - ref) <= ulp).all() and (th[ci] == ref).mean() > 0.999:
                    matches.append(u)
                    if sigma:
                        deltas.append((th[ci].astype(np.float64) - tp) / sigma)
            # exactly one adjacent agent is the parent (with sigma = 0 a
            # sibling's identical copy may match too)
            assert len(matches) >= 1 if sigma == 0.0 else len(matches) == 1
            checked += 1
    assert checked >= 5
    if deltas:
        d = np.concatenate(deltas)
        assert stats.kstest(d, "norm").pvalue > 1e-3
