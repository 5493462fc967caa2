"""Pins of the oracle's paper dynamics (App. B; the rules the benchmark
workloads replace): regrowth from the four direct neighbours and the climate
c(x), energy clipped at E_max, reproduction after T_repr steps above E_repr
with the offspring on the parent's cell, death after T_death steps below it,
past L_max or at a wall, stacking, one eater per resource.

Every check uses a closed form, the pinned primitives (Philox) or a
recomputation from snapshots; none re-types the oracle's formulas.
"""
import math

import numpy as np

BIG = 1 << 30


def paper_cfg(oracle_lib, **kw):
    d = dict(H=40, W=64, cap=600, n_init=200, obs_radius=2, hidden=16, res_init_p=0.2,
             E0=120, E_max=120, decay=1, gain=40, E_repr=0, T_repr=140, T_death=200, L_max=650,
             spont=5e-5, regrow_pI=0.002, regrow_alpha=200.0, dynamics=oracle_lib.DYN_PAPER)
    d.update(kw)
    return oracle_lib.OracleConfig(**d)


def image(ow, R, agents, genome=None):
    """A canonical image with the given grid and agents [(row, col), ...]."""
    n = len(agents)
    st = ow.state(with_hidden=True, with_theta=True)
    th = st["theta"][:1] if len(st["theta"]) else np.zeros((1, ow.P), np.float32)
    return dict(t=0, n_live=n, next_uid=n, R=np.asarray(R, np.uint8),
                uid=np.arange(n, dtype=np.uint32), row=np.array([a[0] for a in agents], np.int32),
                col=np.array([a[1] for a in agents], np.int32), energy=np.full(n, ow.cfg.E0, np.int32),
                age=np.zeros(n, np.int32), streak=np.zeros(n, np.int32),
                h=np.zeros((n, ow.cfg.state_size), np.float32), theta=np.repeat(th, n, axis=0),
                last_action=np.full(n, 5, np.uint8), ate=np.zeros(n, np.uint8))


def test_regrowth_exactly_one_neighbour(oracle_lib):
    # p = p_I * c(x) + c with c(bottom row) = 1: at p_I = 1, c = 0 exactly the
    # empty cells of the bottom row with exactly one resource neighbour grow
    cfg = paper_cfg(oracle_lib, H=6, W=12, n_init=0, cap=4, regrow_pI=1.0, spont=0.0)
    ow = oracle_lib.OracleWorld(cfg, 1)
    rng = np.random.default_rng(0)
    for trial in range(20):
        R = (rng.random((6, 12)) < 0.3).astype(np.uint8)
        ow.load(image(ow, R, []))
        ow.step()
        R1 = ow.grid()
        for r in range(6):
            for c in range(12):
                if R[r, c]:
                    assert R1[r, c] == 1
                    continue
                n = sum(R[r + dr, c + dc] for dr, dc in ((-1, 0), (1, 0), (0, 1), (0, -1))
                        if 0 <= r + dr < 6 and 0 <= c + dc < 12)
                want = 1 if (r == 5 and n == 1) else 0
                if r < 5:   # c(x) < 1: random; only bounded checks
                    assert R1[r, c] in (0, 1) and (n == 1 or R1[r, c] == 0)
                else:
                    assert R1[r, c] == want, (trial, r, c, n)


def test_regrowth_frequencies_follow_the_climate(oracle_lib):
    # p_I = 0.9, c = 0.02 on 5 rows: x = row / 4, climate (200^x + 1) / 201
    H, W = 5, 61   # resource columns 0, 3, ..., 60: every empty cell has exactly one beside it
    cfg = paper_cfg(oracle_lib, H=H, W=W, n_init=0, cap=4, regrow_pI=0.9, spont=0.02)
    ow = oracle_lib.OracleWorld(cfg, 2)
    # resources on every third column: empty cells beside them have exactly
    # one resource neighbour (class 1), the others none (class 0)
    R = np.zeros((H, W), np.uint8)
    R[:, ::3] = 1
    grow = np.zeros((H, 2))
    tries = np.zeros((H, 2))
    for s in range(300):
        ow = oracle_lib.OracleWorld(cfg, 100 + s)
        ow.load(image(ow, R, []))
        ow.step()
        R1 = ow.grid()
        for c in range(W):
            if c % 3 == 0:
                continue
            cls = 1   # every empty cell touches exactly one resource column here
            for r in range(H):
                tries[r, cls] += 1
                grow[r, cls] += R1[r, c]
    for r in range(H):
        x = r / (H - 1)
        p = 0.9 * (200 ** x + 1) / 201 + 0.02
        n = tries[r, 1]
        assert abs(grow[r, 1] - n * p) < 5 * math.sqrt(n * p * (1 - p)) + 1, (r, grow[r, 1] / n, p)
    # the top row has the lowest and the bottom row the highest climate
    f = grow[:, 1] / tries[:, 1]
    assert all(np.diff(f) > 0)


def run_alone(oracle_lib, steps, R, pos=(10, 10), forced=4, **kw):
    cfg = paper_cfg(oracle_lib, H=20, W=20, n_init=0, cap=8, **kw)
    ow = oracle_lib.OracleWorld(cfg, 3)
    ow.load(image(ow, R, [pos]))
    ow.set_forced(None, default=forced)
    infos = [ow.step() for _ in range(steps)]
    return ow, infos


def test_fed_agent_energy_clip_and_first_birth(oracle_lib):
    # every empty cell regrows every step: a staying agent eats every step,
    # its energy stays clipped at E_max, its streak grows by one per step and
    # it has exactly one child on its own cell after T_repr steps
    full = np.ones((20, 20), np.uint8)
    ow, infos = run_alone(oracle_lib, 141, full, spont=1.0, regrow_pI=0.0)
    births = [i for i, x in enumerate(infos) if x["births"]]
    assert births[0] == 139 and infos[139]["births"] == 1   # 140th step
    a = ow.agents()
    assert list(a["uid"]) == [0, 1]
    assert (a["row"][1], a["col"][1]) == (10, 10)            # the parent's cell
    # parent and child share the cell's one resource in the next step: one of
    # them eats (back at the clip), the other loses the decay
    assert sorted(a["energy"]) == [119, 120]
    assert a["streak"][0] == 1                               # restarted at the birth


def test_starving_agent_dies_after_T_death_below(oracle_lib):
    # no resources, no regrowth: e = 120 - t; below E_repr = 0 from t = 121;
    # death when 200 steps below have passed: at step 320
    ow, infos = run_alone(oracle_lib, 330, np.zeros((20, 20), np.uint8), spont=0.0, regrow_pI=0.0)
    deaths = [i for i, x in enumerate(infos) if x["deaths"]]
    assert deaths == [319] and infos[319]["dead_age"] == 320
    assert sum(x["births"] for x in infos) == 0


def test_age_limit(oracle_lib):
    full = np.ones((20, 20), np.uint8)
    ow, infos = run_alone(oracle_lib, 660, full, spont=1.0, regrow_pI=0.0, T_repr=BIG, L_max=650)
    deaths = [i for i, x in enumerate(infos) if x["deaths"]]
    assert deaths == [650] and infos[650]["dead_age"] == 651   # age > L_max


def test_wall_kills(oracle_lib):
    ow, infos = run_alone(oracle_lib, 1, np.zeros((20, 20), np.uint8), pos=(0, 5), forced=0)
    assert infos[0]["deaths"] == 1 and ow.n_live == 0
    ow, infos = run_alone(oracle_lib, 1, np.zeros((20, 20), np.uint8), pos=(19, 5), forced=1)
    assert infos[0]["deaths"] == 1
    ow, infos = run_alone(oracle_lib, 1, np.zeros((20, 20), np.uint8), pos=(5, 19), forced=2)
    assert infos[0]["deaths"] == 1
    ow, infos = run_alone(oracle_lib, 1, np.zeros((20, 20), np.uint8), pos=(5, 0), forced=3)
    assert infos[0]["deaths"] == 1
    ow, infos = run_alone(oracle_lib, 1, np.zeros((20, 20), np.uint8), pos=(5, 5), forced=0)
    assert infos[0]["deaths"] == 0 and ow.agents()["row"][0] == 4


def test_energy_at_the_threshold_counts_neither_way(oracle_lib):
    # an agent held exactly at E_min = 0 (no decay, no food) neither progresses
    # towards reproduction nor towards death: no child and no death however long
    cfg = paper_cfg(oracle_lib, H=20, W=20, n_init=0, cap=8, decay=0, T_repr=3, T_death=3, spont=0.0,
                    regrow_pI=0.0)
    ow = oracle_lib.OracleWorld(cfg, 3)
    im = image(ow, np.zeros((20, 20), np.uint8), [(10, 10)])
    im["energy"][:] = 0
    ow.load(im)
    ow.set_forced(None, default=4)
    infos = [ow.step() for _ in range(20)]
    assert not any(i["births"] for i in infos) and not any(i["deaths"] for i in infos)
    a = ow.agents()
    assert a["energy"][0] == 0 and a["streak"][0] == 0


def test_births_fill_the_free_slots_in_uid_order(oracle_lib):
    # three eligible agents stacked on one cell, two free slots: the first two
    # (uid order) have a child on that cell, the third keeps its streak; with
    # the table full, nobody has one
    cfg = paper_cfg(oracle_lib, H=20, W=20, n_init=0, cap=5, decay=0, T_repr=1, spont=0.0, regrow_pI=0.0)
    ow = oracle_lib.OracleWorld(cfg, 3)
    ow.load(image(ow, np.zeros((20, 20), np.uint8), [(10, 10)] * 3))
    ow.set_forced(None, default=4)
    info = ow.step()
    a = ow.agents()
    assert info["births"] == 2 and ow.n_live == 5
    assert list(a["uid"]) == [0, 1, 2, 3, 4]
    assert all(a["row"] == 10) and all(a["col"] == 10)
    assert list(a["streak"]) == [0, 0, 1, 0, 0]
    info = ow.step()
    assert info["births"] == 0 and ow.agents()["streak"][2] == 2


def test_wall_death_eats_nothing(oracle_lib):
    # an agent on a resource cell that walks into the wall dies where it stood
    # and eats nothing: the resource stays (regrowth off)
    R = np.zeros((20, 20), np.uint8)
    R[0, 5] = 1
    ow, infos = run_alone(oracle_lib, 1, R, pos=(0, 5), forced=0, spont=0.0, regrow_pI=0.0)
    assert infos[0]["deaths"] == 1 and infos[0]["eaten"] == 0
    assert ow.grid()[0, 5] == 1
    # the same cell with a staying agent: it eats the resource
    ow, infos = run_alone(oracle_lib, 1, R, pos=(0, 5), forced=4, spont=0.0, regrow_pI=0.0)
    assert infos[0]["eaten"] == 1 and ow.grid()[0, 5] == 0


def test_climate_thresholds_high_precision(oracle_lib):
    # floor(2^32 p), p = p_I c(x) + c, c(x) = (alpha^x + 1) / (alpha + 1),
    # x = row / (H - 1), for one resource neighbour (p_I on) and for two (off),
    # recomputed in 50-digit decimal arithmetic from the same doubles; the
    # double computation may differ by one only where 2^32 p lies within a
    # hair of the integer between the two results
    from decimal import Decimal, getcontext
    getcontext().prec = 50
    for H, pI, alpha, spont in ((200, 0.002, 200.0, 5e-5), (7, 0.9, 3.5, 0.01), (33, 0.25, 1000.0, 0.0)):
        cfg = paper_cfg(oracle_lib, H=H, regrow_pI=pI, regrow_alpha=alpha, spont=spont)
        tab = oracle_lib.threshold_table(cfg)
        a, c, p1 = Decimal(alpha), Decimal(spont), Decimal(pI)
        for row in range(H):
            x = Decimal(row) / Decimal(H - 1)
            cx = (a ** x + 1) / (a + 1)
            for n, pin in ((1, p1), (2, Decimal(0))):
                real = (pin * cx + c) * Decimal(2 ** 32)
                ex = min(int(real), 2 ** 32) if real > 0 else 0
                got = int(tab[row, n])
                if got != ex:
                    assert abs(got - ex) == 1 and abs(real - max(got, ex)) < Decimal("1e-4"), (H, row, n, got, ex)


def test_stacked_agents_one_eater(oracle_lib):
    # three agents step onto one resource cell: they stack, the smallest
    # (EAT draw, uid) eats (EAT = stream 9 of the pinned Philox)
    cfg = paper_cfg(oracle_lib, H=20, W=20, n_init=0, cap=8, spont=0.0, regrow_pI=0.0)
    for seed in range(10):
        ow = oracle_lib.OracleWorld(cfg, seed)
        R = np.zeros((20, 20), np.uint8)
        R[10, 10] = 1
        ow.load(image(ow, R, [(9, 10), (11, 10), (10, 11)]))
        ow.set_forced(np.array([1, 0, 3], np.int32))   # S, N, W: all onto (10, 10)
        info = ow.step()
        a = ow.agents()
        assert all(a["row"] == 10) and all(a["col"] == 10)
        ctr = np.array([[u, 0, 9, 0] for u in range(3)], np.uint32)
        words = oracle_lib.philox(ctr, [seed & 0xFFFFFFFF, seed >> 32])[:, 0]
        keys = [(int(words[u]) << 32) | u for u in range(3)]
        eater = int(np.argmin(keys))
        e = a["energy"]
        assert info["eaten"] == 1
        for u in range(3):
            assert e[u] == (120 if u == eater else 119)
        assert ow.grid()[10, 10] == 0


def test_observation_counts_stacked_agents(oracle_lib):
    cfg = paper_cfg(oracle_lib, H=30, W=30, n_init=0, cap=8, obs_radius=7, hidden=4,
                    controller=oracle_lib.CTRL_CNN_LSTM, spont=0.0, regrow_pI=0.0)
    ow = oracle_lib.OracleWorld(cfg, 1)
    ow.load(image(ow, np.zeros((30, 30), np.uint8), [(10, 10), (10, 10), (10, 10), (12, 9)]))
    o = ow.obs_cnn(0)
    assert o[7, 7, 1] == 3 and o[9, 6, 1] == 1 and o[:, :, 1].sum() == 4


def test_paper_run_invariants(oracle_lib):
    for ctrl, extra in ((0, {}), (1, dict(obs_radius=7, hidden=4, controller=1))):
        cfg = paper_cfg(oracle_lib, T_repr=25, T_death=30, regrow_pI=0.2, spont=0.002, **extra)
        ow = oracle_lib.OracleWorld(cfg, 4)
        stacked = births = deaths = 0
        res = int(ow.grid().sum())
        for _ in range(150):
            before = ow.agents()
            info = ow.step()
            a = ow.agents()
            R = ow.grid()
            births += info["births"]
            deaths += info["deaths"]
            assert len(a["uid"]) == len(before["uid"]) + info["births"] - info["deaths"]
            assert np.all(a["energy"] <= cfg.E_max)
            assert np.all((0 <= a["row"]) & (a["row"] < cfg.H) & (0 <= a["col"]) & (a["col"] < cfg.W))
            cells = a["row"] * cfg.W + a["col"]
            stacked = max(stacked, int(np.bincount(cells).max()) if len(cells) else 0)
            # resources only fall by what was eaten, and only rise where empty cells grew
            assert int(R.sum()) >= res - info["eaten"]
            res = int(R.sum())
            assert info["resources"] == res
        assert births > 20 and deaths > 5 and stacked >= 2
