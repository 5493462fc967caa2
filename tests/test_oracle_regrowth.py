"""Pins of the oracle's resource regrowth (App. B.1, Eq. (1), with the rate
linear in the row, the 24-cell neighbourhood count and a spontaneous term).

* The threshold table against exact rational arithmetic.
* One full regrowth step recomputed independently (numpy neighbour counts,
  rational thresholds, the pinned generator) on small grids.
* Closed forms: no growth at zero rates; full rate at the bottom row.
* Empirical growth frequencies per (row, count) class against p.
"""
import numpy as np
import pytest

from oracle_ref import exact_threshold, neighbour_counts


def cfg_dict(**kw):
    d = dict(H=20, W=30, cap=4, n_init=0, obs_radius=2, hidden=16, res_init_p=0.2,
             rate_bottom=0.02, rate_top=0.002, rate_scale=1.0, spont=1e-5)
    d.update(kw)
    return d


@pytest.mark.parametrize("over", [dict(), dict(H=200, W=5, rate_scale=5.0),
                                  dict(H=2, rate_bottom=0.9, rate_top=0.3, spont=0.3),
                                  dict(H=7, rate_bottom=0.5, rate_top=0.0, spont=0.0)])
def test_threshold_table_exact(oracle_lib, over):
    d = cfg_dict(**over)
    tab = oracle_lib.threshold_table(oracle_lib.OracleConfig.from_dict(d))
    for row in range(d["H"]):
        for n in range(25):
            ex = exact_threshold(d, row, n)
            got = int(tab[row, n])
            assert abs(got - ex) <= 1, (row, n, got, ex)
            if got != ex:
                # double rounding may only move the result across an integer
                # that p * 2^32 lies within a hair of: max(got, ex)
                assert abs(exact_threshold(d, row, n, real=True) - max(got, ex)) < 1e-4, (row, n, got, ex)
    # orientation: the bottom row grows fastest, the top row slowest
    assert tab[-1, 24] >= tab[0, 24]


def regrow_reference(oracle_lib, R_before, d, seed, t):
    """Next grid from the post-eating grid: an empty cell grows iff its REGROW
    draw (counter = (cell, t, 7, 0)) is below floor(p 2^32)."""
    H, W = R_before.shape
    n = neighbour_counts(R_before)
    ctr = np.zeros((H * W, 4), np.uint32)
    ctr[:, 0] = np.arange(H * W)
    ctr[:, 1] = t
    ctr[:, 2] = 7
    draws = oracle_lib.philox(ctr, [seed & 0xFFFFFFFF, seed >> 32])[:, 0].reshape(H, W)
    thr = np.array([[exact_threshold(d, r, k) for k in range(25)] for r in range(H)], dtype=object)
    out = R_before.copy()
    for r in range(H):
        for c in range(W):
            if not R_before[r, c] and int(draws[r, c]) < thr[r, n[r, c]]:
                out[r, c] = 1
    return out


@pytest.mark.parametrize("seed,over", [(0, dict(rate_bottom=0.6, rate_top=0.1)),
                                       (7, dict(H=9, W=11, rate_bottom=0.3, rate_top=0.3, spont=0.05)),
                                       (2**40 + 5, dict())])
def test_regrowth_step_recomputed(oracle_lib, seed, over):
    d = cfg_dict(**over)
    w = oracle_lib.OracleWorld(oracle_lib.OracleConfig.from_dict(d), seed)
    for t in range(6):
        before = w.grid().copy()
        w.step()
        assert np.array_equal(w.grid(), regrow_reference(oracle_lib, before, d, seed, t))


def test_no_rates_no_growth(oracle_lib):
    d = cfg_dict(rate_bottom=0.0, rate_top=0.0, spont=0.0, res_init_p=0.3)
    w = oracle_lib.OracleWorld(oracle_lib.OracleConfig.from_dict(d), 11)
    g0 = w.grid().copy()
    for _ in range(50):
        w.step()
    assert np.array_equal(w.grid(), g0)
    # an empty grid with no spontaneous growth stays empty
    d = cfg_dict(res_init_p=0.0, spont=0.0, rate_bottom=0.9, rate_top=0.9)
    w = oracle_lib.OracleWorld(oracle_lib.OracleConfig.from_dict(d), 11)
    for _ in range(20):
        w.step()
    assert w.grid().sum() == 0


def test_initial_density(oracle_lib):
    d = cfg_dict(H=200, W=400, res_init_p=0.3)
    g = oracle_lib.OracleWorld(oracle_lib.OracleConfig.from_dict(d), 0).grid()
    n = g.size
    assert abs(g.mean() - 0.3) < 4 * np.sqrt(0.3 * 0.7 / n)


def test_growth_frequencies(oracle_lib):
    """Empirical growth per (row band, neighbour count) class against p."""
    d = cfg_dict(H=40, W=200, rate_bottom=0.4, rate_top=0.04, spont=0.01, res_init_p=0.15)
    w = oracle_lib.OracleWorld(oracle_lib.OracleConfig.from_dict(d), 99)
    H = d["H"]
    tries = {}
    grows = {}
    for t in range(60):
        before = w.grid().copy()
        n = neighbour_counts(before)
        w.step()
        after = w.grid()
        empty = before == 0
        for r in range(H):
            for k in np.unique(n[r][empty[r]]):
                m = empty[r] & (n[r] == k)
                key = (r, int(k))
                tries[key] = tries.get(key, 0) + int(m.sum())
                grows[key] = grows.get(key, 0) + int(after[r][m].sum())
    checked = 0
    for (r, k), nt in tries.items():
        if nt < 200:
            continue
        rate = d["rate_top"] + (d["rate_bottom"] - d["rate_top"]) * r / (H - 1)
        p = rate * k / 24 + d["spont"]
        sd = np.sqrt(p * (1 - p) / nt)
        assert abs(grows[(r, k)] / nt - p) < 5 * sd + 1e-9, (r, k, nt, grows[(r, k)] / nt, p)
        checked += 1
    assert checked > 50
