"""Pins of the oracle's version of the paper's controller (App. B.5).

* Architecture: the parameter count the paper states (2445) and the 72 CNN
  features follow from the SAME/VALID and bias readings.
* Forward pass: against torch float64 library layers (conv2d with stride 2
  and one cell of zero padding, avg_pool2d 2x2 stride 1, LSTMCell with gates
  i, f, g, o and a zero input bias, linear + tanh, linear).
* Observation: closed forms (a world full of resources: resource channel =
  inside the grid, wall channel = outside) and every agent's window rebuilt
  from the world's grid and agent positions.
* Sampling: the Gumbel transform against its CDF exp(-exp(-x)) and its two
  extreme words; sampled actions against softmax(50 l) frequencies.
* Integration: with forced actions the integer dynamics do not depend on the
  controller; the previous action and the ate bit carried between steps.
"""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F

torch.set_default_dtype(torch.float64)

P_PAPER = 2445   # App. B.5: total parameters of the agent network
WIN = 15         # App. B.4: field of view 15 x 15


def split_genome(th):
    """Genome order of the paper's controller -> torch-shaped float64 arrays."""
    th = np.asarray(th, np.float64)
    o = 0

    def take(n):
        nonlocal o
        v = th[o:o + n]
        o += n
        return v
    c1w = take(3 * 3 * 3 * 4).reshape(3, 3, 3, 4)      # ky kx ci co
    c1b = take(4)
    c2w = take(3 * 3 * 4 * 8).reshape(3, 3, 4, 8)
    c2b = take(8)
    wi = take(78 * 16).reshape(78, 4, 4)                # i gate unit
    wh = take(4 * 16).reshape(4, 4, 4)                  # j gate unit
    lb = take(16).reshape(4, 4)                         # gate unit
    d8w = take(82 * 8).reshape(82, 8)
    d8b = take(8)
    d5w = take(8 * 5).reshape(8, 5)
    d5b = take(5)
    assert o == th.size
    return dict(c1w=c1w, c1b=c1b, c2w=c2w, c2b=c2b, wi=wi, wh=wh, lb=lb, d8w=d8w, d8b=d8b, d5w=d5w, d5b=d5b)


def torch_forward(th, obs, prev_action, ate, h, c):
    g = {k: torch.from_numpy(np.ascontiguousarray(v)) for k, v in split_genome(th).items()}
    x = torch.from_numpy(np.asarray(obs, np.float64)).permute(2, 0, 1)[None]       # 1 x 3 x 15 x 15
    y = F.conv2d(x, g["c1w"].permute(3, 2, 0, 1), g["c1b"], stride=2, padding=1)
    y = F.avg_pool2d(y, 2, stride=1)
    y = F.conv2d(y, g["c2w"].permute(3, 2, 0, 1), g["c2b"], stride=2, padding=1)
    y = F.avg_pool2d(y, 2, stride=1)
    feat = y[0].permute(1, 2, 0).reshape(-1)                                      # (row, col, ch)
    onehot = torch.zeros(5)
    if prev_action < 5:
        onehot[prev_action] = 1.0
    emb = torch.cat([feat, onehot, torch.tensor([float(ate)])])
    cell = torch.nn.LSTMCell(78, 4)
    with torch.no_grad():
        cell.weight_ih.copy_(g["wi"].permute(1, 2, 0).reshape(16, 78))
        cell.weight_hh.copy_(g["wh"].permute(1, 2, 0).reshape(16, 4))
        cell.bias_ih.zero_()
        cell.bias_hh.copy_(g["lb"].reshape(16))
        h1, c1 = cell(emb[None], (torch.from_numpy(np.float64(h))[None], torch.from_numpy(np.float64(c))[None]))
        cat = torch.cat([emb, h1[0]])
        z = torch.tanh(F.linear(cat, g["d8w"].T, g["d8b"]))
        logits = F.linear(z, g["d5w"].T, g["d5b"])
    return feat.numpy(), h1[0].numpy(), c1[0].numpy(), logits.numpy()


def cnn_cfg(oracle_lib, **kw):
    d = dict(H=40, W=64, cap=600, n_init=300, obs_radius=7, hidden=4, res_init_p=0.3, rate_scale=5.0,
             T_repr=8, L_max=90, w_init_gain=1.0, controller=oracle_lib.CTRL_CNN_LSTM)
    d.update(kw)
    return oracle_lib.OracleConfig(**d)


def test_param_count_matches_paper(oracle_lib):
    assert oracle_lib.cnn_n_params() == P_PAPER
    assert oracle_lib.cnn_n_features() == 72
    # 112 + 296 + 1328 + 664 + 45 by layer
    assert (3 * 3 * 3 * 4 + 4) + (3 * 3 * 4 * 8 + 8) + (78 * 16 + 4 * 16 + 16) + (82 * 8 + 8) + (8 * 5 + 5) == P_PAPER


def test_initial_genome_spread(oracle_lib):
    """The initial genome of the paper's network: each weight layer N(0, gain^2
    / fan_in) with fan_in 27 and 36 (the convolutions), 78 and 4 (the LSTM's
    input and hidden kernels), 82 and 8 (the dense layers); every bias zero."""
    from scipy import stats
    gain = 0.7
    w = oracle_lib.OracleWorld(cnn_cfg(oracle_lib, n_init=300, w_init_gain=gain), 9)
    th = w.theta()
    layers = [split_genome(t) for t in th]
    for name, fan in (("c1w", 27), ("c2w", 36), ("wi", 78), ("wh", 4), ("d8w", 82), ("d5w", 8)):
        v = np.concatenate([g[name].ravel() for g in layers]) / (gain / np.sqrt(fan))
        assert stats.kstest(v, "norm").pvalue > 1e-3, name
    for name in ("c1b", "c2b", "lb", "d8b", "d5b"):
        assert not any(g[name].any() for g in layers), name
    w.close()


@pytest.mark.parametrize("trial", range(8))
def test_forward_matches_torch(oracle_lib, trial):
    rng = np.random.default_rng(100 + trial)
    th = rng.normal(0, 0.4, P_PAPER).astype(np.float32)
    obs = rng.integers(0, 2, (WIN, WIN, 3)).astype(np.float64)
    if trial % 2:
        obs[:, :, 2] = 0.0
        obs[: trial, :, :] = [0.0, 0.0, 1.0]          # a wall band along the top
    prev = int(trial % 6)                              # 5 = no previous action
    ate = trial % 3 == 0
    h = rng.normal(0, 0.5, 4).astype(np.float32)
    c = rng.normal(0, 1.0, 4).astype(np.float32)
    ho, co, lg = oracle_lib.cnn_eval(th, obs, prev, ate, h, c)
    _, rh, rc, rl = torch_forward(th, obs, prev, ate, h, c)
    assert np.abs(ho - rh).max() <= 1e-12
    assert np.abs(co - rc).max() <= 1e-12
    assert np.abs(lg - rl).max() <= 1e-11 * max(1.0, np.abs(rl).max())


def test_forward_features_see_the_window(oracle_lib):
    # a single resource pixel moves the logits through a conv tap that SAME
    # padding keeps (corner pixel) -- a dropped padding row would lose it
    rng = np.random.default_rng(5)
    th = rng.normal(0, 0.4, P_PAPER).astype(np.float32)
    zero = np.zeros((WIN, WIN, 3))
    z4 = np.zeros(4, np.float32)
    base = oracle_lib.cnn_eval(th, zero, 5, 0, z4, z4)[2]
    for (y, x) in [(0, 0), (14, 14), (0, 14), (7, 7)]:
        o = zero.copy()
        o[y, x, 0] = 1.0
        lg = oracle_lib.cnn_eval(th, o, 5, 0, z4, z4)[2]
        ref = torch_forward(th, o, 5, 0, z4, z4)[3]
        assert np.abs(lg - ref).max() <= 1e-12
        assert np.abs(lg - base).max() > 1e-6, (y, x)


def test_observation_closed_form(oracle_lib):
    cfg = cnn_cfg(oracle_lib, H=20, W=30, n_init=1, cap=4, res_init_p=1.0)
    for seed in range(8):
        ow = oracle_lib.OracleWorld(cfg, seed)
        a = ow.agents()
        r, c = int(a["row"][0]), int(a["col"][0])
        o = ow.obs_cnn(0)
        for dy in range(-7, 8):
            for dx in range(-7, 8):
                inside = 0 <= r + dy < 20 and 0 <= c + dx < 30
                px = o[dy + 7, dx + 7]
                assert px[0] == (1.0 if inside else 0.0)
                assert px[2] == (0.0 if inside else 1.0)
                assert px[1] == (1.0 if (dy == 0 and dx == 0) else 0.0)


def test_observation_from_state(oracle_lib):
    ow = oracle_lib.OracleWorld(cnn_cfg(oracle_lib), 3)
    for _ in range(3):
        ow.step()
    R = ow.grid()
    a = ow.agents()
    occ = np.zeros(R.shape, np.float64)
    occ[a["row"], a["col"]] = 1.0
    H, W = R.shape
    for i in range(0, len(a["uid"]), 7):
        o = ow.obs_cnn(i)
        r, c = int(a["row"][i]), int(a["col"][i])
        ref = np.zeros((WIN, WIN, 3))
        for y in range(WIN):
            for x in range(WIN):
                rr, cc = r + y - 7, c + x - 7
                if 0 <= rr < H and 0 <= cc < W:
                    ref[y, x] = [R[rr, cc], occ[rr, cc], 0.0]
                else:
                    ref[y, x] = [0.0, 0.0, 1.0]
        assert np.array_equal(o, ref), i


def test_gumbel_extremes_and_cdf(oracle_lib):
    g = oracle_lib.gumbel(np.array([0, 0xFFFFFFFF], np.uint32))
    u_lo, u_hi = 2.0 ** -24, 1.0 - 2.0 ** -24
    assert abs(g[0] - (-math.log(-math.log(u_lo)))) < 1e-5
    assert abs(g[1] - (-math.log(-math.log(u_hi)))) < 1e-4
    words = oracle_lib.philox(np.stack([np.arange(200000, dtype=np.uint32), np.zeros(200000, np.uint32),
                                        np.full(200000, 8, np.uint32), np.zeros(200000, np.uint32)], 1),
                              [1, 2])[:, 0]
    x = np.sort(oracle_lib.gumbel(words).astype(np.float64))
    cdf = np.exp(-np.exp(-x))
    emp = np.arange(1, x.size + 1) / x.size
    assert np.abs(cdf - emp).max() < 0.005
    assert abs(x.mean() - 0.5772156649) < 0.01       # Euler-Mascheroni constant
    assert abs(x.var() - math.pi ** 2 / 6) < 0.03


def test_sampling_frequencies(oracle_lib):
    lg = np.array([0.0, 0.02, -0.01, 0.03, 0.0], np.float32)
    p = np.exp(50.0 * lg.astype(np.float64))
    p /= p.sum()
    N = 30000
    counts = np.zeros(5)
    for u in range(N):
        a, sc = oracle_lib.sample_action(7, u, 11, lg)
        counts[a] += 1
        assert a == int(np.argmax(sc))
    sd = np.sqrt(N * p * (1 - p))
    assert np.all(np.abs(counts - N * p) < 5 * sd), (counts, N * p)
    # a gap of 1 in the logits is 50 in the scores: the top action always wins
    lg2 = np.array([0.0, 1.0, 0.0, 0.0, 0.0], np.float32)
    assert all(oracle_lib.sample_action(7, u, 3, lg2)[0] == 1 for u in range(2000))


def test_forced_dynamics_independent_of_controller(oracle_lib):
    kw = dict(H=30, W=50, cap=500, n_init=200, res_init_p=0.3, rate_scale=5.0, T_repr=8, L_max=90)
    a = oracle_lib.OracleWorld(cnn_cfg(oracle_lib, **kw), 9)
    b = oracle_lib.OracleWorld(oracle_lib.OracleConfig(obs_radius=2, hidden=16, **kw), 9)
    rng = np.random.default_rng(0)
    births = 0
    for s in range(60):
        forced = rng.integers(0, 5, a.next_uid + 500).astype(np.int32)
        a.set_forced(forced)
        b.set_forced(forced)
        ia, ib = a.step(), b.step()
        births += ia["births"]
        ia.pop("seen"), ib.pop("seen")   # depends on the field of view (15 x 15 against 5 x 5)
        assert ia == ib, s
        assert np.array_equal(a.grid(), b.grid())
        sa, sb = a.agents(), b.agents()
        for k in sa:
            assert np.array_equal(sa[k], sb[k]), (s, k)
        assert np.array_equal(a.recurrent_inputs()["last_action"], b.recurrent_inputs()["last_action"])
    assert births > 10


def test_recurrent_inputs_and_state(oracle_lib):
    cfg = cnn_cfg(oracle_lib)
    ow = oracle_lib.OracleWorld(cfg, 4)
    ri = ow.recurrent_inputs()
    assert np.all(ri["last_action"] == oracle_lib.NO_ACTION) and np.all(ri["ate"] == 0)
    assert np.all(ow.hidden() == 0) and ow.hidden().shape == (cfg.n_init, 8)
    births = deaths = 0
    # 100 steps: births from step 8, deaths by starvation and age from step 50,
    # so the survivors are compacted many times; each survivor's previous
    # action, ate bit, streak and recurrent state must stay its own
    for s in range(100):
        before = ow.agents()
        e0 = {int(u): int(e) for u, e in zip(before["uid"], before["energy"])}
        k0 = {int(u): int(k) for u, k in zip(before["uid"], before["streak"])}
        if s % 10 == 9:
            ri0 = ow.recurrent_inputs()
            hs0 = ow.hidden()
            sample = {int(before["uid"][i]): (ow.obs_cnn(i), int(ri0["last_action"][i]), int(ri0["ate"][i]), hs0[i])
                      for i in range(0, len(before["uid"]), 17)}
            thetas = dict(zip((int(u) for u in before["uid"]), ow.theta()))
        info = ow.step()
        births += info["births"]
        deaths += info["deaths"]
        last = ow.last_controller()
        acted = {int(u): int(x) for u, x in zip(last["uid"], last["action"])}
        after = ow.agents()
        ri = ow.recurrent_inputs()
        hs = ow.hidden()
        for i, u in enumerate(after["uid"]):
            u = int(u)
            if u in acted:
                assert ri["last_action"][i] == acted[u]
                ate = after["energy"][i] - e0[u] == cfg.gain - cfg.decay
                assert ri["ate"][i] == int(ate)
                # at or above E_repr the count goes on (or restarts at 0 with a
                # birth, possible only once it has reached T_repr); below, 0
                k = int(after["streak"][i])
                if after["energy"][i] >= cfg.E_repr:
                    assert k == k0[u] + 1 or (k == 0 and k0[u] + 1 >= cfg.T_repr), (s, u)
                else:
                    assert k == 0, (s, u)
                if s % 10 == 9 and u in sample:
                    obs, pa, at, h0 = sample[u]
                    _, h1, c1, _ = torch_forward(thetas[u], obs, pa, at, h0[:4], h0[4:])
                    assert np.abs(hs[i][:4] - h1).max() < 1e-6 and np.abs(hs[i][4:] - c1).max() < 1e-6, (s, u)
            else:   # born in this step
                assert ri["last_action"][i] == oracle_lib.NO_ACTION and ri["ate"][i] == 0
                assert np.all(hs[i] == 0)
    assert births > 5 and deaths > 50
    # sampled actions are not all the same
    assert len(set(acted.values())) > 1
