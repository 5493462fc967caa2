"""Pins of the oracle's controller, genome and observation.

* The GRU cell against torch.nn.GRUCell in float64 (gate order r, z, n, the
  reset gate applied to the hidden projection plus its bias), the head against
  a numpy matrix product.
* Initial genomes: each parameter recomputed from the pinned generator and
  Box-Muller primitives, and the per-layer spread against N(0, gain/sqrt(fan_in)).
* Observations: logits of every agent of a world recomputed from its state
  (resource window, occupancy window with outside cells occupied, energy/E0).
"""
import numpy as np
import pytest
import torch
from scipy import stats

from oracle_ref import genome_to_torch, layer_slices, observation

torch.set_default_dtype(torch.float64)


@pytest.mark.parametrize("rho,hd", [(2, 16), (3, 32), (1, 16)])
def test_gru_matches_torch(oracle_lib, rho, hd):
    rng = np.random.default_rng(rho * 100 + hd)
    n_in = oracle_lib.n_inputs(rho)
    P = oracle_lib.n_params(rho, hd)
    assert P == n_in * hd * 3 + hd * hd * 3 + 6 * hd + 5 * hd + 5
    for trial in range(5):
        theta = rng.normal(0, 0.3, P).astype(np.float32)
        x = rng.integers(0, 2, n_in).astype(np.float64)
        x[-1] = rng.uniform(0, 3)
        h = rng.normal(0, 0.5, hd).astype(np.float32)
        h_out, logits = oracle_lib.gru_eval(n_in, hd, theta, x, h)
        wih, whh, bih, bhh, wo, bo = genome_to_torch(theta, n_in, hd)
        cell = torch.nn.GRUCell(n_in, hd)
        with torch.no_grad():
            cell.weight_ih.copy_(torch.from_numpy(wih))
            cell.weight_hh.copy_(torch.from_numpy(whh))
            cell.bias_ih.copy_(torch.from_numpy(bih))
            cell.bias_hh.copy_(torch.from_numpy(bhh))
            ref_h = cell(torch.from_numpy(x)[None], torch.from_numpy(h.astype(np.float64))[None])[0].numpy()
        assert np.abs(h_out - ref_h).max() <= 1e-12
        ref_logits = wo @ h_out + bo
        assert np.abs(logits - ref_logits).max() <= 1e-12


def test_param_counts(oracle_lib):
    # workload sizes: 5x5x2+1 inputs / GRU 16 and 7x7x2+1 / GRU 32
    assert oracle_lib.n_inputs(2) == 51 and oracle_lib.n_params(2, 16) == 3397
    assert oracle_lib.n_inputs(3) == 99 and oracle_lib.n_params(3, 32) == 12933
    assert oracle_lib.n_params(3, 16) == 5701


def test_initial_genome(oracle_lib):
    cfg = oracle_lib.OracleConfig(H=8, W=8, cap=40, n_init=40, obs_radius=2, hidden=16)
    w = oracle_lib.OracleWorld(cfg, seed=0x1234_0000_0042)
    th = w.theta()
    n_in = oracle_lib.n_inputs(2)
    sl = layer_slices(n_in, 16)
    # exact recomputation of agent uid 3 from the primitives
    u = 3
    P = th.shape[1]
    blocks = (P + 3) // 4
    ctr = np.zeros((blocks, 4), np.uint32)
    ctr[:, 0] = u
    ctr[:, 2] = 3          # INIT_W stream
    ctr[:, 3] = np.arange(blocks)
    seed = 0x1234_0000_0042
    r = oracle_lib.philox(ctr, [seed & 0xFFFFFFFF, seed >> 32])
    z0, z1 = oracle_lib.gauss_pair(r[:, 0], r[:, 1])
    z2, z3 = oracle_lib.gauss_pair(r[:, 2], r[:, 3])
    z = np.stack([z0, z1, z2, z3], axis=1).ravel()[:P]
    std_ih = np.float32(0.5 / np.sqrt(n_in))
    std_hd = np.float32(0.5 / np.sqrt(16))
    ref = np.zeros(P, np.float32)
    ref[sl["W_ih"]] = std_ih * z[sl["W_ih"]]
    ref[sl["W_hh"]] = std_hd * z[sl["W_hh"]]
    ref[sl["W_o"]] = std_hd * z[sl["W_o"]]
    assert np.array_equal(th[u], ref)
    # spread per layer over all agents
    for name, std in (("W_ih", 0.5 / np.sqrt(n_in)), ("W_hh", 0.5 / 4), ("W_o", 0.5 / 4)):
        v = th[:, sl[name]].ravel().astype(np.float64) / std
        assert stats.kstest(v, "norm").pvalue > 1e-3, name
    for name in ("b_ih", "b_hh", "b_o"):
        assert not th[:, sl[name]].any()


@pytest.mark.parametrize("rho,hd,seed", [(2, 16, 3), (3, 32, 4)])
def test_logits_from_observation(oracle_lib, rho, hd, seed):
    cfg = oracle_lib.OracleConfig(H=12, W=9, cap=60, n_init=30, obs_radius=rho, hidden=hd,
                                  res_init_p=0.4)
    w = oracle_lib.OracleWorld(cfg, seed)
    n_in = oracle_lib.n_inputs(rho)
    for step in range(4):
        s = w.state(with_hidden=True, with_theta=True)
        occ = np.zeros((cfg.H, cfg.W))
        occ[s["row"], s["col"]] = 1
        w.step()
        lc = w.last_controller()
        assert np.array_equal(lc["uid"], s["uid"])
        for a in range(s["n_live"]):
            x = observation(s["R"], occ, s["row"][a], s["col"][a], s["energy"][a], cfg.E0, rho)
            wih, whh, bih, bhh, wo, bo = genome_to_torch(s["theta"][a], n_in, hd)
            h = s["h"][a].astype(np.float64)
            gi = wih @ x + bih
            gh = whh @ h + bhh
            r_ = 1 / (1 + np.exp(-(gi[:hd] + gh[:hd])))
            z_ = 1 / (1 + np.exp(-(gi[hd:2 * hd] + gh[hd:2 * hd])))
            n_ = np.tanh(gi[2 * hd:] + r_ * gh[2 * hd:])
            hn = (1 - z_) * n_ + z_ * h
            ref = wo @ hn + bo
            assert np.abs(lc["logits"][a] - ref).max() < 1e-12
            lf = lc["logits"][a].astype(np.float32)
            assert lc["action"][a] == int(np.argmax(lf))
