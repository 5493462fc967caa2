"""Lab environments (Sec. 2.2): the greediness and efficiency measures on
hand-made counter series, and the lab world's semantics in the oracle (no
regrowth, no births, one agent) with G recomputed from per-step snapshots."""
import numpy as np
import pytest

from paper_2302_09334_amd import lab


def test_greediness_windows():
    seen = np.zeros(100, int)
    eaten = np.zeros(100, int)
    seen[3] = 1                      # window 0: seen, not eaten
    seen[25] = 1; eaten[30] = 1      # window 1: seen and eaten
    eaten[45] = 1; seen[59] = 1      # window 2: both (in different steps)
    # window 3: nothing; window 4: seen only
    seen[95] = 1
    G, t_r, c_r = lab.greediness(seen, eaten)
    assert (t_r, c_r) == (4, 2) and G == 0.5
    assert np.isnan(lab.greediness(np.zeros(40), np.zeros(40))[0])
    # a partial last window is ignored
    assert lab.greediness(np.ones(39), np.ones(39))[1:] == (1, 1)


def test_efficiency():
    assert lab.efficiency(np.array([1, 0, 2]), np.array([0, 1, 1])) == 1.0   # 3 eaten, 3 individuals
    assert lab.efficiency(np.array([5]), np.array([0])) == 5.0


def test_anova_tukey_detects_a_difference():
    rng = np.random.default_rng(0)
    a, b, c = rng.normal(0, 0.1, 10), rng.normal(0, 0.1, 10), rng.normal(1, 0.1, 10)
    st = lab.anova_tukey([a, b, c])
    assert st["anova_p"] < 1e-6 and st["tukey_p"][0][2] < 0.05 and st["tukey_p"][0][1] > 0.05


def test_lab_config():
    from paper_2302_09334_amd import workloads
    c = lab.lab_config(workloads.WORKLOADS["net1k"], 0.3, False)
    assert (c["H"], c["W"], c["cap"], c["n_init"]) == (40, 40, 1, 1)
    assert c["rate_top"] == c["rate_bottom"] == c["spont"] == 0.0 and c["T_repr"] >= 1 << 30
    r = lab.lab_config(workloads.WORKLOADS["net1k"], 0.3, True)
    assert r["cap"] == 64 and r["T_repr"] == 20


@pytest.mark.parametrize("controller", [0, 1])
def test_lab_world_in_the_oracle(oracle_lib, controller):
    from paper_2302_09334_amd import workloads
    base = dict(workloads.WORKLOADS["cfg0"])
    if controller:
        base.update(obs_radius=7, hidden=4, controller=1, w_init_gain=1.0)
    cfg = lab.lab_config(base, 0.15, False)
    ow = oracle_lib.OracleWorld(oracle_lib.OracleConfig.from_dict(cfg), 5)
    # an "evolved" agent: any genome, alone at the centre
    s = ow.state(with_hidden=True, with_theta=True)
    genome = np.random.default_rng(1).normal(0, 0.5, ow.P).astype(np.float32)
    img = dict(t=0, n_live=1, next_uid=1, R=s["R"], uid=np.array([0], np.uint32),
               row=np.array([20], np.int32), col=np.array([20], np.int32), energy=np.array([cfg["E0"]], np.int32),
               age=np.array([0], np.int32), streak=np.array([0], np.int32),
               h=np.zeros((1, oracle_lib.OracleConfig.from_dict(cfg).state_size), np.float32), theta=genome[None],
               last_action=np.array([oracle_lib.NO_ACTION], np.uint8), ate=np.array([0], np.uint8))
    ow.load(img)
    seen, eaten, seen_ref, eaten_ref = [], [], [], []
    res_prev = int(ow.grid().sum())
    for _ in range(200):
        a = ow.agents()
        R = ow.grid()
        rho = cfg["obs_radius"]
        if len(a["uid"]):
            r, c = int(a["row"][0]), int(a["col"][0])
            seen_ref.append(int(R[max(r - rho, 0):r + rho + 1, max(c - rho, 0):c + rho + 1].any()))
        else:
            seen_ref.append(0)
        e0 = int(a["energy"][0]) if len(a["uid"]) else None
        info = ow.step()
        a1 = ow.agents()
        eaten_ref.append(int(e0 is not None and (len(a1["uid"]) == 0 and info["eaten"] > 0 or
                                                 len(a1["uid"]) and int(a1["energy"][0]) - e0 == cfg["gain"] - cfg["decay"])))
        seen.append(info["seen"])
        eaten.append(info["eaten"])
        assert info["births"] == 0 and info["n_live"] <= 1
        res = int(ow.grid().sum())
        assert res == res_prev - info["eaten"]          # nothing regrows
        res_prev = res
    assert seen == seen_ref and eaten == eaten_ref
    G, t_r, c_r = lab.greediness(np.array(seen), np.array(eaten))
    assert t_r > 0
