"""The segmented parity harness (tests/parity_util.py) on the CPU: a stand-in
device that is itself an oracle world passes it, and a stand-in whose state,
counters or logits carry one planted difference is caught by it."""
import numpy as np
import pytest

from parity_util import run_parity_segmented


class OracleDevice:
    """A World-like object backed by the oracle: step / sync / counters /
    action_log / snapshot / move_hist, with optional planted differences."""

    def __init__(self, cfg, seed, plant=None):
        import oracle
        self.ow = oracle.OracleWorld(oracle.OracleConfig.from_dict(cfg), seed)
        self.logs, self.ctrs = {}, {}
        self.plant = plant or {}

    def step(self, k):
        for _ in range(k):
            t = self.ow.t
            info = self.ow.step()
            oc = self.ow.last_controller()
            logits = oc["logits"].astype(np.float32)
            if self.plant.get("logit_step") == t and len(logits):
                logits[0, 0] += 1e-3 * max(1.0, float(np.abs(logits[0]).max()))
            self.logs[t] = {"uid": oc["uid"], "action": oc["action"], "logits": logits}
            c = dict(info)
            if self.plant.get("eaten_step") == t:
                c["eaten"] += 1
            self.ctrs[t] = c

    def sync(self):
        pass

    def counters(self, first, n):
        keys = ("n_live", "births", "deaths", "eaten", "resources", "claim_wins", "dead_age", "seen")
        return {k: np.array([self.ctrs[first + i][k] for i in range(n)], np.int64) for k in keys}

    def action_log(self, t):
        return self.logs[t]

    def snapshot(self, hidden=False, theta=False):
        s = self.ow.state(with_hidden=True, with_theta=theta)
        if self.plant.get("energy_at") == s["t"] and s["n_live"]:
            s["energy"] = s["energy"].copy()
            s["energy"][-1] += 1
        if self.plant.get("theta_at") == s["t"] and theta and s["n_live"]:
            s["theta"] = s["theta"].copy()
            s["theta"][0, 7] = np.nextafter(s["theta"][0, 7], np.float32(9))
        return s

    def move_hist(self, first, n):
        return self.ow.move_hist()[first:first + n]


@pytest.fixture(scope="module")
def cfg0(oracle_lib):
    from paper_2302_09334_amd import workloads
    return workloads.WORKLOADS["cfg0"]


def test_segmented_harness_accepts_oracle(cfg0):
    st = run_parity_segmented(OracleDevice(cfg0, 0), cfg0, 0, 300, 20, 100, workers=2)
    assert st["segments"] == 3 and st["steps"] == 300 and st["agent_steps"] > 0


@pytest.mark.parametrize("plant", [dict(energy_at=200), dict(theta_at=100), dict(eaten_step=150),
                                   dict(logit_step=250)])
def test_segmented_harness_catches_planted_difference(cfg0, plant):
    with pytest.raises(AssertionError):
        run_parity_segmented(OracleDevice(cfg0, 0, plant), cfg0, 0, 300, 20, 100, workers=2)
