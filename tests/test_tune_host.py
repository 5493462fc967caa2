"""Host logic of the autotuner (no GPU): every combination of launch mode,
act rows per round trip and steps per launch is timed from the same saved
state, the fastest one is applied, and the batch is left at the state it
started from."""
import pytest

from paper_2302_09334_amd import tune


class FakeBatch:
    """Records the calls; a step costs a known time on a fake clock."""

    def __init__(self, clock, cost):
        self.clock = clock
        self.cost = cost
        self.mode = None
        self.rows = None
        self.state = "start"
        self.calls = []

    def snapshots(self):
        return "saved:" + self.state

    def set_mode(self, m):
        self.mode = m

    def set_tuning(self, r):
        self.rows = r

    def load(self, s):
        self.calls.append(("load", s))
        self.state = s.split(":", 1)[1]

    def step(self, k):
        self.calls.append(("step", self.mode, self.rows, k, self.state))
        self.clock[0] += self.cost(self.mode, self.rows, k) * k
        self.state = "advanced"

    def sync(self):
        pass


def test_autotune_picks_the_fastest_and_restores_the_state(monkeypatch):
    import torch
    monkeypatch.setattr(torch.cuda, "synchronize", lambda: None)
    clock = [0.0]
    monkeypatch.setattr(tune.time, "perf_counter", lambda: clock[0])

    # per-step cost: graph with 16 rows and 50 steps per launch is the fastest
    def cost(mode, rows, k):
        c = 1e-3
        if mode == "graph":
            c -= 2e-4
        if rows == 16:
            c -= 1e-4
        if k == 50:
            c -= 5e-5
        return c

    b = FakeBatch(clock, cost)
    out = tune.autotune(b, trial_steps=100)
    assert len(out["trials"]) == len(tune.MODES) * len(tune.ROWS) * len(tune.KS)
    assert (out["best"]["mode"], out["best"]["act_rows"], out["best"]["K"]) == ("graph", 16, 50)
    assert out["best"]["us_per_step"] == pytest.approx((1e-3 - 2e-4 - 1e-4 - 5e-5) * 1e6)
    # applied, and back at the saved state
    assert (b.mode, b.rows) == ("graph", 16)
    assert b.calls[-1] == ("load", "saved:start") and b.state == "start"
    # every timed trial starts from the saved state: each run of steps follows a load
    for i, c in enumerate(b.calls):
        if c[0] == "step" and (i == 0 or b.calls[i - 1][0] == "load"):
            assert c[4] == "start"
