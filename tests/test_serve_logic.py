"""Serving loop logic on the CPU: the server drives an oracle-backed fake
backend (the backend interface is the server's only dependency).  Checks:
every request runs exactly its steps, the HBM budget is never exceeded,
admission is first-come first-served, and every result equals the same
request run alone."""
import numpy as np

from paper_2302_09334_amd import serve, workloads


class OracleBackend:
    def __init__(self, oracle_lib):
        self.o = oracle_lib
        self.used = 0
        self.peak = 0
        self.created = []

    def required_bytes(self, cfg):
        return cfg["cap"] * 1000 + cfg["H"] * cfg["W"]

    def create(self, cfg, seed):
        w = {"ow": self.o.OracleWorld(self.o.OracleConfig.from_dict(cfg), seed), "acted": 0, "cfg": cfg}
        self.used += self.required_bytes(cfg)
        self.peak = max(self.peak, self.used)
        self.created.append(seed)
        return w

    def step_many(self, ws, k):
        kinds = {serve.world_kind(w["cfg"]) for w in ws}
        assert len(kinds) == 1, kinds   # one controller and rule set per launch
        for w in ws:
            for _ in range(k):
                w["acted"] += w["ow"].n_live
                w["ow"].step()

    def mark(self):
        return None

    def wait(self, m):
        pass

    def agent_steps(self, w, steps):
        return w["acted"]

    def result(self, w):
        s = w["ow"].state(with_hidden=True, with_theta=True)
        return {"digest": serve.state_digest(s), "n_live": s["n_live"], "t": s["t"]}

    def close(self, w):
        self.used -= self.required_bytes(w["cfg"])
        w["ow"].close()


def small_trace():
    reqs = []
    for i in range(9):
        cfg = workloads.make(H=12 + 2 * (i % 3), W=16 + i, cap=40 + 10 * (i % 4), n_init=12, obs_radius=1 + i % 3,
                             hidden=16 if i % 2 else 32, res_init_p=0.4, rate_scale=4.0, T_repr=6, L_max=60)
        reqs.append(serve.Request(i, arrival=0.01 * i, cfg=cfg, seed=100 + i, steps=7 + 5 * (i % 4)))
    return reqs


def test_server_schedules_and_isolates(oracle_lib):
    reqs = small_trace()
    be = OracleBackend(oracle_lib)
    budget = 3 * 80 * 1000
    srv = serve.Server(be, budget_bytes=budget, K=4)
    results, m = srv.run(reqs, realtime=False)
    assert len(results) == len(reqs)
    assert be.peak <= budget and m["peak_budget_used_bytes"] <= budget
    assert be.created == sorted(be.created)          # first come, first served
    for r in reqs:
        res = results[r.rid]
        assert res["steps"] == r.steps and res["t"] == r.steps
        ow = oracle_lib.OracleWorld(oracle_lib.OracleConfig.from_dict(r.cfg), r.seed)
        acted = 0
        for _ in range(r.steps):
            acted += ow.n_live
            ow.step()
        assert res["digest"] == serve.state_digest(ow.state(with_hidden=True, with_theta=True)), r.rid
        assert res["agent_steps"] == acted
    assert m["agent_steps"] == sum(results[r.rid]["agent_steps"] for r in reqs)
    assert m["launches"] > len(reqs) // 3


def test_oversized_request_rejected(oracle_lib):
    be = OracleBackend(oracle_lib)
    big = workloads.make(H=10, W=10, cap=500, n_init=5, obs_radius=1, hidden=16)
    small = workloads.make(H=10, W=10, cap=20, n_init=5, obs_radius=1, hidden=16)
    reqs = [serve.Request(0, 0.0, big, 1, 5), serve.Request(1, 0.0, small, 2, 5)]
    results, _ = serve.Server(be, budget_bytes=100_000, K=5).run(reqs, realtime=False)
    assert "error" in results[0] and results[1]["steps"] == 5


def test_trace_generators_are_seeded():
    a = workloads.serve_trace(duration_s=5, seed=3)
    b = workloads.serve_trace(duration_s=5, seed=3)
    assert [x["arrival"] for x in a] == [x["arrival"] for x in b]
    assert all(500 <= x["steps"] <= 5000 for x in a)
    rate = len(workloads.serve_trace(duration_s=200, seed=1)) / 200
    assert 17 < rate < 23
    m = workloads.batch_manifest(64)
    assert len(m) == 64 and len({e["seed"] for e in m}) == 64
    assert all(512 <= e["cfg"]["cap"] <= 8192 and e["cfg"]["cap"] % 64 == 0 for e in m)
    assert np.all([(e["cfg"]["H"], e["cfg"]["W"]) in workloads.GRID_SET for e in m])


def test_mixed_kinds_are_launched_apart(oracle_lib):
    # requests with both controllers and both rule sets in one trace: every
    # launch holds worlds of one kind; every result equals the request alone
    reqs = []
    for i in range(8):
        kw = dict(H=14, W=18 + i, cap=40, n_init=12, res_init_p=0.4, rate_scale=4.0, T_repr=6, L_max=60)
        if i % 2:
            kw.update(obs_radius=7, hidden=4, controller=1)
        else:
            kw.update(obs_radius=2, hidden=16)
        if i % 4 >= 2:
            kw.update(dynamics=1, E0=120, E_max=120, decay=1, gain=40, E_repr=0, T_repr=12, T_death=15,
                      regrow_pI=0.3, regrow_alpha=200.0, spont=0.01)
        reqs.append(serve.Request(i, arrival=0.0, cfg=workloads.make(**kw), seed=300 + i, steps=10 + 3 * i))
    be = OracleBackend(oracle_lib)
    results, m = serve.Server(be, budget_bytes=10 ** 9, K=5).run(reqs, realtime=False)
    assert len(results) == len(reqs)
    for r in reqs:
        ow = oracle_lib.OracleWorld(oracle_lib.OracleConfig.from_dict(r.cfg), r.seed)
        for _ in range(r.steps):
            ow.step()
        assert results[r.rid]["digest"] == serve.state_digest(ow.state(with_hidden=True, with_theta=True))
