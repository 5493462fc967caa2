"""GPU-vs-oracle parity harness (used by the gpu-marked tests and smoke).

The GPU world runs K steps with its controller log on; the oracle then takes
the same K steps, one at a time, receiving the GPU's actions as near-tie
hints (adopted only where the oracle's own top logits are within 1e-5 of each
other).  Compared: every step's counters (including the sum of ages at death) and
acting uids exactly, the controller logits within 1e-5 * max(1, max|logit|)
per agent, at every chunk end the integer state bit-exactly (with the
previous action and ate bit) and the recurrent state within 1e-5 * max(1, |v|),
and at the end every completed movement window's histogram exactly.
"""
import sys

import numpy as np

STATE_KEYS = ("uid", "row", "col", "energy", "age", "streak")
LOGIT_TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare_state(g, o, where, hidden=True, theta=False):
    assert g["t"] == o["t"], (where, g["t"], o["t"])
    assert g["n_live"] == o["n_live"], (where, g["n_live"], o["n_live"])
    assert g["next_uid"] == o["next_uid"], (where, "next_uid")
    assert np.array_equal(g["R"], o["R"]), (where, "R", int((g["R"] != o["R"]).sum()))
    for k in STATE_KEYS:
        assert np.array_equal(g[k], o[k]), (where, k)
    if hidden and g["n_live"]:
        oh = o["h"].astype(np.float64)
        d = (np.abs(g["h"].astype(np.float64) - oh) / np.maximum(1.0, np.abs(oh))).max()
        assert d <= LOGIT_TOL, (where, "h", d)
        for k in ("last_action", "ate"):
            assert np.array_equal(g[k], o[k]), (where, k)
    if theta and g["n_live"]:
        assert np.array_equal(g["theta"], o["theta"]), (where, "theta")


def run_parity(World, OracleWorld, OracleConfig, cfg, seed, steps, K, mode="kernels", theta_every=0,
               forced=None):
    gw = World(cfg, seed, mode=mode, log_steps=K)
    ow = OracleWorld(OracleConfig.from_dict(cfg), seed)
    if forced is not None:
        gw.set_forced_action(forced)
        ow.set_forced(None, default=forced)
    compare_state(gw.snapshot(hidden=True, theta=True), ow.state(with_hidden=True, with_theta=True),
                  "init", theta=True)
    stats = dict(resyncs=0, max_logit_err=0.0, births=0, deaths=0, agent_steps=0)
    t = 0
    chunk = 0
    while t < steps:
        k = min(K, steps - t)
        gw.step(k)
        gw.sync()
        ctr = gw.counters(t, k)
        for s in range(k):
            log = gw.action_log(t + s)
            info = ow.step(log["uid"], log["action"])
            oc = ow.last_controller()
            assert np.array_equal(log["uid"], oc["uid"]), ("acting uids", t + s)
            if len(oc["uid"]):
                ref = oc["logits"]
                err = np.abs(log["logits"].astype(np.float64) - ref).max(axis=1)
                scale = np.maximum(1.0, np.abs(ref).max(axis=1))
                rel = (err / scale).max()
                stats["max_logit_err"] = max(stats["max_logit_err"], float(rel))
                assert rel <= LOGIT_TOL, ("logits", t + s, rel)
            assert info["mismatches"] == 0, ("action outside the near-tie band", t + s)
            stats["resyncs"] += info["resyncs"]
            stats["births"] += info["births"]
            stats["deaths"] += info["deaths"]
            stats["agent_steps"] += len(oc["uid"])
            for key in ("n_live", "births", "deaths", "eaten", "resources", "claim_wins", "dead_age", "seen"):
                assert ctr[key][s] == info[key], (key, t + s, int(ctr[key][s]), info[key])
        t += k
        chunk += 1
        want_theta = theta_every and chunk % theta_every == 0
        compare_state(gw.snapshot(hidden=True, theta=want_theta),
                      ow.state(with_hidden=True, with_theta=want_theta), f"t={t}", theta=want_theta)
    # movement windows (App. C) that ended, bit-exact
    nw = t // 50
    if nw > 0:
        k0 = max(0, nw - 64)
        gh = gw.move_hist(k0, nw - k0)
        oh = ow.move_hist()[k0:nw]
        assert np.array_equal(gh, oh), ("movement histograms", k0, gh, oh)
        stats["move_windows"] = nw - k0
    gw.close()
    ow.close()
    return stats
