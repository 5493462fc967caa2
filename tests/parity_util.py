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


def new_stats():
    return dict(resyncs=0, max_logit_err=0.0, births=0, deaths=0, agent_steps=0)


def check_chunk(gw, ow, t, k, stats):
    """The oracle takes steps [t, t + k) that the device `gw` has taken (its
    controller log holds them): acting uids and counters exactly, logits
    within the tolerance, actions outside the near-tie band equal."""
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


def run_parity(World, OracleWorld, OracleConfig, cfg, seed, steps, K, mode="kernels", theta_every=0,
               forced=None):
    gw = World(cfg, seed, mode=mode, log_steps=K)
    ow = OracleWorld(OracleConfig.from_dict(cfg), seed)
    if forced is not None:
        gw.set_forced_action(forced)
        ow.set_forced(None, default=forced)
    compare_state(gw.snapshot(hidden=True, theta=True), ow.state(with_hidden=True, with_theta=True),
                  "init", theta=True)
    stats = new_stats()
    t = 0
    chunk = 0
    while t < steps:
        k = min(K, steps - t)
        gw.step(k)
        gw.sync()
        check_chunk(gw, ow, t, k, stats)
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


# --------------------------------------------------------------------------
# Long windows: the device runs ahead while the oracle checks segments in
# parallel worker processes.  At every segment boundary the device's complete
# state (integer state, recurrent state and every genome) is taken; a worker
# loads the start image into a fresh oracle, takes the segment's steps with
# the device's per-step log as near-tie hints, compares every step as
# run_parity does, and at the end compares its state with the device's end
# image: integers and genomes bit-exactly, the recurrent state within the
# logit tolerance.  Each segment thus starts from an image that the previous
# segment's check has matched, so the whole window is compared step by step;
# the only difference from one oracle run is that each segment continues from
# the device's float recurrent state (equal to the oracle's within 1e-5).

COUNTER_KEYS = ("n_live", "births", "deaths", "eaten", "resources", "claim_wins", "dead_age", "seen")


def _worker_init(paths):
    for p in paths:
        if p not in sys.path:
            sys.path.insert(0, p)


def check_segment(cfg, seed, start, logs, end, hists):
    """Oracle check of one segment (runs in a worker process).  `logs`: per
    step (uid, action, logits, counters); `hists`: {absolute window:
    histogram row} of the movement windows inside the segment."""
    import oracle
    ow = oracle.OracleWorld(oracle.OracleConfig.from_dict(cfg), seed)
    ow.load(start)
    t0 = int(start["t"])
    stats = dict(resyncs=0, max_logit_err=0.0, births=0, deaths=0, agent_steps=0, steps=len(logs))
    for s, (uid, act, logits, ctr) in enumerate(logs):
        t = t0 + s
        info = ow.step(uid, act)
        oc = ow.last_controller()
        assert np.array_equal(uid, oc["uid"]), ("acting uids", t)
        if len(oc["uid"]):
            ref = oc["logits"]
            err = np.abs(logits.astype(np.float64) - ref).max(axis=1)
            rel = float((err / np.maximum(1.0, np.abs(ref).max(axis=1))).max())
            stats["max_logit_err"] = max(stats["max_logit_err"], rel)
            assert rel <= LOGIT_TOL, ("logits", t, rel)
        assert info["mismatches"] == 0, ("action outside the near-tie band", t)
        for key in COUNTER_KEYS:
            assert ctr[key] == info[key], (key, t, int(ctr[key]), info[key])
        stats["resyncs"] += info["resyncs"]
        stats["births"] += info["births"]
        stats["deaths"] += info["deaths"]
        stats["agent_steps"] += len(oc["uid"])
    compare_state(end, ow.state(with_hidden=True, with_theta="theta" in end), f"t={t0 + len(logs)}",
                  theta="theta" in end)
    if hists:
        # the oracle lists the windows it closed since the load; the first is
        # the one containing t0 (counting nobody if it began before t0)
        oh = ow.move_hist()
        for k, row in hists.items():
            assert np.array_equal(row, oh[k - t0 // 50]), ("movement histogram", k, row, oh[k - t0 // 50])
    ow.close()
    return stats


def run_parity_segmented(device, cfg, seed, steps, K, seg, workers=None, theta=True, on_segment=None):
    """Compare steps [0, steps) of `device` (a World-like object created from
    (cfg, seed) with a controller log of at least K steps, stepped in chunks
    of K) with the oracle, segment by segment in worker processes.  seg must
    be a multiple of K.  Returns the summed statistics."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import os

    import oracle
    assert seg % K == 0
    ow = oracle.OracleWorld(oracle.OracleConfig.from_dict(cfg), seed)
    start = device.snapshot(hidden=True, theta=True)
    compare_state(start, ow.state(with_hidden=True, with_theta=True), "init", theta=True)
    ow.close()
    here = os.path.dirname(os.path.abspath(__file__))
    n_workers = workers or max(1, min(12, (os.cpu_count() or 2) - 1))
    ctx = mp.get_context("spawn")
    totals = dict(resyncs=0, max_logit_err=0.0, births=0, deaths=0, agent_steps=0, steps=0, segments=0)
    with cf.ProcessPoolExecutor(n_workers, mp_context=ctx, initializer=_worker_init,
                                initargs=([here, os.path.dirname(here)],)) as pool:
        futs = []
        t = 0
        logs = []
        seg_t0 = 0
        while t < steps:
            k = min(K, steps - t)
            device.step(k)
            device.sync()
            ctr = device.counters(t, k)
            for s in range(k):
                lg = device.action_log(t + s)
                logs.append((lg["uid"], lg["action"], lg["logits"], {key: int(ctr[key][s]) for key in COUNTER_KEYS}))
            t += k
            if t % seg == 0 or t == steps:
                end = device.snapshot(hidden=True, theta=theta)
                w0, w1 = (seg_t0 + 49) // 50, t // 50
                hists = {}
                if w1 > w0:
                    rows = device.move_hist(w0, w1 - w0)
                    hists = {w0 + i: rows[i] for i in range(w1 - w0)}
                futs.append(pool.submit(check_segment, cfg, seed, start, logs, end, hists))
                if on_segment:
                    on_segment(seg_t0, t)
                # bounded look-ahead: at most one queued segment per worker
                # (the images of a segment can be hundreds of MB)
                while sum(not f.done() for f in futs) > n_workers:
                    cf.wait([f for f in futs if not f.done()], return_when=cf.FIRST_COMPLETED)
                for f in futs:
                    if f.done() and f.exception() is not None:
                        raise f.exception()
                if not theta:
                    end = device.snapshot(hidden=True, theta=True)
                start, logs, seg_t0 = end, [], t
        for f in futs:
            st = f.result()
            for key in ("resyncs", "births", "deaths", "agent_steps", "steps"):
                totals[key] += st[key]
            totals["max_logit_err"] = max(totals["max_logit_err"], st["max_logit_err"])
            totals["segments"] += 1
    return totals
