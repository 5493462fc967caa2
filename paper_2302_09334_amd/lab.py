"""Lab environments of arXiv 2302.09334 (Sec. 2.2; measures of App. C).

Evolved agents are taken from a natural-environment run and tested in small
worlds whose resources do not regrow:

* greediness (one agent that cannot reproduce, three resource densities): the
  run is cut into non-overlapping windows of 20 steps; T_r counts the windows in
  which the agent had a resource in its field of view, C_r those in which it
  ate; G = C_r / T_r.  Per agent, an ANOVA over the densities (trials as
  samples) and Tukey's range test between pairs, significance at p < 0.05.
* peer pressure (high density, reproduction on with T_repr = 20): efficiency
  E = resources eaten per individual of the trial, against the same agents
  without reproduction.

Readings where the text is silent: a lab world is 40 x 40 with the agent at
its centre, densities 0.05 / 0.15 / 0.3 (Bernoulli per cell, from the trial's
seed), 400 steps per trial, the agent's memory starts empty, the dynamics
(energy, moves, births) are the world's own; a world that allows reproduction
has 64 slots.  Every lab world is an ordinary world of the library, so all of
them run together in shared launches (`world.step_many`); the per-step
counters (resources seen, eaten, births) give both measures.
"""
from __future__ import annotations

import numpy as np

from . import world as W

LAB_H, LAB_W = 40, 40
WINDOW = 20                       # greediness windows (Sec. 2.2)
DENSITIES = {"low": 0.05, "medium": 0.15, "high": 0.3}
STEPS = 400
T_REPR_LAB = 20                   # reproduction in the peer-pressure lab (Sec. 2.2)
NO_REPRODUCTION = 1 << 30
REPRO_CAP = 64


def lab_config(base: dict, density: float, reproduce: bool) -> dict:
    """World parameters of a lab world derived from the natural world's."""
    c = dict(base)
    c.update(H=LAB_H, W=LAB_W, cap=REPRO_CAP if reproduce else 1, n_init=1, res_init_p=float(density),
             rate_bottom=0.0, rate_top=0.0, spont=0.0, T_repr=T_REPR_LAB if reproduce else NO_REPRODUCTION)
    return c


def evolve(cfg: dict, seed: int, steps: int, stream=None, chunk: int = 100) -> dict:
    """Run the natural environment for `steps` steps; its canonical image."""
    w = W.World(cfg, seed, stream=stream, mode="graph")
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        w.step(k)
        done += k
    snap = w.snapshot(hidden=True, theta=True)
    w.close()
    return snap


def sample_agents(snap: dict, k: int, seed: int = 0) -> np.ndarray:
    """Genomes of k agents drawn without replacement from an image."""
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(int(snap["n_live"]), size=min(k, int(snap["n_live"])), replace=False))
    return np.ascontiguousarray(snap["theta"][idx])


def place_agent(w: "W.World", genome: np.ndarray):
    """Replace the world's population by one agent with `genome` at the centre
    of the grid: energy E0, age 0, empty memory, no previous action."""
    cfg = w.cfg
    s = w.snapshot(hidden=True, theta=True)
    one = lambda v, dt: np.array([v], dt)   # noqa: E731
    img = {"t": s["t"], "n_live": 1, "next_uid": 1, "R": s["R"],
           "uid": one(0, np.uint32), "row": one(cfg["H"] // 2, np.int32), "col": one(cfg["W"] // 2, np.int32),
           "energy": one(cfg["E0"], np.int32), "age": one(0, np.int32), "streak": one(0, np.int32),
           "h": np.zeros((1, W.state_size(cfg)), np.float32), "theta": np.asarray(genome, np.float32)[None],
           "last_action": one(W.NO_ACTION, np.uint8), "ate": one(0, np.uint8)}
    w.load(img)
    return img


def greediness(seen: np.ndarray, eaten: np.ndarray, window: int = WINDOW):
    """G = C_r / T_r from per-step counts of one agent (Sec. 2.2): T_r windows
    with a resource in view, C_r of those with a resource eaten."""
    n = (len(seen) // window) * window
    sw = np.asarray(seen[:n]).reshape(-1, window).max(axis=1) > 0
    ew = np.asarray(eaten[:n]).reshape(-1, window).max(axis=1) > 0
    t_r = int(sw.sum())
    c_r = int((sw & ew).sum())
    return (c_r / t_r if t_r else float("nan")), t_r, c_r


def efficiency(eaten: np.ndarray, births: np.ndarray, n0: int = 1) -> float:
    """Resources eaten per individual of a trial (the initial agents and every
    child born in it)."""
    return float(np.sum(eaten)) / float(n0 + int(np.sum(births)))


def anova_tukey(groups: list[np.ndarray]) -> dict:
    """ANOVA across conditions and Tukey's range test between pairs (App. C)."""
    from scipy import stats
    gs = [np.asarray(g, np.float64)[~np.isnan(np.asarray(g, np.float64))] for g in groups]
    if min(len(g) for g in gs) < 2 or all(np.ptp(g) == 0 for g in gs):
        return {"anova_p": float("nan"), "tukey_p": None}
    f = stats.f_oneway(*gs)
    t = stats.tukey_hsd(*gs)
    return {"anova_p": float(f.pvalue), "tukey_p": np.asarray(t.pvalue).tolist()}


class LabRun:
    """A set of lab worlds (one per (agent, condition, trial)) stepped together."""

    def __init__(self, genomes: np.ndarray, base_cfg: dict, conditions: dict, trials: int, seed0: int = 1000,
                 stream=None, mode: str = "graph", log_steps: int = 0):
        import torch
        self.stream = stream or torch.cuda.Stream()
        self.keys = []
        self.worlds = []
        self.seeds = []
        self.cfgs = []
        self.images = []   # the state each world starts from
        for a, g in enumerate(genomes):
            for name, (density, reproduce) in conditions.items():
                cfg = lab_config(base_cfg, density, reproduce)
                for tr in range(trials):
                    seed = seed0 + (a * 1000 + tr) * 16 + list(conditions).index(name)
                    w = W.World(cfg, seed, stream=self.stream, mode=mode, log_steps=log_steps)
                    self.images.append(place_agent(w, g))
                    self.worlds.append(w)
                    self.keys.append((a, name, tr))
                    self.seeds.append(seed)
                    self.cfgs.append(cfg)
        self.t0 = int(self.worlds[0].snapshot()["t"]) if self.worlds else 0

    def step(self, steps: int, chunk: int = 100):
        done = 0
        while done < steps:
            k = min(chunk, steps - done)
            W.step_many(self.worlds, k)
            done += k

    def sync(self):
        self.worlds[0].sync()

    def counters(self, steps: int) -> list[dict]:
        return [w.counters(self.t0, steps) for w in self.worlds]

    def close(self):
        for w in self.worlds:
            w.close()
        self.worlds = []


def greediness_study(run: LabRun, ctrs: list[dict], n_agents: int) -> dict:
    """Per agent: G per density (trials as samples), ANOVA, Tukey; an agent is a
    sustainable forager when low and high differ significantly with the higher
    greediness at low density (Sec. 2.2)."""
    names = list(DENSITIES)
    per = {(a, n): [] for a in range(n_agents) for n in names}
    for key, c in zip(run.keys, ctrs):
        a, name, _ = key
        if name in DENSITIES:
            per[(a, name)].append(greediness(c["seen"], c["eaten"])[0])
    agents = []
    sustainable = 0
    for a in range(n_agents):
        groups = [np.array(per[(a, n)]) for n in names]
        st = anova_tukey(groups)
        means = [float(np.nanmean(g)) if np.isfinite(g).any() else float("nan") for g in groups]
        sig = st["tukey_p"] is not None and st["anova_p"] < 0.05 and st["tukey_p"][0][2] < 0.05
        if sig and means[0] > means[2]:
            sustainable += 1
        agents.append({"G_mean": dict(zip(names, means)), **st})
    return {"agents": agents, "sustainable_foragers": sustainable,
            "G_mean_by_density": {n: float(np.nanmean([ag["G_mean"][n] for ag in agents])) for n in names}}


def peer_pressure_study(run: LabRun, ctrs: list[dict]) -> dict:
    """Efficiency with and without reproduction at high density (Sec. 2.2)."""
    e = {"off": [], "on": []}
    for key, c in zip(run.keys, ctrs):
        _, name, _ = key
        if name == "high":
            e["off"].append(efficiency(c["eaten"], c["births"]))
        elif name == "high_repro":
            e["on"].append(efficiency(c["eaten"], c["births"]))
    st = anova_tukey([np.array(e["off"]), np.array(e["on"])])
    return {"E_mean_off": float(np.mean(e["off"])), "E_mean_on": float(np.mean(e["on"])),
            "trials": len(e["on"]), "anova_p": st["anova_p"]}


def conditions() -> dict:
    """The three greediness densities and the peer-pressure condition."""
    c = {name: (p, False) for name, p in DENSITIES.items()}
    c["high_repro"] = (DENSITIES["high"], True)
    return c
