"""ctypes binding of liboracle.so (the plain CPU reference of the world step).

TEST INFRASTRUCTURE ONLY.  The oracle follows App. B of arXiv 2302.09334
(environment, agents, non-episodic neuroevolution, hyperparameters) in the
parameterisation of the benchmark workloads; see ``oracle.c`` for the
section-by-section readings.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# The planted-mistake test builds edited copies of the source on the side and
# points a child process at them; otherwise these are the committed files.
SRC_PATH = os.environ.get("ORACLE_SRC", os.path.join(HERE, "oracle.c"))
LIB_PATH = os.environ.get("ORACLE_LIB", os.path.join(HERE, "liboracle.so"))


def build(quiet: bool = True) -> str:
    """Compile liboracle.so with the host C compiler (no contraction, no fast-math)."""
    tmp = f"{LIB_PATH}.{os.getpid()}.tmp"   # per process: parallel test workers build at once
    cmd = [
        "gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
        "-Wall", "-Wextra", "-Wno-unused-parameter",
        SRC_PATH, "-o", tmp, "-lm",
    ]
    subprocess.run(cmd, check=True, capture_output=quiet)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Cfg(C.Structure):
    _fields_ = [
        ("H", C.c_int32), ("W", C.c_int32), ("cap", C.c_int32), ("n_init", C.c_int32),
        ("obs_radius", C.c_int32), ("hidden", C.c_int32),
        ("res_init_p", C.c_double), ("rate_bottom", C.c_double), ("rate_top", C.c_double),
        ("rate_scale", C.c_double), ("spont", C.c_double),
        ("E0", C.c_int32), ("decay", C.c_int32), ("gain", C.c_int32),
        ("E_repr", C.c_int32), ("T_repr", C.c_int32), ("L_max", C.c_int32),
        ("sigma_mut", C.c_double), ("w_init_gain", C.c_double), ("controller", C.c_int32),
        ("dynamics", C.c_int32), ("E_max", C.c_int32), ("T_death", C.c_int32), ("pad", C.c_int32),
        ("regrow_pI", C.c_double), ("regrow_alpha", C.c_double),
    ]


DYN_BENCH = 0       # the benchmark workloads' rules
DYN_PAPER = 1       # the paper's rules (App. B): stacking, walls, clip, offspring on the parent's cell
CTRL_GRU = 0        # the benchmark workloads' GRU with arg-max actions
CTRL_CNN_LSTM = 1   # the paper's CNN + LSTM with sampled actions (App. B.5)
NO_ACTION = 5       # previous action of an agent that has not acted yet
MOVE_WINDOW = 50   # steps per movement window (App. C)
MOVE_BINS = 17     # distance bins (distance // 3 for distances 0..50)


class StepInfo(C.Structure):
    _fields_ = [
        ("n_live", C.c_int32), ("births", C.c_int32), ("deaths", C.c_int32),
        ("eaten", C.c_int32), ("resources", C.c_int32), ("resyncs", C.c_int32),
        ("mismatches", C.c_int32), ("claim_wins", C.c_int32), ("dead_age", C.c_int64),
        ("seen", C.c_int32), ("pad", C.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_ if name != "pad"}


@dataclass
class OracleConfig:
    """World parameters (App. B.4, benchmark parameterisation)."""
    H: int
    W: int
    cap: int
    n_init: int
    obs_radius: int = 3
    hidden: int = 32
    res_init_p: float = 0.05
    rate_bottom: float = 0.02
    rate_top: float = 0.002
    rate_scale: float = 1.0
    spont: float = 1e-5
    E0: int = 50
    decay: int = 1
    gain: int = 10
    E_repr: int = 40
    T_repr: int = 20
    L_max: int = 2000
    sigma_mut: float = 0.02
    w_init_gain: float = 0.5
    controller: int = CTRL_GRU
    dynamics: int = 0          # DYN_BENCH or DYN_PAPER
    E_max: int = 0             # paper dynamics: energy clip
    T_death: int = 0           # paper dynamics: steps below E_repr before death
    pad: int = 0
    regrow_pI: float = 0.0     # paper dynamics: p_I of Eq. (1)
    regrow_alpha: float = 1.0  # paper dynamics: alpha of c(x)

    @property
    def state_size(self) -> int:
        """Recurrent state floats per agent: h (GRU), h then c (LSTM)."""
        return 2 * self.hidden if self.controller == CTRL_CNN_LSTM else self.hidden

    def to_c(self) -> _Cfg:
        c = _Cfg()
        for name, _ in _Cfg._fields_:
            setattr(c, name, getattr(self, name))
        return c

    @classmethod
    def from_dict(cls, d: dict) -> "OracleConfig":
        names = {f for f in cls.__dataclass_fields__}
        return cls(**{k: v for k, v in d.items() if k in names})


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.oracle_philox4x32_10.argtypes = [P, P, P, C.c_size_t]
        L.oracle_ln_unit.argtypes = [P, P, C.c_size_t]
        L.oracle_sincos_2pi.argtypes = [P, P, P, C.c_size_t]
        L.oracle_gauss_pair.argtypes = [P, P, P, P, C.c_size_t]
        L.oracle_n_inputs.argtypes = [C.c_int32]
        L.oracle_n_inputs.restype = C.c_int32
        L.oracle_n_params.argtypes = [C.c_int32, C.c_int32]
        L.oracle_n_params.restype = C.c_int32
        L.oracle_threshold_table.argtypes = [C.POINTER(_Cfg), P]
        L.oracle_threshold_table.restype = C.c_int
        L.oracle_gru_eval.argtypes = [C.c_int32, C.c_int32, P, P, P, P, P]
        L.oracle_create.argtypes = [C.POINTER(_Cfg), C.c_uint64, C.c_char_p, C.c_size_t]
        L.oracle_create.restype = P
        L.oracle_destroy.argtypes = [P]
        L.oracle_set_forced.argtypes = [P, P, C.c_int32, C.c_int32]
        L.oracle_step.argtypes = [P, P, P, C.c_int32, C.POINTER(StepInfo)]
        L.oracle_step.restype = C.c_int
        L.oracle_t.argtypes = [P]
        L.oracle_t.restype = C.c_int64
        L.oracle_n_live.argtypes = [P]
        L.oracle_n_live.restype = C.c_int32
        L.oracle_next_uid.argtypes = [P]
        L.oracle_next_uid.restype = C.c_uint32
        L.oracle_get_grid.argtypes = [P, P]
        L.oracle_get_agents.argtypes = [P, P, P, P, P, P, P]
        L.oracle_get_hidden.argtypes = [P, P]
        L.oracle_get_theta.argtypes = [P, P]
        L.oracle_last_n_acted.argtypes = [P]
        L.oracle_last_n_acted.restype = C.c_int32
        L.oracle_get_last_logits.argtypes = [P, P, P, P]
        L.oracle_n_move_windows.argtypes = [P]
        L.oracle_n_move_windows.restype = C.c_int32
        L.oracle_get_move_hist.argtypes = [P, C.c_int32, P, P]
        L.oracle_get_move_hist.restype = C.c_int
        L.oracle_cnn_n_params.restype = C.c_int32
        L.oracle_cnn_n_features.restype = C.c_int32
        L.oracle_cnn_eval.argtypes = [P, P, C.c_int32, C.c_int32, P, P, P, P, P]
        L.oracle_gumbel.argtypes = [P, P, C.c_size_t]
        L.oracle_sample_action.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, P, P]
        L.oracle_sample_action.restype = C.c_int32
        L.oracle_get_recurrent_inputs.argtypes = [P, P, P]
        L.oracle_get_obs_cnn.argtypes = [P, C.c_int32, P]
        L.oracle_get_obs_cnn.restype = C.c_int
        L.oracle_load.argtypes = [P, C.c_int64, C.c_int32, C.c_uint32] + [P] * 11
        L.oracle_load.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- primitives

def philox(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x32-10 blocks for an (n, 4) uint32 array of counters."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, dtype=np.uint32).reshape(2)
    out = np.empty_like(ctr)
    lib().oracle_philox4x32_10(_ptr(ctr), _ptr(k), _ptr(out), ctr.shape[0])
    return out


def ln_unit(u: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float32)
    out = np.empty_like(u)
    lib().oracle_ln_unit(_ptr(u), _ptr(out), u.size)
    return out


def sincos_2pi(u: np.ndarray):
    u = np.ascontiguousarray(u, dtype=np.float32)
    s = np.empty_like(u)
    c = np.empty_like(u)
    lib().oracle_sincos_2pi(_ptr(u), _ptr(s), _ptr(c), u.size)
    return s, c


def gauss_pair(a: np.ndarray, b: np.ndarray):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    b = np.ascontiguousarray(b, dtype=np.uint32)
    z0 = np.empty(a.shape, np.float32)
    z1 = np.empty(a.shape, np.float32)
    lib().oracle_gauss_pair(_ptr(a), _ptr(b), _ptr(z0), _ptr(z1), a.size)
    return z0, z1


def n_inputs(obs_radius: int) -> int:
    return int(lib().oracle_n_inputs(obs_radius))


def n_params(obs_radius: int, hidden: int) -> int:
    return int(lib().oracle_n_params(obs_radius, hidden))


def threshold_table(cfg: OracleConfig) -> np.ndarray:
    out = np.zeros((cfg.H, 25), np.uint64)
    c = cfg.to_c()
    rc = lib().oracle_threshold_table(C.byref(c), _ptr(out))
    if rc != 0:
        raise ValueError("invalid config for the threshold table")
    return out


def gru_eval(n_in: int, hidden: int, theta: np.ndarray, x: np.ndarray, h: np.ndarray):
    theta = np.ascontiguousarray(theta, dtype=np.float32)
    x = np.ascontiguousarray(x, dtype=np.float64)
    h = np.ascontiguousarray(h, dtype=np.float32)
    h_out = np.empty(hidden, np.float64)
    logits = np.empty(5, np.float64)
    lib().oracle_gru_eval(n_in, hidden, _ptr(theta), _ptr(x), _ptr(h), _ptr(h_out), _ptr(logits))
    return h_out, logits


def cnn_n_params() -> int:
    return int(lib().oracle_cnn_n_params())


def cnn_n_features() -> int:
    return int(lib().oracle_cnn_n_features())


def cnn_eval(theta, obs, prev_action: int, ate: int, h, c):
    """The paper's controller in double: (h', c', logits)."""
    theta = np.ascontiguousarray(theta, dtype=np.float32)
    obs = np.ascontiguousarray(obs, dtype=np.float64)
    assert theta.size == cnn_n_params() and obs.size == 15 * 15 * 3
    h = np.ascontiguousarray(h, dtype=np.float32)
    c = np.ascontiguousarray(c, dtype=np.float32)
    ho = np.empty(4, np.float64)
    co = np.empty(4, np.float64)
    lg = np.empty(5, np.float64)
    lib().oracle_cnn_eval(_ptr(theta), _ptr(obs), int(prev_action), int(ate), _ptr(h), _ptr(c),
                          _ptr(ho), _ptr(co), _ptr(lg))
    return ho, co, lg


def gumbel(words) -> np.ndarray:
    w = np.ascontiguousarray(words, dtype=np.uint32)
    g = np.empty(w.shape, np.float32)
    lib().oracle_gumbel(_ptr(w), _ptr(g), w.size)
    return g


def sample_action(seed: int, uid: int, step: int, logits):
    lf = np.ascontiguousarray(logits, dtype=np.float32)
    sc = np.empty(5, np.float32)
    a = lib().oracle_sample_action(C.c_uint64(seed), uid, step, _ptr(lf), _ptr(sc))
    return int(a), sc


# --------------------------------------------------------------------- world

class OracleWorld:
    """One simulated world advanced step by step on the CPU."""

    def __init__(self, cfg: OracleConfig, seed: int):
        self.cfg = cfg
        self.seed = int(seed)
        err = C.create_string_buffer(256)
        c = cfg.to_c()
        self._h = lib().oracle_create(C.byref(c), C.c_uint64(self.seed), err, 256)
        if not self._h:
            raise ValueError(err.value.decode())
        self.P = cnn_n_params() if cfg.controller == CTRL_CNN_LSTM else n_params(cfg.obs_radius, cfg.hidden)

    def close(self):
        if getattr(self, "_h", None):
            lib().oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def set_forced(self, act_by_uid=None, default: int = -1):
        if act_by_uid is None:
            lib().oracle_set_forced(self._h, None, 0, default)
        else:
            a = np.ascontiguousarray(act_by_uid, dtype=np.int32)
            lib().oracle_set_forced(self._h, _ptr(a), a.size, default)

    def step(self, hint_uid=None, hint_act=None) -> dict:
        info = StepInfo()
        if hint_uid is not None and len(hint_uid):
            hu = np.ascontiguousarray(hint_uid, dtype=np.uint32)
            ha = np.ascontiguousarray(hint_act, dtype=np.uint8)
            lib().oracle_step(self._h, _ptr(hu), _ptr(ha), hu.size, C.byref(info))
        else:
            lib().oracle_step(self._h, None, None, 0, C.byref(info))
        return info.as_dict()

    @property
    def t(self) -> int:
        return int(lib().oracle_t(self._h))

    @property
    def n_live(self) -> int:
        return int(lib().oracle_n_live(self._h))

    @property
    def next_uid(self) -> int:
        return int(lib().oracle_next_uid(self._h))

    def grid(self) -> np.ndarray:
        R = np.empty(self.cfg.H * self.cfg.W, np.uint8)
        lib().oracle_get_grid(self._h, _ptr(R))
        return R.reshape(self.cfg.H, self.cfg.W)

    def agents(self) -> dict:
        n = self.n_live
        out = {k: np.empty(n, np.int32) for k in ("row", "col", "energy", "age", "streak")}
        out["uid"] = np.empty(n, np.uint32)
        lib().oracle_get_agents(self._h, _ptr(out["uid"]), _ptr(out["row"]), _ptr(out["col"]),
                                _ptr(out["energy"]), _ptr(out["age"]), _ptr(out["streak"]))
        return out

    def hidden(self) -> np.ndarray:
        """Recurrent state per agent: h (GRU), h then c (LSTM)."""
        h = np.empty((self.n_live, self.cfg.state_size), np.float32)
        lib().oracle_get_hidden(self._h, _ptr(h))
        return h

    def load(self, s: dict):
        """Overwrite the state from a canonical image (the keys of state(with_hidden=True,
        with_theta=True))."""
        n = int(s["n_live"])
        arr = {"R": np.ascontiguousarray(s["R"], np.uint8).ravel(), "uid": np.ascontiguousarray(s["uid"], np.uint32)}
        for k in ("row", "col", "energy", "age", "streak"):
            arr[k] = np.ascontiguousarray(s[k], np.int32)
        arr["h"] = np.ascontiguousarray(s["h"], np.float32).reshape(n, self.cfg.state_size)
        arr["theta"] = np.ascontiguousarray(s["theta"], np.float32).reshape(n, self.P)
        arr["last_action"] = np.ascontiguousarray(s["last_action"], np.uint8)
        arr["ate"] = np.ascontiguousarray(s["ate"], np.uint8)
        rc = lib().oracle_load(self._h, int(s["t"]), n, int(s["next_uid"]),
                               *[_ptr(arr[k]) for k in ("R", "uid", "row", "col", "energy", "age", "streak", "h",
                                                        "theta", "last_action", "ate")])
        if rc != 0:
            raise ValueError("invalid image")

    def recurrent_inputs(self) -> dict:
        """Previous action (NO_ACTION before the first) and ate-in-previous-step bit."""
        n = self.n_live
        la = np.empty(n, np.uint8)
        ate = np.empty(n, np.uint8)
        lib().oracle_get_recurrent_inputs(self._h, _ptr(la), _ptr(ate))
        return {"last_action": la, "ate": ate}

    def obs_cnn(self, a: int) -> np.ndarray:
        """Observation (15, 15, 3) of the paper's controller for live agent a."""
        o = np.empty((15, 15, 3), np.float64)
        rc = lib().oracle_get_obs_cnn(self._h, int(a), _ptr(o))
        if rc != 0:
            raise ValueError("not a paper-controller world or agent out of range")
        return o

    def theta(self) -> np.ndarray:
        th = np.empty((self.n_live, self.P), np.float32)
        lib().oracle_get_theta(self._h, _ptr(th))
        return th

    def move_hist(self) -> np.ndarray:
        """Movement histograms of the windows that have ended (App. C): one row
        per window, MOVE_BINS bin counts then the number of agents counted."""
        k = int(lib().oracle_n_move_windows(self._h))
        out = np.zeros((k, MOVE_BINS + 1), np.int32)
        for i in range(k):
            cnt = C.c_int32(0)
            rc = lib().oracle_get_move_hist(self._h, i, _ptr(out[i]), C.byref(cnt))
            assert rc == 0
            out[i, MOVE_BINS] = cnt.value
        return out

    def last_controller(self) -> dict:
        n = int(lib().oracle_last_n_acted(self._h))
        uid = np.empty(n, np.uint32)
        logits = np.empty((n, 5), np.float64)
        act = np.empty(n, np.uint8)
        lib().oracle_get_last_logits(self._h, _ptr(uid), _ptr(logits), _ptr(act))
        return {"uid": uid, "logits": logits, "action": act}

    def state(self, with_hidden=False, with_theta=False) -> dict:
        s = {"t": self.t, "n_live": self.n_live, "next_uid": self.next_uid, "R": self.grid()}
        s.update(self.agents())
        if with_hidden:
            s["h"] = self.hidden()
            s.update(self.recurrent_inputs())
        if with_theta:
            s["theta"] = self.theta()
        return s
