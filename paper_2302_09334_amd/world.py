"""ctypes binding of libworld.so (include/world.h).

Only argument marshalling lives here: every step of the world runs in the
library's HIP kernels.  torch supplies the device arena (a uint8 tensor) and
the HIP stream; the library never allocates world state itself.  If the
library is missing the import of this module fails loudly -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("ECO_WORLD_LIB", os.path.join(HERE, "libworld.so"))

WORLD_OK = 0
ERRORS = {-1: "invalid argument", -2: "invalid config", -3: "buffer too small", -4: "HIP failure",
          -5: "poisoned", -6: "state"}
MODE_KERNELS, MODE_GRAPH = 0, 1
MODES = {"kernels": MODE_KERNELS, "graph": MODE_GRAPH}
SNAP_HIDDEN, SNAP_THETA = 1, 2
CTRL_GRU, CTRL_CNN_LSTM = 0, 1   # GRU + arg-max; the paper's network (App. B.5) + sampling
DYN_BENCH, DYN_PAPER = 0, 1      # the benchmark workloads' rules; the paper's (App. B)
# configuration fields a workload dict may leave out (the benchmark rules' values)
OPTIONAL = {"controller": CTRL_GRU, "dynamics": DYN_BENCH, "E_max": 0, "T_death": 0, "regrow_pI": 0.0,
            "regrow_alpha": 1.0}
NO_ACTION = 5                    # previous action of an agent that has not acted yet


class WorldError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("H", C.c_int32), ("W", C.c_int32), ("cap", C.c_int32),
        ("n_init", C.c_int32), ("obs_radius", C.c_int32), ("hidden", C.c_int32),
        ("res_init_p", C.c_double), ("rate_bottom", C.c_double), ("rate_top", C.c_double),
        ("rate_scale", C.c_double), ("spont", C.c_double),
        ("E0", C.c_int32), ("decay", C.c_int32), ("gain", C.c_int32), ("E_repr", C.c_int32),
        ("T_repr", C.c_int32), ("L_max", C.c_int32),
        ("sigma_mut", C.c_double), ("w_init_gain", C.c_double),
        ("log_steps", C.c_int32), ("flags", C.c_uint32), ("controller", C.c_int32),
        ("dynamics", C.c_int32), ("E_max", C.c_int32), ("T_death", C.c_int32), ("pad", C.c_int32),
        ("regrow_pI", C.c_double), ("regrow_alpha", C.c_double),
    ]


class Counters(C.Structure):
    _fields_ = [("n_live", C.c_int32), ("births", C.c_int32), ("deaths", C.c_int32),
                ("eaten", C.c_int32), ("resources", C.c_int32), ("claim_wins", C.c_int32),
                ("dead_age_sum", C.c_int64), ("seen_resource", C.c_int32), ("rows_read", C.c_int32)]

MOVE_WINDOW = 50   # steps per movement window (App. C)
MOVE_BINS = 17     # distance bins of a movement window


class Image(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("flags", C.c_uint32), ("step", C.c_int64),
        ("n_live", C.c_int32), ("next_uid", C.c_uint32), ("agent_capacity", C.c_int32),
        ("reserved", C.c_int32),
        ("R", C.c_void_p), ("uid", C.c_void_p), ("row", C.c_void_p), ("col", C.c_void_p),
        ("energy", C.c_void_p), ("age", C.c_void_p), ("streak", C.c_void_p),
        ("h", C.c_void_p), ("theta", C.c_void_p), ("last_action", C.c_void_p), ("ate", C.c_void_p),
    ]


# Every symbol include/world.h declares (checked by the ABI test).
EXPORTS = [
    "world_required_bytes", "world_dims", "world_create", "world_step", "world_step_many",
    "world_set_mode", "world_set_tuning", "world_set_stream", "world_sync", "world_snapshot", "world_load", "world_counters_get",
    "world_destroy", "world_last_error", "world_set_forced_action", "world_action_log",
    "world_test_philox", "world_test_gauss", "world_threshold_table", "world_phase_times",
    "world_test_copy", "world_move_hist", "world_test_gumbel", "world_test_stall_lookback",
    "world_set_forced_actions", "world_validate_image", "world_step_many_noalloc",
]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; "
                               "g.build()'` (there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.world_required_bytes.argtypes = [C.POINTER(Config), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
        L.world_dims.argtypes = [C.POINTER(Config), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.world_create.argtypes = [C.POINTER(Config), C.c_uint64, P, C.c_size_t, P, C.POINTER(P)]
        L.world_step.argtypes = [P, C.c_int32]
        L.world_step_many.argtypes = [C.POINTER(P), C.c_int32, C.c_int32]
        L.world_step_many_noalloc.argtypes = [C.POINTER(P), C.c_int32, C.c_int32]
        L.world_set_mode.argtypes = [P, C.c_int32]
        L.world_set_tuning.argtypes = [P, C.c_int32, C.c_int32, C.c_int32]
        L.world_set_stream.argtypes = [P, P]
        L.world_sync.argtypes = [P]
        L.world_snapshot.argtypes = [P, C.POINTER(Image)]
        L.world_load.argtypes = [P, C.POINTER(Image)]
        L.world_counters_get.argtypes = [P, C.c_int64, C.c_int32, P]
        L.world_destroy.argtypes = [P]
        L.world_last_error.argtypes = [P]
        L.world_last_error.restype = C.c_char_p
        L.world_set_forced_action.argtypes = [P, C.c_int32]
        L.world_action_log.argtypes = [P, C.c_int64, C.c_int32, P, P, P, P, C.POINTER(C.c_int32)]
        L.world_set_forced_actions.argtypes = [P, P, C.c_int32, C.c_int32]
        L.world_validate_image.argtypes = [C.POINTER(Config), C.POINTER(Image)]
        L.world_test_philox.argtypes = [P, C.c_size_t, C.c_uint32, C.c_uint32, P, P]
        L.world_test_gauss.argtypes = [P, P, C.c_size_t, P, P, P]
        L.world_threshold_table.argtypes = [C.POINTER(Config), P]
        L.world_phase_times.argtypes = [P, C.c_int32, P]
        L.world_test_copy.argtypes = [P, P, C.c_size_t, P]
        L.world_move_hist.argtypes = [P, C.c_int64, C.c_int32, P]
        L.world_test_gumbel.argtypes = [P, C.c_size_t, P, P]
        L.world_test_stall_lookback.argtypes = [P, C.c_int32, C.c_uint32]
        for name in EXPORTS:
            getattr(L, name).restype = getattr(L, name).restype or C.c_int
        L.world_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc: int, handle=None):
    if rc != WORLD_OK:
        msg = lib().world_last_error(handle)
        raise WorldError(rc, msg.decode() if msg else "")


def make_config(d: dict, log_steps: int = 0) -> Config:
    c = Config()
    c.struct_size = C.sizeof(Config)
    for name, _ in Config._fields_:
        if name in ("struct_size", "log_steps", "flags", "pad"):
            continue
        if name in OPTIONAL:
            setattr(c, name, d.get(name, OPTIONAL[name]))
            continue
        setattr(c, name, d[name])
    c.log_steps = int(d.get("log_steps", log_steps))
    c.flags = 0
    return c


def state_size(cfg: dict) -> int:
    """Recurrent state floats per agent: h (GRU), h then c (LSTM)."""
    return 2 * cfg["hidden"] if cfg.get("controller", CTRL_GRU) == CTRL_CNN_LSTM else cfg["hidden"]


def required_bytes(cfg: dict) -> int:
    n = C.c_size_t()
    c = make_config(cfg)
    _check(lib().world_required_bytes(C.byref(c), C.byref(n), None))
    return int(n.value)


def snapshot_bytes(cfg: dict) -> int:
    """Host bytes of a complete image of a world of this configuration."""
    n = C.c_size_t()
    c = make_config(cfg)
    _check(lib().world_required_bytes(C.byref(c), None, C.byref(n)))
    return int(n.value)


def dims(cfg: dict) -> tuple[int, int]:
    a, b = C.c_int32(), C.c_int32()
    c = make_config(cfg)
    _check(lib().world_dims(C.byref(c), C.byref(a), C.byref(b)))
    return int(a.value), int(b.value)


def threshold_table(cfg: dict) -> np.ndarray:
    out = np.zeros((cfg["H"], 25), np.uint64)
    c = make_config(cfg)
    _check(lib().world_threshold_table(C.byref(c), out.ctypes.data_as(C.c_void_p)))
    return out


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def image_of(cfg: dict, s: dict):
    """A world_image over the arrays of a canonical state dict (the keys of
    World.snapshot(hidden=True, theta=True)); returns (image, arrays to keep
    alive while the image is used)."""
    n = int(s["n_live"])
    P = dims(cfg)[1]
    arrs = {"R": np.ascontiguousarray(s["R"], np.uint8).ravel(), "uid": np.ascontiguousarray(s["uid"], np.uint32)}
    for k in ("row", "col", "energy", "age", "streak"):
        arrs[k] = np.ascontiguousarray(s[k], np.int32)
    arrs["h"] = np.ascontiguousarray(s["h"], np.float32).reshape(n, state_size(cfg))
    arrs["last_action"] = np.ascontiguousarray(s["last_action"], np.uint8)
    arrs["ate"] = np.ascontiguousarray(s["ate"], np.uint8)
    arrs["theta"] = np.ascontiguousarray(s["theta"], np.float32).reshape(n, P)
    img = Image()
    img.struct_size = C.sizeof(Image)
    img.flags = SNAP_HIDDEN | SNAP_THETA
    img.step = int(s["t"])
    img.n_live = n
    img.next_uid = int(s["next_uid"])
    img.agent_capacity = n
    for k, a in arrs.items():
        setattr(img, k, _np_ptr(a))
    return img, arrs


def validate_image(cfg: dict, s: dict):
    """Raise WorldError unless world_load would accept the state dict `s` for
    a world of configuration `cfg` (host only, no device)."""
    img, keep = image_of(cfg, s)
    c = make_config(cfg)
    _check(lib().world_validate_image(C.byref(c), C.byref(img)))
    del keep


class World:
    """One world resident in a torch-allocated device arena."""

    def __init__(self, cfg: dict, seed: int, device: str = "cuda:0", stream=None, mode: str = "kernels",
                 log_steps: int = 0):
        import torch
        self.cfg = dict(cfg)
        self.seed = int(seed)
        self._c = make_config(cfg, log_steps)
        self.log_steps = int(self._c.log_steps)
        nbytes = C.c_size_t()
        _check(lib().world_required_bytes(C.byref(self._c), C.byref(nbytes), None))
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        # torch's caching allocator returns 512-byte aligned blocks
        self.arena = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.nbytes = int(nbytes.value)
        self.n_inputs, self.n_params = dims(cfg)
        h = C.c_void_p()
        _check(lib().world_create(C.byref(self._c), C.c_uint64(self.seed), C.c_void_p(self.arena.data_ptr()),
                                  nbytes.value, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self.set_mode(mode)

    # -- lifecycle -------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().world_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_mode(self, mode: str):
        self.mode = mode
        _check(lib().world_set_mode(self._h, MODES[mode]), self._h)

    def set_stream(self, stream):
        """Move the world to another torch/HIP stream (synchronises the old one)."""
        _check(lib().world_set_stream(self._h, C.c_void_p(stream.cuda_stream)), self._h)
        self.stream = stream

    def set_tuning(self, act_rows: int = 16, act_waves: int | None = None, regrow_tile: int | None = None):
        """Launch shape: act rows per round trip (8, 16, 32), agents per act
        block (2, 4, 8), regrowth tile edge (8, 16, 32); results are identical
        for every choice.  Unnamed knobs keep their current values."""
        self.act_rows = int(act_rows)
        self.act_waves = int(act_waves if act_waves is not None else getattr(self, "act_waves", 4))
        self.regrow_tile = int(regrow_tile if regrow_tile is not None else getattr(self, "regrow_tile", 16))
        _check(lib().world_set_tuning(self._h, self.act_rows, self.act_waves, self.regrow_tile), self._h)

    def step(self, K: int = 1):
        _check(lib().world_step(self._h, int(K)), self._h)

    def sync(self):
        _check(lib().world_sync(self._h), self._h)

    def set_forced_action(self, a: int):
        _check(lib().world_set_forced_action(self._h, int(a)), self._h)

    def set_forced_actions(self, act_by_uid, default: int = -1):
        """Scripted policy: uid u takes act_by_uid[u] when >= 0, else `default`
        (-1 = the controller)."""
        a = np.ascontiguousarray(act_by_uid if act_by_uid is not None else [], np.int32)
        _check(lib().world_set_forced_actions(self._h, _np_ptr(a) if a.size else None, int(a.size), int(default)),
               self._h)

    def test_stall_lookback(self, tile: int, spin_ticks: int = 0):
        """Failure injection: move tile `tile` withholds its look-back word and
        waits end after `spin_ticks` wall-clock ticks (include/world.h)."""
        _check(lib().world_test_stall_lookback(self._h, int(tile), int(spin_ticks)), self._h)

    def phase_times(self, K: int) -> np.ndarray:
        """Run K steps as per-phase kernels timed with HIP events; mean ms per
        step of act (+ child genomes), move, claim (+ regrowth)."""
        ms = np.zeros(3, np.float32)
        _check(lib().world_phase_times(self._h, int(K), _np_ptr(ms)), self._h)
        return ms

    # -- state -----------------------------------------------------------
    def snapshot(self, hidden: bool = False, theta: bool = False) -> dict:
        H, W, cap = self.cfg["H"], self.cfg["W"], self.cfg["cap"]
        out = {"R": np.empty(H * W, np.uint8), "uid": np.empty(cap, np.uint32)}
        for k in ("row", "col", "energy", "age", "streak"):
            out[k] = np.empty(cap, np.int32)
        img = Image()
        img.struct_size = C.sizeof(Image)
        img.flags = (SNAP_HIDDEN if hidden else 0) | (SNAP_THETA if theta else 0)
        img.agent_capacity = cap
        img.R = _np_ptr(out["R"])
        for k in ("uid", "row", "col", "energy", "age", "streak"):
            setattr(img, k, _np_ptr(out[k]))
        if hidden:
            out["h"] = np.empty((cap, state_size(self.cfg)), np.float32)
            out["last_action"] = np.empty(cap, np.uint8)
            out["ate"] = np.empty(cap, np.uint8)
            img.h = _np_ptr(out["h"])
            img.last_action = _np_ptr(out["last_action"])
            img.ate = _np_ptr(out["ate"])
        if theta:
            out["theta"] = np.empty((cap, self.n_params), np.float32)
            img.theta = _np_ptr(out["theta"])
        _check(lib().world_snapshot(self._h, C.byref(img)), self._h)
        n = int(img.n_live)
        res = {"t": int(img.step), "n_live": n, "next_uid": int(img.next_uid), "R": out["R"].reshape(H, W)}
        for k in ("uid", "row", "col", "energy", "age", "streak"):
            res[k] = out[k][:n].copy()
        if hidden:
            for k in ("h", "last_action", "ate"):
                res[k] = out[k][:n].copy()
        if theta:
            res["theta"] = out["theta"][:n].copy()
        return res

    def load(self, s: dict):
        img, keep = image_of(self.cfg, s)
        _check(lib().world_load(self._h, C.byref(img)), self._h)
        del keep

    def counters(self, first: int, n: int) -> dict:
        buf = (Counters * max(n, 1))()
        _check(lib().world_counters_get(self._h, int(first), int(n), C.cast(buf, C.c_void_p)), self._h)
        keys = ("n_live", "births", "deaths", "eaten", "resources", "claim_wins")
        out = {k: np.array([getattr(buf[i], k) for i in range(n)], np.int64) for k in keys}
        out["dead_age"] = np.array([buf[i].dead_age_sum for i in range(n)], np.int64)
        out["seen"] = np.array([buf[i].seen_resource for i in range(n)], np.int64)
        out["rows_read"] = np.array([buf[i].rows_read for i in range(n)], np.int64)
        return out

    def move_hist(self, first: int, n: int) -> np.ndarray:
        """Movement histograms of windows [first, first + n) (App. C): one row
        per window, MOVE_BINS bin counts then the number of agents counted."""
        out = np.zeros((max(n, 0), MOVE_BINS + 1), np.int32)
        _check(lib().world_move_hist(self._h, int(first), int(n), out.ctypes.data_as(C.c_void_p)), self._h)
        return out

    def life_expectancy(self, first: int, n: int) -> float:
        """Mean age at death over steps [first, first + n) (App. C; NaN when no
        agent died)."""
        c = self.counters(first, n)
        d = int(c["deaths"].sum())
        return float(c["dead_age"].sum()) / d if d else float("nan")

    def action_log(self, step: int) -> dict:
        cap = self.cfg["cap"]
        uid = np.empty(cap, np.uint32)
        act = np.empty(cap, np.uint8)
        logits = np.empty((cap, 5), np.float32)
        margin = np.empty(cap, np.float32)
        n = C.c_int32()
        _check(lib().world_action_log(self._h, int(step), cap, _np_ptr(uid), _np_ptr(act), _np_ptr(logits),
                                      _np_ptr(margin), C.byref(n)), self._h)
        k = int(n.value)
        return {"uid": uid[:k].copy(), "action": act[:k].copy(), "logits": logits[:k].copy(),
                "margin": margin[:k].copy()}


def step_many(worlds: list[World], K: int = 1):
    """Advance several worlds (same stream) by K steps in shared launches."""
    arr = (C.c_void_p * len(worlds))(*[w.handle for w in worlds])
    rc = lib().world_step_many(arr, len(worlds), int(K))
    if rc != WORLD_OK:
        _check(rc, worlds[0].handle if rc != -1 else None)


def step_many_noalloc(worlds: list[World], K: int = 1):
    """world_step_many without device allocation (per-phase launches; the
    launch table in the library's fixed device array): for code under graph
    capture or serving loops that must not allocate."""
    arr = (C.c_void_p * len(worlds))(*[w.handle for w in worlds])
    rc = lib().world_step_many_noalloc(arr, len(worlds), int(K))
    if rc != WORLD_OK:
        _check(rc, worlds[0].handle if rc != -1 else None)


def test_copy(src, dst, stream=None):
    """Plain device copy kernel of src into dst (torch tensors, same size)."""
    import torch
    s = stream or torch.cuda.current_stream()
    _check(lib().world_test_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                                 src.numel() * src.element_size(), C.c_void_p(s.cuda_stream)))


def test_philox(ctr, key, stream=None):
    """Philox4x32-10 computed by the device code (test hook)."""
    import torch
    c = torch.as_tensor(np.ascontiguousarray(ctr, np.uint32).view(np.int32)).cuda()
    out = torch.empty_like(c)
    s = stream or torch.cuda.current_stream()
    _check(lib().world_test_philox(C.c_void_p(c.data_ptr()), c.numel() // 4, int(key[0]), int(key[1]),
                                   C.c_void_p(out.data_ptr()), C.c_void_p(s.cuda_stream)))
    return out.cpu().numpy().view(np.uint32).reshape(-1, 4)


def test_gauss(a, b, stream=None):
    """Box-Muller normals computed by the device code (test hook)."""
    import torch
    ta = torch.as_tensor(np.ascontiguousarray(a, np.uint32).view(np.int32)).cuda()
    tb = torch.as_tensor(np.ascontiguousarray(b, np.uint32).view(np.int32)).cuda()
    z0 = torch.empty(ta.numel(), dtype=torch.float32, device=ta.device)
    z1 = torch.empty_like(z0)
    s = stream or torch.cuda.current_stream()
    _check(lib().world_test_gauss(C.c_void_p(ta.data_ptr()), C.c_void_p(tb.data_ptr()), ta.numel(),
                                  C.c_void_p(z0.data_ptr()), C.c_void_p(z1.data_ptr()), C.c_void_p(s.cuda_stream)))
    return z0.cpu().numpy(), z1.cpu().numpy()


def test_gumbel(words, stream=None):
    """Gumbel deviates of the action sampling computed by the device code (test hook)."""
    import torch
    w = torch.as_tensor(np.ascontiguousarray(words, np.uint32).view(np.int32)).cuda()
    g = torch.empty(w.numel(), dtype=torch.float32, device=w.device)
    s = stream or torch.cuda.current_stream()
    _check(lib().world_test_gumbel(C.c_void_p(w.data_ptr()), w.numel(), C.c_void_p(g.data_ptr()),
                                   C.c_void_p(s.cuda_stream)))
    return g.cpu().numpy()
