"""The C-ABI library loads and exports every symbol include/world.h declares;
its pure host functions (sizes, dimensions, threshold table, config checks)
work without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def wlib():
    from paper_2302_09334_amd import world
    if not os.path.exists(world.LIB_PATH):
        from paper_2302_09334_amd import build
        build.build()
    return world


def header_symbols():
    text = open(os.path.join(ROOT, "include", "world.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(world_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(wlib):
    syms = header_symbols()
    assert len(syms) >= 15
    raw = ctypes.CDLL(wlib.LIB_PATH)
    for s in syms:
        assert hasattr(raw, s), s
    assert sorted(wlib.EXPORTS) == syms


def test_required_bytes_and_dims(wlib):
    from paper_2302_09334_amd import workloads
    for name, cfg in workloads.WORKLOADS.items():
        n = wlib.required_bytes(cfg)
        n_in, P = wlib.dims(cfg)
        if cfg.get("controller", 0) == wlib.CTRL_CNN_LSTM:
            assert (n_in, P) == (15 * 15 * 3, 2445)
            assert cfg["cap"] * P * 4 < n < cfg["cap"] * ((P + 64) * 4 + 1024) + 64 * cfg["H"] * cfg["W"] + (1 << 20)
            continue
        assert n_in == 2 * (2 * cfg["obs_radius"] + 1) ** 2 + 1
        # the genome dominates the arena: per agent slot the genome, three more
        # rows of 3*hidden floats (the two window totals and a zero row), up to
        # 64 floats of row padding, and under 1 KiB of records and state
        assert n > cfg["cap"] * P * 4
        per_slot = (P + 9 * cfg["hidden"] + 64) * 4 + 1024
        assert n < cfg["cap"] * per_slot + 64 * cfg["H"] * cfg["W"] + (1 << 20)
    assert wlib.dims(workloads.WORKLOADS["m1_4k"]) == (99, 12933)
    assert wlib.dims(workloads.WORKLOADS["cfg0"]) == (51, 3397)


@pytest.mark.parametrize("bad,code", [(dict(H=1), -2), (dict(hidden=24), -2), (dict(obs_radius=4), -2),
                                      (dict(n_init=300, cap=256), -2), (dict(E0=0), -2),
                                      (dict(cap=0), -2), (dict(T_repr=0), -2), (dict(controller=2), -2),
                                      (dict(controller=1), -2), (dict(controller=1, obs_radius=7), -2),
                                      (dict(controller=1, hidden=4), -2)])
def test_invalid_configs(wlib, bad, code):
    from paper_2302_09334_amd import workloads
    cfg = dict(workloads.WORKLOADS["cfg0"])
    cfg.update(bad)
    with pytest.raises(wlib.WorldError) as ei:
        wlib.required_bytes(cfg)
    assert ei.value.code == code


def test_threshold_table_matches_oracle(wlib, oracle_lib):
    """The library builds its own regrowth table; it must equal the oracle's
    (both evaluate the same double-precision expression)."""
    from paper_2302_09334_amd import workloads
    for name in ("cfg0", "m1_4k", "cfg2", "paper1k"):
        cfg = workloads.WORKLOADS[name]
        a = wlib.threshold_table(cfg)
        b = oracle_lib.threshold_table(oracle_lib.OracleConfig.from_dict(cfg))
        assert np.array_equal(a, b), name
    for m in workloads.batch_manifest(8):
        cfg = m["cfg"]
        assert np.array_equal(wlib.threshold_table(cfg),
                              oracle_lib.threshold_table(oracle_lib.OracleConfig.from_dict(cfg)))


def test_network_config_accepted(wlib):
    from paper_2302_09334_amd import workloads
    cfg = dict(workloads.WORKLOADS["cfg0"], controller=1, obs_radius=7, hidden=4)
    assert wlib.dims(cfg) == (675, 2445)
    assert wlib.required_bytes(cfg) > 0


def header_prototypes():
    """name -> parameter list of every call include/world.h declares."""
    text = open(os.path.join(ROOT, "include", "world.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for m in re.finditer(r"\b(world_[a-z_]+)\s*\(([^)]*)\)\s*;", text):
        params = [p.strip() for p in m.group(2).split(",") if p.strip() and p.strip() != "void"]
        out[m.group(1)] = params
    return out


def test_binding_signatures_match_header(wlib):
    """The binding marshals exactly the parameters the header declares."""
    protos = header_prototypes()
    L = wlib.lib()
    assert set(protos) == set(wlib.EXPORTS)
    for name, params in protos.items():
        assert len(getattr(L, name).argtypes) == len(params), (name, params)
    assert protos["world_required_bytes"][-1].endswith("*snapshot_bytes")
    assert "float *margin" in protos["world_action_log"]
    assert protos["world_set_forced_actions"] == ["world_t *w", "const int32_t *act_by_uid", "int32_t n",
                                                  "int32_t default_action"]


def test_snapshot_bytes(wlib):
    """world_required_bytes reports the host bytes of a full image at capacity:
    the grid, six int32 agent arrays, the recurrent state, the genome and two
    byte arrays per slot."""
    from paper_2302_09334_amd import workloads
    for name in ("cfg0", "m1_4k", "net_m1_4k", "paper1k"):
        cfg = workloads.WORKLOADS[name]
        _, P = wlib.dims(cfg)
        want = cfg["H"] * cfg["W"] + cfg["cap"] * (6 * 4 + 4 * wlib.state_size(cfg) + 4 * P + 2)
        assert wlib.snapshot_bytes(cfg) == want, name
    c = wlib.make_config(workloads.WORKLOADS["cfg0"])
    assert wlib.lib().world_required_bytes(ctypes.byref(c), None, None) == -1


def test_null_handles_rejected(wlib):
    """Every call that takes a world rejects NULL with WORLD_E_INVALID_ARG."""
    L = wlib.lib()
    assert L.world_step(None, 1) == -1
    assert L.world_set_forced_actions(None, None, 0, -1) == -1
    assert L.world_set_forced_action(None, 0) == -1
    assert L.world_step_many(None, 0, 1) == -1
    assert L.world_sync(None) == -1
    assert L.world_destroy(None) == 0
