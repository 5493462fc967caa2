"""The parity comparison has teeth: with a planted mistake in the oracle (an
edited copy of its source, built on the host), a short GPU-vs-oracle run of a
world where that mistake matters fails.  The GPU path runs unchanged; only the
oracle side is wrong.  Every mutant is loaded in this process, as its own
ctypes library, next to the committed oracle."""
import importlib.util
import os
import shutil
import sys

import pytest

from parity_util import run_parity, say
from test_oracle_mutants import MUTANTS, ORACLE_DIR

pytestmark = pytest.mark.gpu


def load_mutant(name, tmp):
    old, new, count, _ = MUTANTS[name]
    src = open(os.path.join(ORACLE_DIR, "oracle.c")).read()
    assert src.count(old) == count
    d = tmp / name
    d.mkdir()
    shutil.copy(os.path.join(ORACLE_DIR, "oracle.h"), d)
    (d / "oracle.c").write_text(src.replace(old, new))
    saved = {k: os.environ.get(k) for k in ("ORACLE_SRC", "ORACLE_LIB")}
    os.environ["ORACLE_SRC"] = str(d / "oracle.c")
    os.environ["ORACLE_LIB"] = str(d / "liboracle.so")
    try:
        modname = f"oracle_mutant_{name}"
        spec = importlib.util.spec_from_file_location(modname, os.path.join(ORACLE_DIR, "oracle.py"))
        mod = importlib.util.module_from_spec(spec)
        sys.modules[modname] = mod
        spec.loader.exec_module(mod)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    mod.build()
    assert mod.LIB_PATH == str(d / "liboracle.so")
    return mod


def gru_world(wl, **kw):
    d = dict(H=30, W=50, cap=300, n_init=200, obs_radius=2, hidden=16, res_init_p=0.3, rate_scale=5.0, T_repr=8,
             L_max=40)
    d.update(kw)
    return wl.make(**d)


def paper_world(wl, **kw):
    d = dict(H=40, W=72, cap=400, n_init=200, obs_radius=7, hidden=4, controller=1, w_init_gain=1.0,
             res_init_p=0.2, E0=120, E_max=120, decay=1, gain=40, E_repr=0, T_repr=25, T_death=30, L_max=650,
             spont=0.002, regrow_pI=0.2, regrow_alpha=200.0, rate_top=0.0, rate_bottom=0.0, dynamics=1)
    d.update(kw)
    return wl.make(**d)


# mutant -> the world in which it must show (steps are short: 60 at most)
CASES = {
    "gru_reset_dropped": gru_world,
    "observe_outside_free": gru_world,
    "move_into_occupied": gru_world,
    "death_age_bound": gru_world,
    "regrowth_latitude_flipped": gru_world,
    "mutation_sigma_doubled": gru_world,
    "claims_when_full": gru_world,   # the world fills its 300 slots by step 8
    "ln_correction_sign": gru_world,   # every child's mutation noise goes through ln
    "paper_any_neighbour": paper_world,
    "lstm_input_forget_swapped": paper_world,
    "temperature_inverted": paper_world,
    "paper_walls_block": paper_world,
}


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    import oracle
    from paper_2302_09334_amd import workloads, world
    return world, oracle, workloads


def test_committed_oracle_passes(env):
    world, oracle, wl = env
    for make in (gru_world, paper_world):
        run_parity(world.World, oracle.OracleWorld, oracle.OracleConfig, make(wl), 3, 60, 20, theta_every=1)


@pytest.mark.parametrize("name", list(CASES))
def test_mutant_fails_parity(env, name, tmp_path):
    world, oracle, wl = env
    mod = load_mutant(name, tmp_path)
    cfg = CASES[name](wl)
    say(f"[teeth] {name}")
    with pytest.raises(AssertionError) as ei:
        run_parity(world.World, mod.OracleWorld, mod.OracleConfig, cfg, 3, 60, 20, theta_every=1)
    say(f"[teeth] {name} caught: {str(ei.value)[:120]}")
