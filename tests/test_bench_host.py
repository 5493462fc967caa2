"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the byte
accounting of the roofline against closed forms, the rows the act kernel reads
for a window, and the check that ties a traffic summary to the kernel sources."""
import importlib.util
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_projection_and_act_bytes_closed_form(bench):
    # hidden 32: W_hh 3*32*32 floats, b_hh and the projection out 3*32 each, h 32
    assert bench.proj_bytes_per_agent({"hidden": 32}) == 4 * (3 * 32 * 32 + 3 * 32 + 32 + 3 * 32)
    # act: gh, b_ih, the energy row and each input row 3*hd floats; head 5*hd + 5;
    # h in and out; 21 bytes of scalars
    hd = 16
    rw = 3 * hd * 4
    for rows in (0.0, 1.0, 24.5):
        want = 3 * rw + (5 * hd + 5) * 4 + rows * rw + 2 * hd * 4 + 21
        assert bench.act_bytes_per_agent({"hidden": hd}, rows) == pytest.approx(want)


def one_agent(H, W, row, col, R):
    return {"R": np.asarray(R, np.int32).reshape(H, W), "row": np.array([row]), "col": np.array([col]),
            "n_live": 1}


def test_rows_read_for_a_window(bench):
    cfg = {"H": 9, "W": 9, "obs_radius": 1}
    # empty grid, agent in the middle: no resource; occupancy 1 (itself) of 9
    nnz, rows = bench.observed_inputs(one_agent(9, 9, 4, 4, np.zeros(81)), cfg)
    assert nnz[0] == 1 and rows[0] == 1
    # full grid: 9 ones in the resource window -> its total minus 0 zero rows
    nnz, rows = bench.observed_inputs(one_agent(9, 9, 4, 4, np.ones(81)), cfg)
    assert nnz[0] == 10 and rows[0] == 1 + 1
    # corner agent: 5 outside cells read occupied (+ itself = 6 of 9 ones ->
    # 3 zero rows + the total), resources only inside (4 ones of 9 -> 4 rows)
    nnz, rows = bench.observed_inputs(one_agent(9, 9, 0, 0, np.ones(81)), cfg)
    assert nnz[0] == 4 + 6 and rows[0] == 4 + (9 - 6 + 1)


def test_traffic_summary_tied_to_sources(bench, tmp_path):
    p = tmp_path / "t.txt"
    p.write_text("# header: not a key\nhbm_bytes_per_launch_rows8: 123.0\nhbm_bytes_per_launch: 456\n"
                 "kernel_source_sha256_16: abc\n")
    assert bench.read_traffic("abc", 8, str(p)) == 123.0
    assert bench.read_traffic("abc", None, str(p)) == 456.0
    assert bench.read_traffic("other", 8, str(p)) is None      # sources changed since the counters
    assert bench.read_traffic("abc", 16, str(p)) is None       # no figure for that variant
    assert bench.read_traffic("abc", 8, str(tmp_path / "missing.txt")) is None
    # the committed summaries carry a hash of the current sources or none at all
    h = bench.kernel_source_hash()
    assert len(h) == 16 and all(ch in "0123456789abcdef" for ch in h)


def test_cpu_baseline_fields(bench, oracle_lib):
    from paper_2302_09334_amd import workloads
    out = bench.cpu_baseline(workloads.WORKLOADS["cfg0"], 0, 0.2)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["unit"] == "agent-steps/s"
    assert out["value"] > 0 and 1 <= out["host_cores"] <= os.cpu_count()
    assert "steps 0.." in out["sample"]


def test_step_bytes_closed_form(bench):
    """Step bytes of the sparse-input count: per acting agent W_hh, both
    biases, the head, h in and out with 40 bytes of scalars, the energy row;
    per input row read 3*hd floats; per birth two genomes; the grid."""
    cfg = {"hidden": 32, "H": 200, "W": 400}
    P = 12933
    hd = 32
    per_agent = 4 * (3 * hd * hd + 3 * hd + 3 * hd + 5 * hd + 5) + 8 * hd + 40 + 4 * 3 * hd
    got = bench.step_algorithmic_bytes(cfg, P, np.array([4608, 4600]), np.array([100000, 0]), np.array([5, 0]))
    want = np.array([4608 * per_agent + 100000 * 384 + 5 * 8 * P, 4600 * per_agent]) + 200 * 400 * 10
    assert np.allclose(got, want)


def test_kernel_window_bytes(bench):
    """The act kernel's bytes are its per-agent bytes without input rows,
    plus the rows the device counted, the children's genomes and the grid;
    the projection splits 4/8 (move) and 4/8 of the survivors (claim)."""
    cfg = {"hidden": 16, "H": 10, "W": 20}
    P = 1000
    kb = bench.kernel_window_bytes(cfg, P, np.array([100, 100]), np.array([1000, 3000]), np.array([2, 0]),
                                   np.array([8, 0]), np.array([1, 3]))
    rw = 3 * 16 * 4
    act = 100 * bench.act_bytes_per_agent(cfg, 0.0) + 2000 * rw + 1 * 8 * P + 200 * 5
    assert kb["act"] == pytest.approx(act)
    pb = bench.proj_bytes_per_agent(cfg)
    assert kb["move"] == pytest.approx(100 * (bench.MOVE_BYTES_PER_AGENT + 4 / 8 * pb))
    claim = 4 / 8 * 96 * pb + 100 * bench.CLAIM_BYTES_PER_AGENT + 2 * bench.CLAIM_BYTES_PER_ELIGIBLE + 2 * 200
    assert kb["claim"] == pytest.approx(claim)


def test_traffic_per_agent_tied_to_sources(bench, tmp_path):
    p = tmp_path / "t.txt"
    p.write_text("hbm_bytes_per_acting_agent_rows8: 12345.5\nkernel_source_sha256_16: abc\n")
    assert bench.read_traffic_per_agent("abc", 8, str(p)) == 12345.5
    assert bench.read_traffic_per_agent("abc", 16, str(p)) is None
    assert bench.read_traffic_per_agent("xyz", 8, str(p)) is None


def test_projection_share_matches_library_default(bench):
    """The bench's split of the projection bytes between the move and claim
    kernels is the library's build default."""
    import re
    src = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2302_09334_amd",
                            "csrc", "kernels.h")).read()
    eighths = int(re.search(r"#define ECO_PROJ_MOVE_EIGHTHS (\d+)", src).group(1))
    assert bench.PROJ_MOVE_SHARE == eighths / 8
