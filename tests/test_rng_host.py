"""The library's random-number header (csrc/rng.h), compiled for the host,
against the oracle's primitives, bit for bit: ln over all 2^24 uniform
inputs and about 4 million positive floats (the range of a Gumbel draw's
second logarithm), 2^20 Box-Muller pairs and 2^20 Gumbel deviates from
Philox words.  Both sides perform the same IEEE operations in the same
order, written separately; the GPU test test_primitives_bit_exact repeats
the comparison with the device build.  No GPU is used."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
N_PAIRS = 1 << 20
N_WORDS = 1 << 20


@pytest.fixture(scope="module")
def host_rng(tmp_path_factory, oracle_lib):
    cc = next((c for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc") if c and os.path.exists(c)), None)
    if cc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("rng") / "rng_host")
    b = subprocess.run([cc, "-std=c++17", "-O2", "--offload-arch=gfx950", "-ffp-contract=off", "-fno-fast-math",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "-I", os.path.join(ROOT, "paper_2302_09334_amd", "csrc"),
                        os.path.join(ROOT, "tests", "helpers", "rng_host_main.cpp"), "-o", exe],
                       capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-3000:]
    ctr = np.zeros((N_PAIRS, 4), np.uint32)
    ctr[:, 0] = np.arange(N_PAIRS)
    ctr[:, 2] = 6
    words = oracle_lib.philox(ctr, [11, 3])
    pairs = np.ascontiguousarray(words[:, :2])
    gw = np.ascontiguousarray(words[:, 2])
    r = subprocess.run([exe, str(N_PAIRS), str(N_WORDS)], input=pairs.tobytes() + gw.tobytes(), capture_output=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return np.frombuffer(r.stdout, np.float32), pairs, gw


def test_ln_matches_oracle(host_rng, oracle_lib):
    out, _, _ = host_rng
    u = (np.arange(1, 2 ** 24 + 1, dtype=np.float64) * 2.0 ** -24).astype(np.float32)
    assert np.array_equal(out[:2 ** 24].view(np.uint32), oracle_lib.ln_unit(u).view(np.uint32))
    lo = np.array([2.0 ** -24], np.float32).view(np.uint32)[0]
    hi = np.array([17.0], np.float32).view(np.uint32)[0]
    x = np.arange(lo, hi + 1, 61, dtype=np.uint32).view(np.float32)
    got = out[2 ** 24:2 ** 24 + x.size]
    assert np.array_equal(got.view(np.uint32), oracle_lib.ln_unit(x).view(np.uint32))


def test_gauss_and_gumbel_match_oracle(host_rng, oracle_lib):
    out, pairs, gw = host_rng
    lo = np.array([2.0 ** -24], np.float32).view(np.uint32)[0]
    hi = np.array([17.0], np.float32).view(np.uint32)[0]
    n_ln = 2 ** 24 + len(range(int(lo), int(hi) + 1, 61))
    z = out[n_ln:n_ln + 2 * N_PAIRS].reshape(-1, 2)
    z0, z1 = oracle_lib.gauss_pair(pairs[:, 0], pairs[:, 1])
    assert np.array_equal(z[:, 0].view(np.uint32), np.asarray(z0, np.float32).view(np.uint32))
    assert np.array_equal(z[:, 1].view(np.uint32), np.asarray(z1, np.float32).view(np.uint32))
    g = out[n_ln + 2 * N_PAIRS:]
    assert g.size == N_WORDS
    assert np.array_equal(g.view(np.uint32), np.asarray(oracle_lib.gumbel(gw), np.float32).view(np.uint32))
