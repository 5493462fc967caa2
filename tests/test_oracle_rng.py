"""Pins of the oracle's random primitives (not the GPU path).

* Philox4x32-10 (Salmon et al., SC'11) against rocRAND's engine, an
  independent implementation, on random counters and keys.
* The single-precision Box-Muller normal: the logarithm and the sine/cosine
  exhaustively over every input the generator can produce (2^24 each) against
  numpy's float64 functions; the resulting deviates against N(0, 1).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("rocRAND headers / hipcc not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rr")
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-I/opt/rocm/include", "-O1",
                    os.path.join(HERE, "helpers", "rocrand_philox_ref.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(oracle_lib, rocrand_ref):
    rng = np.random.default_rng(123)
    n = 20000
    rec = rng.integers(0, 2**32, size=(n, 6), dtype=np.uint64).astype(np.uint32)
    rec[:4] = 0
    rec[4:8] = 0xFFFFFFFF
    # counters shaped like the simulator's (entity, step, stream, block)
    rec[8:1000, 0] = np.arange(992)
    rec[8:1000, 1] = 7
    rec[8:1000, 2] = 4
    rec[8:1000, 3] = 0
    out = subprocess.run([rocrand_ref], input=rec.tobytes(), capture_output=True, check=True).stdout
    ref = np.frombuffer(out, np.uint32).reshape(n, 4)
    got = np.concatenate([oracle_lib.philox(rec[i:i + 1, :4], rec[i, 4:6]) for i in range(0, 1000)]
                         + [_batched(oracle_lib, rec[1000:])])
    assert np.array_equal(got, ref)


def _batched(oracle_lib, rec):
    # group by key to use the vectorised entry point
    out = np.empty((rec.shape[0], 4), np.uint32)
    for i in range(rec.shape[0]):
        out[i] = oracle_lib.philox(rec[i:i + 1, :4], rec[i, 4:6])[0]
    return out


def test_philox_uniform_bytes(oracle_lib):
    ctr = np.zeros((1 << 16, 4), np.uint32)
    ctr[:, 0] = np.arange(1 << 16)
    ctr[:, 2] = 7
    out = oracle_lib.philox(ctr, [1, 0])
    b = out.view(np.uint8).ravel()
    counts = np.bincount(b, minlength=256)
    chi2, p = stats.chisquare(counts)
    assert p > 1e-4
    # adjacent counters are not correlated
    x = out[:, 0].astype(np.float64)
    r = np.corrcoef(x[:-1], x[1:])[0, 1]
    assert abs(r) < 0.02


def test_ln_unit_exhaustive(oracle_lib):
    k = np.arange(1, 2**24 + 1, dtype=np.float64)
    u = (k * 2.0**-24).astype(np.float32)
    got = oracle_lib.ln_unit(u).astype(np.float64)
    ref = np.log(u.astype(np.float64))
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    assert got[-1] == 0.0  # ln 1
    ulp[-1] = 1.0
    # faithful: measured 0.835 ulp at most (the leading term f = m - 1 is
    # exact; only the correction f^2/2 - s (f^2/2 + R) is rounded)
    e = np.abs(got - ref) / ulp
    assert e.max() < 1.0


def test_ln_positive_floats(oracle_lib):
    """The Gumbel draw takes the logarithm of -ln u in [2^-24 (about), 16.7]:
    every 61st float from 2^-24 to 17 (about 4 million) within 1 ulp."""
    lo = np.array([2.0 ** -24], np.float32).view(np.uint32)[0]
    hi = np.array([17.0], np.float32).view(np.uint32)[0]
    x = np.arange(lo, hi + 1, 61, dtype=np.uint32).view(np.float32)
    got = oracle_lib.ln_unit(x).astype(np.float64)
    ref = np.log(x.astype(np.float64))
    nz = ref != 0.0
    ulp = np.spacing(np.abs(ref[nz]).astype(np.float32)).astype(np.float64)
    assert (np.abs(got[nz] - ref[nz]) / ulp).max() < 1.0
    assert (got[~nz] == 0.0).all()


def test_sincos_2pi_exhaustive(oracle_lib):
    k = np.arange(0, 2**24, dtype=np.float64)
    u = (k * 2.0**-24).astype(np.float32)
    s, c = oracle_lib.sincos_2pi(u)
    ang = 2 * np.pi * k * 2.0**-24
    for got, ref in ((s, np.sin(ang)), (c, np.cos(ang))):
        err = np.abs(got.astype(np.float64) - ref)
        assert err.max() <= 2.0 * 2.0**-24
        m = np.abs(ref) > 2.0**-10
        ulp = np.spacing(np.abs(ref[m]).astype(np.float32)).astype(np.float64)
        assert (err[m] / ulp).max() <= 2.0   # measured 1.93
    # exact special angles
    assert s[0] == 0 and c[0] == 1
    q = 2**22
    assert c[q] == 0 and s[q] == 1 and s[2 * q] == 0 and c[2 * q] == -1 and s[3 * q] == -1


def test_gauss_is_standard_normal(oracle_lib):
    ctr = np.zeros((1 << 18, 4), np.uint32)
    ctr[:, 0] = np.arange(1 << 18)
    ctr[:, 2] = 6
    r = oracle_lib.philox(ctr, [5, 9])
    z0, z1 = oracle_lib.gauss_pair(r[:, 0], r[:, 1])
    z = np.concatenate([z0, z1]).astype(np.float64)
    assert abs(z.mean()) < 0.005
    assert abs(z.std() - 1.0) < 0.005
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # the two halves of a pair are uncorrelated
    assert abs(np.corrcoef(z0, z1)[0, 1]) < 0.01
    # largest possible deviate: u1 = 2^-24 -> r = sqrt(48 ln 2)
    a0, a1 = oracle_lib.gauss_pair(np.array([0], np.uint32), np.array([0], np.uint32))
    assert abs(a0[0] - np.sqrt(-2 * np.log(2.0**-24))) < 1e-5 and a1[0] == 0.0
