"""The CPU code under AddressSanitizer and UndefinedBehaviorSanitizer (host
only; no GPU involved):

* the oracle (plain C) driven through worlds of both rule sets and both
  controllers with births, deaths and a full slot table, forced actions,
  snapshot -> load -> resume against an uninterrupted run (bit-identical),
  rejected images and the primitives at their extreme inputs
  (tests/helpers/oracle_sanitize_main.c), leak detection on;
* the library's host code that touches no device: configuration checks,
  arena layout and sizes, the regrowth threshold tables, image validation
  and world_create's argument checks (tests/helpers/world_host_sanitize_main.cpp;
  the device code is compiled as usual, only the host side is instrumented).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HELPERS = os.path.join(ROOT, "tests", "helpers")


def run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, **kw)


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    b = run(["gcc", "-std=c11", "-g", "-O2", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer", "-ffp-contract=off", "-I", os.path.join(ROOT, "oracle"),
             os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HELPERS, "oracle_sanitize_main.c"), "-o", exe,
             "-lm"])
    assert b.returncode == 0, b.stderr
    r = run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                            UBSAN_OPTIONS="print_stacktrace=1"), timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_library_host_code_under_asan_ubsan(tmp_path):
    cc = hipcc()
    if cc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "world_asan")
    b = run([cc, "-std=c++17", "-g", "-O1", "--offload-arch=gfx950",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all",
             "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "paper_2302_09334_amd", "csrc", "world.hip"),
             os.path.join(HELPERS, "world_host_sanitize_main.cpp"), "-o", exe, "-lrocprofiler-sdk-roctx"])
    assert b.returncode == 0, b.stderr[-3000:]
    r = run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1"),
            timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
