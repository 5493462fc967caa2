"""Build libworld.so (HIP, gfx950) in-tree with hipcc.

Flags: -O3 for gfx950 only; -ffp-contract=off so that every floating-point
operation that decides an integer (random normals, thresholds) has exactly the
rounding points written in the source (fused multiply-adds are explicit
fmaf calls); packed fp32 instructions are disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libworld.so")
SOURCES = [os.path.join(HERE, "csrc", "world.hip")]
DEPS = [os.path.join(HERE, "csrc", f) for f in ("rng.h", "world_dev.h", "phases.h", "net.h", "kernels.h")]
ARCH = os.environ.get("ECO_OFFLOAD_ARCH", "gfx950")
LIBS = ["-lrocprofiler-sdk-roctx"]   # roctx ranges around the C-ABI calls


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def flags() -> list[str]:
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-ffp-contract=off", "-fno-fast-math",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function",
        "-I", os.path.join(ROOT, "include"),
    ]


def build(verbose: bool = False, out: str = LIB, defines: dict | None = None) -> str:
    """Compile the library to `out`; `defines` are extra -D tuning macros
    (ECO_PROJ_MOVE_EIGHTHS, ECO_PROJ_PER, ECO_PROJ_PER_CLAIM, ECO_NET_WAVES,
    ECO_NET_WAVES_WIDE, ECO_NEWBORN_BLOCKS, ECO_ROWS_STREAM_MIB; none changes a
    result)."""
    tmp = f"{out}.{os.getpid()}.tmp"   # per process
    extra = [f"-D{k}={v}" for k, v in (defines or {}).items()]
    cmd = [hipcc()] + flags() + extra + SOURCES + ["-o", tmp] + LIBS
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose and (res.stdout or res.stderr):
        print(res.stdout + res.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
