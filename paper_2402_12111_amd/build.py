"""Builds libsimr.so, the gfx950 HIP library, in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsimr.so")
SOURCES = [os.path.join(HERE, "csrc", "simr_kernels.hip"), os.path.join(HERE, "csrc", "simr_api.hip")]
HEADERS = [os.path.join(HERE, "csrc", "simr_device.hpp"), os.path.join(HERE, "csrc", "simr_bk.hpp"),
           os.path.join(HERE, "csrc", "simr_kernels.hpp"),
           os.path.join(ROOT, "include", "simr.h")]

FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
    # no implicit multiply-add contraction: the fused operations are the explicit
    # fmaf calls, so a path recomputed in another kernel (the adjoint) is the same
    # FP32 operation sequence, bit for bit
    "-ffp-contract=off",
    # packed FP32 instructions stay off: plain FP32 VALU code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-const-variable",
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: cannot build the gfx950 library")
    return exe


def build(verbose: bool = False) -> str:
    """Compiles every HIP source into libsimr.so (always rebuilds)."""
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + FLAGS + SOURCES + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    if verbose and r.stderr:
        print(r.stderr)
    os.replace(tmp, LIB)
    return LIB


PROBE_SRC = os.path.join(HERE, "csrc", "valu_issue_probe.hip")
PROBE = os.path.join(HERE, "valu_issue_probe")


def build_probe() -> str:
    """Builds the VALU issue-rate probe (a standalone gfx950 program; see its header)."""
    cmd = [hipcc(), "-O3", "--offload-arch=gfx950", "-std=c++17", "-ffp-contract=off",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", PROBE_SRC, "-o", PROBE]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    return PROBE


if __name__ == "__main__":
    import sys
    print(build_probe() if sys.argv[1:] == ["probe"] else build(verbose=True))
