"""Shared pytest set-up: registers the ``gpu`` marker and puts the repository
root on ``sys.path`` so that ``oracle`` and the package import from a checkout."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


KAT_SRC = os.path.join(os.path.dirname(__file__), "kat", "philox_rocrand_kat.cpp")


@pytest.fixture(scope="session")
def rocrand_kat(tmp_path_factory):
    """Host build of the rocRAND Philox header (an independent implementation)."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND header / hipcc not available")
    exe = str(tmp_path_factory.mktemp("kat") / "philox_kat")
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", KAT_SRC, "-o", exe],
                   check=True, capture_output=True)

    def run(tuples):
        inp = "\n".join(f"{s} {st} {n} {p}" for s, st, n, p in tuples) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return np.array([[int(w) for w in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)

    return run
