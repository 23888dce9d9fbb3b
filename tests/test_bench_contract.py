"""The parts of the benchmark's contract that need no GPU: it refuses more than one GPU with a
message and a nonzero status, and the HBM traffic it reports is tied to the kernel sources
the counters were taken on (the committed counter summary names the same source digest and
the same bytes per launch as the constants the benchmark reports; for other sources it
reports none)."""
import os
import re
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_traffic_constants_match_the_committed_counter_summary():
    text = open(os.path.join(ROOT, "profiles", "lsm_risk_step_c2_131072x252_hbm_counters.md")).read()
    assert re.search(r"`([0-9a-f]{16})`", text).group(1) == bench.TRAFFIC_SOURCES_DIGEST
    # the summary's calibrated bytes per launch of the induction kernel are the bench's figure
    row = next(line for line in text.splitlines() if "lsm_persistent_kernel" in line)
    assert float(row.split("|")[5]) == bench.TRAFFIC_BYTES["lsm_backward"]
