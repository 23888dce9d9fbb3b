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


def test_measured_constants_match_a_committed_counter_summary():
    """The HBM bytes and VALU instructions the bench reports per launch come from a committed
    counter summary of the same kernel sources: the summary names the digest, and its rows give
    the bench's figures.  With no summary of the current sources the bench reports none."""
    import glob
    if not bench.TRAFFIC_SOURCES_DIGEST:
        assert bench.TRAFFIC_BYTES == {} and bench.VALU_ISSUE_QUADS == {}
        return
    texts = [open(p).read() for p in glob.glob(os.path.join(ROOT, "profiles", "*counters*.md"))]
    mine = [t for t in texts if re.search(r"`([0-9a-f]{16})`", t) and
            re.search(r"`([0-9a-f]{16})`", t).group(1) == bench.TRAFFIC_SOURCES_DIGEST]
    assert mine, "no committed counter summary names the bench's source digest"
    text = "\n".join(mine)
    for key, nbytes in bench.TRAFFIC_BYTES.items():
        assert f"{nbytes:.4e}" in text, (key, nbytes)
    for key, quads in bench.VALU_ISSUE_QUADS.items():
        assert f"{quads:.4e}" in text, (key, quads)
