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


def test_timed_collects_each_call_and_restores_the_collector():
    """The timing helper returns the mean over its calls, records each call's wall time when
    asked, and leaves the garbage collector as it found it (it pauses it while timing)."""
    import gc
    import time

    class FakeCuda:
        @staticmethod
        def synchronize():
            pass

    class FakeTorch:
        cuda = FakeCuda

    seen = []

    def call():
        seen.append(gc.isenabled())
        time.sleep(0.01)
        return len(seen)

    for enabled in (True, False):
        (gc.enable if enabled else gc.disable)()
        try:
            seen.clear()
            per_call = []
            ms, out = bench.timed(call, 3, FakeTorch, per_call)
            assert out == 3 and seen == [False] * 3 and gc.isenabled() == enabled
            assert len(per_call) == 3 and all(8.0 < t < 500.0 for t in per_call)
            assert abs(ms - sum(per_call) / 3) < 1.0
        finally:
            gc.enable()
