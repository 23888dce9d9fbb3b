"""The GPU path against the stored fixtures of tests/golden/ (written from the oracle alone):
the Philox words bit for bit, and the small European call at equal paths."""
import numpy as np
import pytest

from paper_2402_12111_amd import workloads as W
from test_golden import philox_fixture, reference_fixture

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_12111_amd import simr
    simr.library()
    return simr


def test_gpu_philox_words_equal_the_fixture(S):
    # the debug call takes a 32-bit signed first step (the kernels' step counter); the fixture's
    # all-ones counter is checked against rocRAND on the CPU only
    cases = [c for c in philox_fixture() if c[2] < 2**31]
    assert len(cases) >= 10
    for seed, stream, step, path, words in cases:
        w, _, _ = S.debug_draws(seed, stream, path, 1, step, 1)
        assert [int(x) for x in np.asarray(w).reshape(4)] == words, (seed, stream, step, path)


def test_gpu_european_call_against_the_fixture(S):
    ref = reference_fixture()
    for scheme, name in ((S.SCHEME_QE, "qe"), (S.SCHEME_FTE, "fte")):
        g = S.price(W.option(paths=8192, steps=64, seed=1), scheme)
        key = f"mc_{name}_call_8192x64_seed1"
        assert abs(g.price - ref[key]) <= 1e-4 * 100.0, (name, g.price, ref[key])
        assert g.std_err == pytest.approx(ref[key + "_std_err"], rel=1e-3)
        assert abs(g.price - ref["cf_call"]) <= 3.0 * g.std_err
