"""simr_greeks_batch through the C ABI: a mixed list of European and American options priced
with their adjoint Greeks in one call equals the same options one simr_greeks call at a time,
bit for bit (the same kernels on the same workspace layout, enqueued back to back), and a HIP
failure forced from the host in the middle of a batch reports SIMR_EHIP, leaves the outputs
untouched and leaves the context working."""
import ctypes
import sys

import pytest

from paper_2402_12111_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_12111_amd import simr
    simr.library()
    return simr


def say(*a):
    print(*a, file=sys.stderr, flush=True)


MIXED = [W.option(K=100.0, payoff=W.EURO_PUT, paths=20000, steps=40, seed=4),
         W.option(K=110.0, payoff=W.AMER_PUT, paths=20000, steps=24, seed=7),
         W.option(K=95.0, payoff=W.EURO_CALL, paths=8192 + 37, steps=64, seed=9, stream=3),
         W.option(K=120.0, payoff=W.AMER_PUT, paths=65536, steps=50, seed=5),
         W.option(K=60.0, payoff=W.AMER_PUT, paths=4096, steps=12, seed=2)]  # deep out of the money


def same(a, b):
    """Every field equal: price, standard error, the 7 Greeks and their errors, the LSM flags."""
    return a == b


@pytest.mark.parametrize("scheme", [0, 1, 3])  # QE, full-truncation Euler, truncated Gaussian
def test_batch_equals_single_calls(S, scheme):
    say("greeks batch, scheme", scheme)
    got = S.greeks_batch(MIXED, scheme)
    for o, g in zip(MIXED, got):
        want = S.greeks(o, scheme)
        assert same(g, want), (o, g, want)


def test_batch_of_large_risk_underlyings(S):
    """Four underlyings of the large risk run at 2^18 paths (the 4-path-per-lane induction
    shape is reached at 2^20; 2^18 keeps the test short) against single calls."""
    opts = [dict(o, paths=1 << 18) for o in W.c5_risk(4)]
    got = S.greeks_batch(opts)
    for o, g in zip(opts, got):
        assert same(g, S.greeks(o))


def test_batch_groups_american_inductions(S):
    """Consecutive American options share their induction's cooperative launch: two
    underlyings of the large risk run at full size (2^20 paths x 252 steps: 256-thread blocks,
    16 paths per lane, where a single call takes 1024 x 4), and eight options of 131,072 paths
    (one launch of 256 x 8 where single calls take 1024 x 2).  Every result equals the single
    call's bit for bit."""
    big = W.c5_risk(2)
    small = [dict(o, paths=131072, seed=o["seed"] + 1) for o in W.c5_risk(8)]
    for opts in (big, small):
        got = S.greeks_batch(opts)
        for o, g in zip(opts, got):
            assert same(g, S.greeks(o)), (o, g)


def test_batch_in_the_smallest_workspace(S):
    """A workspace of the largest single option's size (smaller than op 3's) runs the same
    batch one American option at a time, with the same results."""
    L = S.library()
    opts = S._as_options(W.c5_risk(2))
    n = len(opts)
    c_opts = (S._Option * n)(*[o._c() for o in opts])
    prm = S._Params(0, 16, 0, 0)
    small = S.workspace_size(2, [opts[0]], 0, 16)
    assert small < S.workspace_size(3, opts, 0, 16)
    ws = S.workspace(small)
    out = (S._GreeksResult * n)()
    rc = L.simr_greeks_batch(S.context(), c_opts, n, ctypes.byref(prm), out, ctypes.c_void_p(ws.data_ptr()),
                             small, S._stream())
    assert rc == 0, L.simr_last_error()
    want = S.greeks_batch(W.c5_risk(2))
    for r, w in zip(out, want):
        assert (r.price, r.std_err, list(r.g), list(r.g_se)) == (w.price, w.std_err, list(w.grads), list(w.grad_se))


def test_fault_in_the_middle_of_a_batch(S):
    L = S.library()
    opts = S._as_options(MIXED)
    n = len(opts)
    c_opts = (S._Option * n)(*[o._c() for o in opts])
    prm = S._Params(0, 16, 0, 0)
    ws = S.workspace(S.workspace_size(3, opts, 0, 16))
    want = S.greeks_batch(MIXED)
    # launches of the first and the third option; of the group of the last two (27 in all:
    # 4 + 7 + 4 + 12), its shared induction and the finish of its first option's Greeks
    for nth in (3, 12, 22, 25):
        out = (S._GreeksResult * n)()
        for r in out:
            r.price = -7.25
        fired0 = S.debug_fault(2, nth)
        rc = L.simr_greeks_batch(S.context(), c_opts, n, ctypes.byref(prm), out, ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel(), S._stream())
        fired1 = S.debug_fault(0)
        say("fault at launch", nth, "rc", rc, L.simr_last_error().decode())
        assert rc == -3 and b"injected" in L.simr_last_error() and fired1 == fired0 + 1
        assert all(r.price == -7.25 for r in out)
        again = S.greeks_batch(MIXED)
        assert all(same(a, b) for a, b in zip(again, want))
