"""Error paths of the library on the GPU, forced from the host: the context's fault plan makes
its nth HIP allocation, launch or copy/synchronisation report a failure (no kernel is affected,
every kernel that was launched runs to its normal end).  The call that meets the fault returns
SIMR_EHIP with its host outputs untouched; the next call on the same context gives the same
result as before, bit for bit."""
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


SENTINEL = -7.25


def raw_call(S, ctx, op, o, scheme=0):
    """One C-ABI call with sentinel-filled outputs: (status, output struct)."""
    L = S.library()
    c_opt = S.Option.from_dict(o)._c()
    prm = S._Params(scheme, 16 if op == "greeks" else 0, 0, 0)
    ws = S.workspace(S.workspace_size(2 if op == "greeks" else 0, [o], scheme, 16 if op == "greeks" else 0))
    if op == "greeks":
        out = S._GreeksResult()
        out.price = out.std_err = SENTINEL
        for i in range(7):
            out.g[i] = out.g_se[i] = SENTINEL
        rc = L.simr_greeks(ctx, ctypes.byref(c_opt), ctypes.byref(prm), ctypes.byref(out),
                           ctypes.c_void_p(ws.data_ptr()), ws.numel(), S._stream())
    else:
        out = S._Result(SENTINEL, SENTINEL, -7, -7, 0)
        rc = L.simr_price(ctx, ctypes.byref(c_opt), ctypes.byref(prm), ctypes.byref(out),
                          ctypes.c_void_p(ws.data_ptr()), ws.numel(), S._stream())
    return rc, out


def untouched(op, out):
    if op == "greeks":
        return out.price == SENTINEL and out.std_err == SENTINEL and all(out.g[i] == SENTINEL for i in range(7))
    return out.price == SENTINEL and out.std_err == SENTINEL and out.paths == -7


def values(op, out):
    if op == "greeks":
        return (out.price, out.std_err) + tuple(out.g[i] for i in range(7))
    return (out.price, out.std_err, out.paths, out.lsm_flags)


CASES = [("price", W.option(paths=20000, steps=32)),
         ("price", W.option(K=110.0, payoff=W.AMER_PUT, paths=20000, steps=24, seed=7)),
         ("greeks", W.option(K=100.0, payoff=W.EURO_PUT, paths=20000, steps=40, seed=4)),
         ("greeks", W.option(K=110.0, payoff=W.AMER_PUT, paths=20000, steps=24, seed=7))]


@pytest.fixture(autouse=True)
def disarmed(S):
    """Whatever a test does, the shared context leaves it with no fault armed."""
    yield
    S.debug_fault(0)


@pytest.mark.parametrize("kind", [2, 3])  # launches; copies and synchronisations
@pytest.mark.parametrize("case", range(len(CASES)))
def test_injected_fault_at_every_call_site(S, kind, case):
    """Every launch (or copy/synchronisation) of the call in turn fails: the status is
    SIMR_EHIP naming the injected failure, the outputs keep their sentinels, the plan fires
    once; then an unarmed call returns exactly the result of the call before the faults."""
    op, o = CASES[case]
    ctx = S.context()
    L = S.library()
    rc, ref = raw_call(S, ctx, op, o)
    assert rc == 0
    want = values(op, ref)
    seen = 0
    for nth in range(1, 40):
        fired0 = S.debug_fault(kind, nth)
        rc, out = raw_call(S, ctx, op, o)
        fired1 = S.debug_fault(0)
        if rc == 0:  # the call has fewer than nth such sites: nothing fired, result unchanged
            assert fired1 == fired0 and values(op, out) == want
            break
        say(op, case, "kind", kind, "site", nth, L.simr_last_error().decode())
        assert rc == -3 and b"injected" in L.simr_last_error()
        assert fired1 == fired0 + 1
        assert untouched(op, out)
        rc, out = raw_call(S, ctx, op, o)
        assert rc == 0 and values(op, out) == want, (nth, values(op, out), want)
        seen += 1
    assert seen >= 2, seen  # every call has several launches and copies


def test_injected_fault_in_a_captured_batch(S):
    """On a non-default stream the European batch is captured into a graph: a failing launch
    during the capture discards it, a failing graph launch leaves the graph for the next call,
    and the results after either equal those before."""
    import torch
    opts = W.c3_batch(path_cap=2000)[:12]
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        want = [(r.price, r.std_err) for r in S.price_batch(opts)]
        for nth in range(1, 8):
            fired0 = S.debug_fault(2, nth)
            try:
                got = S.price_batch(opts)
                assert S.debug_fault(0) == fired0
                assert [(r.price, r.std_err) for r in got] == want
                break
            except S.SimrError as e:
                assert e.status == -3 and "injected" in str(e)
                assert S.debug_fault(0) == fired0 + 1
            got = S.price_batch(opts)
            assert [(r.price, r.std_err) for r in got] == want
        st.synchronize()


def test_injected_allocation_failure_on_a_new_context(S):
    """A fresh context's first call allocates its pinned staging: that allocation fails, the
    call reports it, and the next call allocates it and prices as the shared context does."""
    L = S.library()
    o = W.option(paths=8192, steps=16)
    want = S.price(o)
    blk, ppl = S.get_tile()
    h = ctypes.c_void_p()
    import torch
    assert L.simr_create(ctypes.byref(h), torch.cuda.current_device()) == 0
    try:
        assert L.simr_set_tile(h, blk, ppl) == 0  # no autotuning on the new context
        fired = ctypes.c_int64()
        assert L.simr_debug_fault(h, 1, 1, ctypes.byref(fired)) == 0 and fired.value == 0
        rc, out = raw_call(S, h, "price", o)
        assert rc == -3 and b"injected alloc failure" in L.simr_last_error() and untouched("price", out)
        rc, out = raw_call(S, h, "price", o)
        assert rc == 0 and out.price == want.price and out.std_err == want.std_err
        assert L.simr_debug_fault(h, 0, 0, ctypes.byref(fired)) == 0 and fired.value == 1
    finally:
        L.simr_destroy(h)
