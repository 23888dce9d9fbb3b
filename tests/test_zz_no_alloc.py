"""The allocation-free entry point, simr_price_noalloc, through the C ABI against simr_price
(the entry point whose kernels it shares) and the FP64 oracle.

Two calls in a row, the second on a smaller option, so the second call finds the first call's
contents in the shared static scratch: both must equal simr_price on the same context bit for
bit (the same kernels on the same tile, the queue counter cleared by a kernel each call) and be
within 1e-4 * S0 of the oracle at equal paths.  Sizes beyond the scratch and American options
are refused before any launch."""
import sys

import pytest

import oracle
from paper_2402_12111_amd import workloads as W

pytestmark = pytest.mark.gpu

PRICE_TOL = 1e-4  # x S0


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


@pytest.mark.parametrize("scheme", [0, 3])  # QE; truncated Gaussian (its table made by simr_create)
def test_noalloc_equals_price_on_two_calls_second_smaller(S, scheme):
    big = W.option(K=105.0, paths=200003, steps=64, seed=21)
    small = W.option(K=95.0, payoff=W.EURO_PUT, paths=3001, steps=16, seed=22, kappa=2.5, xi=0.6)
    say("noalloc scheme", scheme)
    want_big = S.price(big, scheme)      # tunes this context's tile for the scheme
    want_small = S.price(small, scheme)
    got_big = S.price_noalloc(big, scheme)
    got_small = S.price_noalloc(small, scheme)
    for got, want, o in ((got_big, want_big, big), (got_small, want_small, small)):
        assert got.price == want.price and got.std_err == want.std_err and got.paths == want.paths, (got, want)
        r, se, _ = oracle.price_european(oracle.Option(**o, scheme=scheme))
        assert abs(got.price - r) <= PRICE_TOL * o["S0"], (got.price, r)
        assert got.std_err == pytest.approx(se, rel=1e-3)


def test_noalloc_refuses_what_the_scratch_cannot_hold(S):
    from paper_2402_12111_amd.simr import SimrError
    block, ppl = S.get_tile()
    tile = (block or 256) * (ppl or 1)
    too_many = W.option(paths=131072 * tile + 1, steps=2)
    with pytest.raises(SimrError) as e:
        S.price_noalloc(too_many)
    assert e.value.status == -1 and "131072 tiles" in str(e.value)
    with pytest.raises(SimrError) as e:
        S.price_noalloc(W.option(K=110.0, payoff=W.AMER_PUT, paths=4096, steps=8))
    assert e.value.status == -4
    # the refusals launched nothing: a normal call right after still equals simr_price
    o = W.option(paths=5000, steps=8, seed=23)
    want = S.price(o)
    assert S.price_noalloc(o).price == want.price
