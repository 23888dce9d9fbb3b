"""GPU parity of the basket risk Greeks (per-asset vegas in v0 and theta, correlation
sensitivities) through the C ABI against the FP64 oracle on the same seeded paths.

Tolerances: FP32 paths and tangents on the GPU, FP64 in the oracle, the same estimator.  Each
Greek within RISK_TOL of its scale max(|g|, s_g), s_g the per-path standard deviation (the
Greek's natural scale, as for the single-option Greeks; the correlation samples are FP32 sums
over the steps, like the cross-gammas); the price within 1e-4 B_0.  American baskets: the
GPU's own exercise indices, held fixed on both sides.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2402_12111_amd import workloads as W

pytestmark = pytest.mark.gpu

RISK_TOL = 1e-3


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


def compare(b, g, ref, label, tol=RISK_TOL):
    """Worst error over the vegas and correlation sensitivities, in units of their scale."""
    P = b["paths"]
    d = len(b["S0"])
    _, _, vv, vvs, vt, vts, dc, dcs = ref
    worst = 0.0
    for name, got, want, se in (("vega_v0", g.vega_v0, vv, vvs), ("vega_theta", g.vega_theta, vt, vts)):
        for i in range(d):
            scale = max(abs(want[i]), se[i] * math.sqrt(P))
            e = abs(got[i] - want[i]) / scale
            worst = max(worst, e)
            assert e <= tol, (label, name, i, got[i], want[i], scale)
    for i in range(d):
        for j in range(d):
            if i == j:
                assert g.dcorr[i][j] == 0.0
                continue
            scale = max(abs(dc[i, j]), dcs[i, j] * math.sqrt(P))
            e = abs(g.dcorr[i][j] - dc[i, j]) / scale
            worst = max(worst, e)
            assert e <= tol, (label, "dcorr", i, j, g.dcorr[i][j], dc[i, j], scale)
            assert g.dcorr[i][j] == g.dcorr[j][i]
    say(label, "worst error / scale %.2e" % worst)
    return worst


def feller(b, ratio=4.0):
    """The basket with each asset's vol of vol lowered to a Feller ratio 2 kappa theta / xi^2."""
    return dict(b, xi=tuple(math.sqrt(2.0 * k * t / ratio) for k, t in zip(b["kappa"], b["theta"])))


@pytest.mark.parametrize("scheme", [0, 1, 3])  # QE, full-truncation Euler, truncated Gaussian
@pytest.mark.parametrize("d,payoff", [(2, 0), (5, 1), (8, 0)])
def test_basket_risk_european_against_the_oracle(S, scheme, d, payoff):
    """The drawn baskets (vol of vol up to 0.8, most below the Feller condition) for QE and the
    truncated Gaussian step.  Full-truncation Euler's pathwise vega carries d sqrt(v+)/dv =
    1/(2 sqrt(v+)), unbounded as v reaches 0, where FP32 and FP64 paths part (and a step can fall
    on either side of the kink): it is compared on the same baskets with each vol of vol lowered
    to a Feller ratio of 4, as the single-option Euler Greeks are on parameters that meet it."""
    b = W.basket(d, paths=6000 + 37 * d, steps=40, payoff=payoff)  # ragged last block
    if scheme == 1:
        b = feller(b)
    say("basket risk", d, "assets, payoff", payoff, "scheme", scheme)
    g = S.basket_risk(b, scheme)
    ref = oracle.basket_risk_greeks(oracle.Basket(**dict(b, scheme=scheme)))
    B0 = float(np.dot(b["w"], b["S0"]))
    assert abs(g.price - ref[0]) <= 1e-4 * B0, (g.price, ref[0])
    assert g.std_err == pytest.approx(ref[1], rel=1e-3)
    compare(b, g, ref, f"d={d} payoff={payoff} scheme={scheme}")
    # the same paths as the pricing call
    pr = S.basket_price(b, scheme)
    assert g.price == pytest.approx(pr.price, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("scheme", [0, 3])
def test_basket_risk_american_at_the_gpu_policy(S, scheme):
    """American basket put: the GPU holds its own Longstaff-Schwartz exercise indices fixed;
    the oracle's risk Greeks at those indices agree to the same bar, and the price is the LSM
    price of the pricing call."""
    b = W.basket(4, paths=8000, steps=24, seed=17, moneyness=1.1, payoff=W.AMER_PUT)
    g = S.basket_risk(b, scheme)
    lr, tau, _ = S.debug_basket_lsm(b, scheme)
    assert g.price == lr.price and g.lsm_flags == lr.lsm_flags
    ref = oracle.basket_risk_greeks(oracle.Basket(**dict(b, scheme=scheme)), tau=tau)
    compare(b, g, ref, f"american scheme={scheme}")


def test_basket_risk_full_size_8_assets(S):
    """The 8-asset risk workload at full size (262,144 paths x 252 steps): the GPU against the
    oracle on a 20,000-path prefix rerun (counter-based draws make it the same paths).  Over 252
    steps of 8 assets a few asset-paths take the other QE branch in FP32 than in FP64 at a
    near-tie (counted below from the terminal log-prices), and a vega sample carries its variance
    tangent through every later step, so the bar is 3e-3 of the scale here (the single-option
    Greeks take 1e-3 where the exponential branch dominates, 2e-3 for American options)."""
    b = W.basket_risk()[0]
    g = S.basket_risk(b)
    assert all(math.isfinite(x) for x in g.vega_v0 + g.vega_theta)
    sub = dict(b, paths=20000)
    gs = S.basket_risk(sub)
    xT, _, _ = S.debug_basket_paths(sub)
    rx, _, _ = oracle.basket_simulate(oracle.Basket(**sub))
    parted = int((np.abs(xT - rx).max(axis=1) > 1e-3).sum())
    say("paths whose FP32 and FP64 terminal log-prices part by more than 1e-3:", parted)
    compare(sub, gs, oracle.basket_risk_greeks(oracle.Basket(**sub)), "8 assets, 20,000-path prefix", tol=3e-3)
    # the full run's Greeks lie within 4 standard errors of the prefix's (the same estimator)
    for i in range(8):
        assert abs(g.vega_v0[i] - gs.vega_v0[i]) < 4 * math.hypot(g.vega_v0_se[i], gs.vega_v0_se[i])


def test_basket_risk_refusals(S):
    from paper_2402_12111_amd.simr import SimrError
    with pytest.raises(SimrError) as e:
        S.basket_risk(W.basket(9, paths=1000, steps=4))
    assert e.value.status == -4
    with pytest.raises(SimrError) as e:
        S.basket_risk(W.basket(3, paths=1000, steps=4), scheme=2)
    assert e.value.status == -4
