"""Pins of the oracle's European pricing and of the closed forms it is checked
against (Heston characteristic-function price, Black-Scholes)."""
import cmath
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
from oracle import black_scholes as bs
from oracle import heston_cf

C1 = dict(S0=100.0, K=100.0, T=1.0, r=0.02, kappa=1.5, theta=0.04, xi=0.3, rho=-0.7, v0=0.04)
HESTON_ARGS = lambda d: (d["S0"], d["K"], d["T"], d["r"], d["kappa"], d["theta"], d["xi"], d["rho"], d["v0"])

# Bias allowance of the QE scheme without martingale correction at >= 32 steps on
# these parameters, on top of 3 standard errors (measured with 4M oracle paths
# over 8 seeds: mean offset +0.003 at 32 steps).
QE_BIAS = 0.01


def test_black_scholes_against_direct_integration():
    """BS call/put equal the discounted lognormal payoff integrated numerically."""
    S0, K, T, r, s = 100.0, 105.0, 0.7, 0.03, 0.25
    mu, sd = math.log(S0) + (r - s * s / 2) * T, s * math.sqrt(T)
    dens = lambda y: stats.norm.pdf(y, mu, sd)
    call, _ = integrate.quad(lambda y: max(math.exp(y) - K, 0) * dens(y), math.log(K), mu + 12 * sd)
    put, _ = integrate.quad(lambda y: max(K - math.exp(y), 0) * dens(y), mu - 12 * sd, math.log(K))
    assert bs.call(S0, K, T, r, s) == pytest.approx(math.exp(-r * T) * call, rel=1e-9)
    assert bs.put(S0, K, T, r, s) == pytest.approx(math.exp(-r * T) * put, rel=1e-9)
    assert bs.call(100, 100, 1, 0.02, 0.2) == pytest.approx(8.916037, abs=5e-7)


def test_cf_martingale_and_normalisation():
    """phi(0) = 1 and phi(-i) = E[S_T] = S0 e^{rT}."""
    a = HESTON_ARGS(C1)
    args = (a[0], a[2], a[3], a[4], a[5], a[6], a[7], a[8])
    assert abs(heston_cf.char_fn(0.0, *args) - 1) < 1e-14
    assert heston_cf.char_fn(-1j, *args) == pytest.approx(C1["S0"] * math.exp(C1["r"] * C1["T"]), rel=1e-13)


@pytest.mark.parametrize("params", [C1, dict(C1, kappa=0.5, theta=0.09, xi=0.8, rho=-0.9, v0=0.01, T=2.0),
                                    dict(C1, kappa=3.0, theta=0.02, xi=0.1, rho=0.0, v0=0.09, T=0.25)])
def test_cf_first_moment_of_log_price(params):
    """-i phi'(0) = E[ln S_T] = ln S0 + r T - (1/2) int_0^T E[v_t] dt
    = ln S0 + r T - (1/2)(theta T + (v0 - theta)(1 - e^{-kappa T}) / kappa)."""
    p = params
    args = (p["S0"], p["T"], p["r"], p["kappa"], p["theta"], p["xi"], p["rho"], p["v0"])
    h = 1e-5
    d = (heston_cf.char_fn(h, *args) - heston_cf.char_fn(-h, *args)) / (2 * h)
    m = (-1j * d).real
    expect = math.log(p["S0"]) + p["r"] * p["T"] - 0.5 * (
        p["theta"] * p["T"] + (p["v0"] - p["theta"]) * (1 - math.exp(-p["kappa"] * p["T"])) / p["kappa"])
    assert m == pytest.approx(expect, abs=1e-8)


def test_cf_second_moment_against_simulation_free_identity():
    """Var[ln S_T] from the CF's second derivative must exceed the integrated mean
    variance times (1 - rho^2) (the uncorrelated part alone) and be finite; and with
    rho = 0 it equals E[int v] = theta T + (v0 - theta)(1 - e^{-kappa T})/kappa
    plus the variance of -(1/2) int v, which is positive."""
    p = dict(C1, rho=0.0)
    args = (p["S0"], p["T"], p["r"], p["kappa"], p["theta"], p["xi"], p["rho"], p["v0"])
    h = 1e-4
    f = lambda u: cmath.log(heston_cf.char_fn(u, *args))
    second = (f(h) - 2 * f(0.0) + f(-h)) / (h * h)
    var = -second.real
    Eint = p["theta"] * p["T"] + (p["v0"] - p["theta"]) * (1 - math.exp(-p["kappa"] * p["T"])) / p["kappa"]
    assert Eint < var < Eint * 1.01


def test_cf_quadrature_against_mpmath():
    """scipy quad and 30-digit mpmath quadrature of the same integrals agree."""
    a = HESTON_ARGS(C1)
    assert heston_cf.call_price(*a) == pytest.approx(heston_cf.call_price_mp(*a, dps=30), abs=1e-9)


def test_cf_black_scholes_limit():
    """xi -> 0 with rho = 0 and v0 = theta = sigma^2 gives Black-Scholes."""
    a = dict(C1, xi=1e-4, rho=0.0)
    assert heston_cf.call_price(*HESTON_ARGS(a)) == pytest.approx(bs.call(100, 100, 1, 0.02, 0.2), abs=1e-6)
    a = dict(C1, xi=1e-4, rho=0.0, K=110)
    assert heston_cf.put_price(*HESTON_ARGS(a)) == pytest.approx(bs.put(100, 110, 1, 0.02, 0.2), abs=1e-6)


def test_cf_monotone_convex_in_strike():
    Ks = np.linspace(70, 130, 13)
    c = np.array([heston_cf.call_price(*HESTON_ARGS(dict(C1, K=K))) for K in Ks])
    assert (np.diff(c) < 0).all()
    assert (np.diff(c, 2) > 0).all()
    # no-arbitrage bounds
    assert ((c >= np.maximum(100 - Ks * math.exp(-0.02), 0)) & (c <= 100)).all()


def test_european_qe_within_3se_of_cf():
    """The QE Monte Carlo price of C1 (64 steps) is within 3 SE + the QE bias of the CF price."""
    opt = oracle.Option(**C1, steps=64, paths=1 << 20, seed=1)
    p, se, _ = oracle.price_european(opt)
    cf = heston_cf.call_price(*HESTON_ARGS(C1))
    assert abs(p - cf) < 3 * se + QE_BIAS


def test_european_put_qe_and_fte_within_3se_of_cf():
    put = dict(C1, K=110)
    cf = heston_cf.put_price(*HESTON_ARGS(put))
    for scheme, steps in ((oracle.SCHEME_QE, 32), (oracle.SCHEME_FTE, 128)):
        opt = oracle.Option(**put, payoff=oracle.EURO_PUT, steps=steps, paths=1 << 19, seed=40, scheme=scheme)
        p, se, _ = oracle.price_european(opt)
        assert abs(p - cf) < 3 * se + QE_BIAS, (scheme, p, cf, se)


def test_put_call_parity_is_pathwise():
    """With common random numbers, C - P = e^{-rT}(mean S_T - K) to rounding, and it is
    within 3 SE of S0 - K e^{-rT} (the martingale property, up to the QE bias)."""
    opt = oracle.Option(**C1, steps=64, paths=200000, seed=3)
    c, _, _ = oracle.price_european(opt)
    p, _, _ = oracle.price_european(opt.replace(payoff=oracle.EURO_PUT))
    xT, _, _ = oracle.simulate(opt)
    disc = math.exp(-opt.r * opt.T)
    ST = opt.S0 * np.exp(xT)
    assert c - p == pytest.approx(disc * (ST.mean() - opt.K), abs=1e-9)
    se = disc * ST.std(ddof=1) / math.sqrt(ST.size)
    assert abs((c - p) - (opt.S0 - opt.K * disc)) < 3 * se + QE_BIAS


def test_results_do_not_depend_on_thread_count_and_prefixes_are_consistent():
    opt = oracle.Option(**C1, steps=20, paths=5000, seed=2, stream=9)
    a = oracle.price_european(opt, nthreads=1)
    b = oracle.price_european(opt, nthreads=7)
    assert a[0] == b[0] and a[1] == b[1]
    x_all, v_all, p_all = oracle.simulate(opt, nthreads=3)
    x_mid, v_mid, p_mid = oracle.simulate(opt, path0=1234, npaths=100, nthreads=2)
    assert np.array_equal(x_all[1234:1334], x_mid) and np.array_equal(p_all[1234:1334], p_mid)


def test_standard_error_formula():
    """price = sum X / P and SE = sqrt((sum X^2 - (sum X)^2 / P) / (P - 1) / P)."""
    opt = oracle.Option(**C1, steps=8, paths=3000, seed=5)
    price, se, sums = oracle.price_european(opt)
    _, _, pay = oracle.simulate(opt)
    assert price == pytest.approx(pay.mean(), rel=1e-14)
    assert se == pytest.approx(pay.std(ddof=1) / math.sqrt(pay.size), rel=1e-10)
    assert sums[0] == pytest.approx(pay.sum(), rel=1e-14)


def test_european_qe_m_within_3se_of_cf():
    """The martingale-corrected QE prices of the C1 call and the K=110 put (32 steps)
    are within 3 SE + the scheme's discretisation allowance of the CF prices, and their
    put-call parity holds against S0 - K e^{-rT} within 3 SE alone (no martingale bias
    left)."""
    for payoff, K, price in ((oracle.EURO_CALL, 100.0, heston_cf.call_price), (oracle.EURO_PUT, 110.0, heston_cf.put_price)):
        d = dict(C1, K=K)
        opt = oracle.Option(**d, payoff=payoff, steps=32, paths=1 << 19, seed=41, scheme=oracle.SCHEME_QE_M)
        p, se, _ = oracle.price_european(opt)
        cf = price(*HESTON_ARGS(d))
        assert abs(p - cf) < 3 * se + QE_BIAS, (payoff, p, cf, se)
    opt = oracle.Option(**C1, steps=16, paths=1 << 19, seed=42, scheme=oracle.SCHEME_QE_M)
    xT, _, _ = oracle.simulate(opt)
    disc = math.exp(-opt.r * opt.T)
    ST = disc * opt.S0 * np.exp(xT)
    assert abs(ST.mean() - opt.S0) < 3 * ST.std(ddof=1) / math.sqrt(ST.size)
