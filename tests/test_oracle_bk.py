"""Pins of the oracle's Broadie-Kaya exact scheme: the variance draw is the exact CIR
transition (a library quantile), the conditional characteristic function of the integrated
variance integrates against the transition density to the closed-form CIR transform, the
inversion of its Fourier CDF returns that law's mean, and the exact scheme prices without
discretisation bias."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.stats import ncx2

import oracle
from oracle import black_scholes as bs
from oracle import heston_cf

PARAMS = [(1.5, 0.04, 0.3, 0.25), (0.5, 0.02, 0.8, 0.5), (3.0, 0.09, 0.1, 1.0)]  # Feller ok / violated / tight


def cir_transition(kappa, theta, xi, dt, v):
    E = math.exp(-kappa * dt)
    c = xi * xi * (1 - E) / (4 * kappa)
    return c, 4 * kappa * theta / xi ** 2, v * E / c


@pytest.mark.parametrize("kappa,theta,xi,dt", PARAMS)
def test_variance_draw_is_the_cir_quantile(kappa, theta, xi, dt):
    for v in (0.0, 0.01, 0.04, 0.2):
        c, df, lam = cir_transition(kappa, theta, xi, dt, v)
        for u in (1e-6, 0.01, 0.3, 0.5, 0.9, 0.9999):
            ref = c * (ncx2.ppf(u, df, lam) if lam > 0 else ncx2.ppf(u, df, 1e-300))
            assert oracle.bk_variance(v, kappa, theta, xi, dt, u) == pytest.approx(ref, rel=1e-9, abs=1e-300)


def cir_transform(a, kappa, theta, xi, dt, v):
    """E[exp(i a int_0^dt V) | V_0 = v] in closed form (the CIR bond-price formula at s = -i a):
    A exp(-B v), B = 2 s (e^{g dt} - 1) / D, A = (2 g e^{(kappa + g) dt / 2} / D)^{2 kappa theta / xi^2},
    D = (g + kappa)(e^{g dt} - 1) + 2 g.  The power is taken through logarithms of factors with
    positive real part (D = e^{g dt} [(g + kappa)(1 - e^{-g dt}) + 2 g e^{-g dt}]), so its phase
    is continuous in a; the principal power of the base jumps by 2 pi times the exponent."""
    s = -1j * a
    g = np.sqrt(kappa * kappa + 2 * xi * xi * s)
    e = np.exp(-g * dt)
    Dr = (g + kappa) * (1 - e) + 2 * g * e  # D e^{-g dt}
    B = 2 * s * (1 - e) / Dr
    logA = (2 * kappa * theta / xi ** 2) * (np.log(2 * g) + (kappa - g) * dt / 2 - np.log(Dr))
    return np.exp(logA - B * v)


@pytest.mark.parametrize("kappa,theta,xi,dt", PARAMS)
def test_conditional_cf_integrates_to_the_cir_transform(kappa, theta, xi, dt):
    """E[ phi(a; v_u, V_t) ] over the exact law of V_t equals the unconditional transform of
    the integrated variance: the Bessel ratio, its continuous phase and the other factors of
    the conditional characteristic function, at frequencies where its phase turns many times."""
    for vu in (0.04, 0.0):
        c, df, lam = cir_transition(kappa, theta, xi, dt, vu)
        lam = max(lam, 1e-300)
        q = 2.0 / df if df < 2.0 else 1.0  # v = w^q removes a density singular like v^(df/2 - 1) at 0
        hi = (c * ncx2.ppf(1 - 1e-15, df, lam)) ** (1.0 / q)
        for a in (1.0, 20.0, 100.0, 400.0, 2000.0):
            def f(w, part):
                v = w ** q
                z = (np.exp(oracle.bk_log_cf(a, vu, v, kappa, theta, xi, dt)) * ncx2.pdf(v / c, df, lam) / c
                     * q * w ** (q - 1))
                return z.real if part == 0 else z.imag
            got = complex(integrate.quad(f, 0, hi, args=(0,), limit=500, epsabs=1e-13)[0],
                          integrate.quad(f, 0, hi, args=(1,), limit=500, epsabs=1e-13)[0])
            assert abs(got - cir_transform(a, kappa, theta, xi, dt, vu)) < 1e-9, (vu, a, got)


@pytest.mark.parametrize("kappa,theta,xi,dt", PARAMS)
def test_integrated_variance_inversion_returns_the_conditional_mean(kappa, theta, xi, dt):
    """The integral over u of the inverted draws (their mean) equals the conditional mean read
    off the characteristic function (-i d/da ln phi at 0, a central difference), also for the
    strongly skewed law of small endpoints with the Feller condition violated (where a Fourier
    period too short for the tail would pile the upper quantiles up at half the period); the
    draws increase with u."""
    for vu, vt in ((0.04, 0.05), (0.01, 0.002), (0.09, 0.12)):
        def q(u):
            return oracle.bk_integrated_variance(vu, vt, kappa, theta, xi, dt, u)
        draws = np.array([q(u) for u in (1e-6, 0.01, 0.5, 0.99, 0.999, 0.9999, 0.99999)])
        assert np.all(np.diff(draws) > 0) and draws[0] > 0
        m = integrate.quad(q, 0, 1, limit=200, points=[0.9, 0.99, 0.999, 0.9999])[0]
        h = 1e-3 / (0.5 * (vu + vt) * dt)
        mean = (oracle.bk_log_cf(h, vu, vt, kappa, theta, xi, dt).imag
                - oracle.bk_log_cf(-h, vu, vt, kappa, theta, xi, dt).imag) / (2 * h)
        assert m == pytest.approx(mean, rel=1e-4), (vu, vt, m, mean)


C1 = dict(S0=100.0, T=1.0, r=0.02, kappa=1.5, theta=0.04, xi=0.3, rho=-0.7, v0=0.04)


@pytest.mark.parametrize("steps", [1, 4])
@pytest.mark.parametrize("payoff,K", [(oracle.EURO_CALL, 100.0), (oracle.EURO_PUT, 110.0)])
def test_exact_scheme_prices_without_bias(steps, payoff, K):
    """Exact simulation: the price is within 3 SE of the characteristic-function price with
    no discretisation allowance, at one step and at four."""
    o = oracle.Option(**C1, K=K, payoff=payoff, steps=steps, paths=1 << 15, seed=31, scheme=oracle.SCHEME_BK)
    p, se, _ = oracle.price_european(o)
    cf = heston_cf.call_price if payoff == oracle.EURO_CALL else heston_cf.put_price
    ref = cf(100.0, K, 1.0, 0.02, 1.5, 0.04, 0.3, -0.7, 0.04)
    assert abs(p - ref) < 3 * se, (p, ref, se)


def test_exact_scheme_deterministic_variance():
    """xi = 0: the variance follows the CIR mean exactly and the log-price is Gaussian with the
    integrated variance, so the call is Black-Scholes with that total variance."""
    o = oracle.Option(**dict(C1, xi=0.0, v0=0.09, rho=-0.5), K=100.0, steps=2, paths=1 << 16, seed=2,
                      scheme=oracle.SCHEME_BK)
    p, se, _ = oracle.price_european(o)
    iv = 0.04 * 1.0 + (0.09 - 0.04) * (1 - math.exp(-1.5)) / 1.5
    assert abs(p - bs.call(100.0, 100.0, 1.0, 0.02, math.sqrt(iv))) < 3 * se
