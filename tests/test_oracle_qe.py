"""Pins of the oracle's Heston steps (Andersen's QE variance and log-price
steps, full-truncation Euler) against the mathematics of the CIR / Heston
processes rather than against the oracle's own formulas."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle


def cir_moments(v, kappa, theta, xi, dt):
    """Exact conditional mean and variance of the CIR variance process over dt
    (Cox-Ingersoll-Ross 1985), written from the noncentral chi-square law:
    v(t+dt) = c * X, X ~ ncx2(df = 4 kappa theta / xi^2, nc = v e^{-kappa dt} / c),
    c = xi^2 (1 - e^{-kappa dt}) / (4 kappa).  Mean c (df + nc), variance c^2 (2 df + 4 nc)."""
    c = xi * xi * (1 - math.exp(-kappa * dt)) / (4 * kappa)
    df = 4 * kappa * theta / (xi * xi)
    nc = v * math.exp(-kappa * dt) / c
    return c * (df + nc), c * c * (2 * df + 4 * nc)


# (v, kappa, theta, xi, dt): the first three land in the quadratic branch (psi <= 1.5),
# the last three in the exponential branch (psi > 1.5)
QUAD_CASES = [(0.04, 1.5, 0.04, 0.3, 1 / 64), (0.09, 3.0, 0.02, 0.8, 1 / 252), (0.01, 0.5, 0.09, 0.1, 0.25)]
EXP_CASES = [(0.0005, 1.5, 0.04, 0.9, 1 / 64), (0.0, 0.5, 0.02, 0.8, 1 / 252), (0.002, 2.0, 0.03, 1.2, 0.5)]


def psi_of(v, kappa, theta, xi, dt):
    m, s2 = cir_moments(v, kappa, theta, xi, dt)
    return s2 / (m * m)


@pytest.mark.parametrize("case", QUAD_CASES)
def test_qe_quadratic_branch_matches_cir_moments_exactly(case):
    """In the quadratic branch V is a degree-2 polynomial of the Gaussian Z, so a
    Gauss-Hermite rule with 10 nodes integrates E[V] and E[V^2] exactly: both must
    equal the CIR moments to rounding (Andersen's moment matching)."""
    v, kappa, theta, xi, dt = case
    assert psi_of(*case) <= 1.5
    nodes, weights = np.polynomial.hermite_e.hermegauss(10)
    weights = weights / weights.sum()
    V = np.array([oracle.qe_variance_step(v, kappa, theta, xi, dt, z, 0.5) for z in nodes])
    m, s2 = cir_moments(v, kappa, theta, xi, dt)
    mean = (weights * V).sum()
    var = (weights * V * V).sum() - mean * mean
    assert mean == pytest.approx(m, rel=1e-12)
    assert var == pytest.approx(s2, rel=1e-9)
    assert (V >= 0).all()


@pytest.mark.parametrize("case", EXP_CASES)
def test_qe_exponential_branch_matches_cir_moments_exactly(case):
    """In the exponential branch V is a function of the uniform U alone: integrating
    it over U in (0,1) must give the CIR mean and variance to quadrature accuracy."""
    v, kappa, theta, xi, dt = case
    assert psi_of(*case) > 1.5
    f = lambda u: oracle.qe_variance_step(v, kappa, theta, xi, dt, 0.0, u)
    # locate the atom at zero: V == 0 for u <= p
    us = np.linspace(1e-9, 1 - 1e-9, 20001)
    zero = np.array([f(u) == 0.0 for u in us])
    p = us[zero].max() if zero.any() else 0.0
    m1, _ = integrate.quad(f, p, 1, limit=400, points=None, epsabs=1e-16, epsrel=1e-12)
    m2, _ = integrate.quad(lambda u: f(u) ** 2, p, 1, limit=400, epsabs=1e-18, epsrel=1e-12)
    m, s2 = cir_moments(v, kappa, theta, xi, dt)
    assert m1 == pytest.approx(m, rel=1e-6)
    assert m2 - m1 * m1 == pytest.approx(s2, rel=1e-5)
    # continuity at the atom: V -> 0 as u -> p from above, and V >= 0 everywhere
    assert f(min(p + 1e-7, 1 - 1e-9)) < 1e-5 * m
    assert all(f(u) >= 0 for u in us[::97])


def test_qe_switch_level_and_deterministic_limit():
    """psi exactly at psi_c takes the quadratic branch (V depends on Z, not on U);
    xi = 0 moves the variance deterministically to its conditional mean."""
    v, kappa, theta, dt = 0.03, 1.0, 0.05, 0.1
    assert oracle.qe_variance_step(v, kappa, theta, 0.0, dt, 1.3, 0.9) == pytest.approx(
        theta + (v - theta) * math.exp(-kappa * dt), rel=1e-15)
    # quadratic branch ignores U
    a = oracle.qe_variance_step(0.04, 1.5, 0.04, 0.3, 1 / 64, 0.7, 0.1)
    b = oracle.qe_variance_step(0.04, 1.5, 0.04, 0.3, 1 / 64, 0.7, 0.9)
    assert a == b
    # exponential branch ignores Z
    a = oracle.qe_variance_step(0.0005, 1.5, 0.04, 0.9, 1 / 64, -2.0, 0.95)
    b = oracle.qe_variance_step(0.0005, 1.5, 0.04, 0.9, 1 / 64, 2.0, 0.95)
    assert a == b and a > 0


def test_qe_one_large_step_close_to_exact_cir_law():
    """Over one coarse step the QE draw approximates the exact noncentral chi-square
    transition: the Kolmogorov distance must be small (QE is an approximation)."""
    v, kappa, theta, xi, dt = 0.04, 1.5, 0.04, 0.3, 0.25
    w = oracle.rng_words(seed=3, stream=0, path0=0, npaths=20000, step0=0, nsteps=1).reshape(-1, 4)
    V = []
    for a, b, c, _ in w:
        z1, _ = oracle.box_muller(oracle.uniform(a), oracle.uniform(b))
        V.append(oracle.qe_variance_step(v, kappa, theta, xi, dt, z1, oracle.uniform(c)))
    V = np.array(V)
    c = xi * xi * (1 - math.exp(-kappa * dt)) / (4 * kappa)
    law = stats.ncx2(df=4 * kappa * theta / xi**2, nc=v * math.exp(-kappa * dt) / c, scale=c)
    ks = stats.kstest(V, law.cdf).statistic
    assert ks < 0.02


def test_logprice_step_against_sde_decomposition():
    """Andersen's log-price step comes from integrating the Heston SDE and replacing
    the time integral of v by the trapezoid dt (v + V)/2:
        dx = r dt - (1/2) I + (rho/xi)(V - v - kappa theta dt + kappa I) + sqrt(1 - rho^2) sqrt(I) Z
    with I = dt (v + V)/2.  Its conditional mean and standard deviation must match."""
    rng = np.random.default_rng(8)
    for _ in range(50):
        v, V = rng.uniform(0.001, 0.2, size=2)
        r, kappa, theta, xi, rho, dt = 0.02, rng.uniform(0.5, 3), rng.uniform(0.02, 0.09), rng.uniform(0.1, 0.8), rng.uniform(-0.9, 0.0), 1 / 252
        I = dt * (v + V) / 2
        mean = r * dt - 0.5 * I + (rho / xi) * (V - v - kappa * theta * dt + kappa * I)
        sd = math.sqrt(1 - rho * rho) * math.sqrt(I)
        x0 = 0.3
        at0 = oracle.qe_logprice_step(x0, v, V, r, kappa, theta, xi, rho, dt, 0.0) - x0
        at1 = oracle.qe_logprice_step(x0, v, V, r, kappa, theta, xi, rho, dt, 1.0) - x0
        assert at0 == pytest.approx(mean, rel=1e-9, abs=1e-15)
        assert at1 - at0 == pytest.approx(sd, rel=1e-9)


@pytest.mark.parametrize("scheme", [oracle.SCHEME_QE, oracle.SCHEME_FTE])
def test_gbm_limit_paths_are_exact(scheme):
    """xi = 0, rho = 0, v0 = theta = sigma^2: the model is GBM and each path's
    x_T must equal (r - sigma^2/2) T + sigma sqrt(dt) sum_n Z2_n, with Z2 the
    second Box-Muller output of each step, evaluated here by numpy."""
    sig2, T, N, r = 0.04, 1.0, 16, 0.03
    opt = oracle.Option(xi=0.0, rho=0.0, v0=sig2, theta=sig2, kappa=1.7, T=T, r=r, steps=N, paths=64,
                        seed=4, scheme=scheme)
    xT, vT, _ = oracle.simulate(opt, nthreads=1)
    w = oracle.rng_words(4, 0, 0, 64, 0, N)
    u0 = ((w[..., 0] >> 9).astype(np.float64) + 0.5) * 2.0**-23
    u1 = ((w[..., 1] >> 9).astype(np.float64) + 0.5) * 2.0**-23
    z2 = np.sqrt(-2 * np.log(u0)) * np.sin(2 * np.pi * u1)
    dt = T / N
    expect = (r - sig2 / 2) * T + math.sqrt(sig2 * dt) * z2.sum(axis=1)
    assert np.allclose(xT, expect, rtol=0, atol=1e-12)
    assert np.allclose(vT, sig2, rtol=1e-14)


def test_fte_step_reduces_to_euler_maruyama_for_positive_variance():
    """For v > 0 the truncation is inactive: the FTE step is the Euler step of the
    Heston SDE with correlated drivers rho Z1 + sqrt(1 - rho^2) Z2."""
    x, v = 0.1, 0.05
    r, kappa, theta, xi, rho, dt, z1, z2 = 0.02, 1.5, 0.04, 0.3, -0.7, 0.01, 0.4, -1.1
    xn, vn = oracle.fte_step(x, v, r, kappa, theta, xi, rho, dt, z1, z2)
    dW1 = math.sqrt(dt) * z1
    dW2 = math.sqrt(dt) * (rho * z1 + math.sqrt(1 - rho * rho) * z2)
    assert vn == pytest.approx(v + kappa * (theta - v) * dt + xi * math.sqrt(v) * dW1, rel=1e-14)
    assert xn == pytest.approx(x + (r - v / 2) * dt + math.sqrt(v) * dW2, rel=1e-14)
    # negative variance is truncated inside the drift and diffusion only
    xn, vn = oracle.fte_step(x, -0.01, r, kappa, theta, xi, rho, dt, z1, z2)
    assert vn == pytest.approx(-0.01 + kappa * theta * dt, rel=1e-14)
    assert xn == pytest.approx(x + r * dt, rel=1e-14)


def test_mean_variance_path_matches_cir_mean():
    """E[v_T] = theta + (v0 - theta) e^{-kappa T} for the QE variance path (within SE)."""
    opt = oracle.Option(v0=0.09, theta=0.04, kappa=1.5, xi=0.5, steps=32, paths=200000, seed=21)
    _, vT, _ = oracle.simulate(opt)
    expect = opt.theta + (opt.v0 - opt.theta) * math.exp(-opt.kappa * opt.T)
    assert abs(vT.mean() - expect) < 4 * vT.std() / math.sqrt(vT.size)
    assert (vT >= 0).all()


# ---------------------------------------------------------------------------------------------
# Martingale-corrected QE (Andersen 2008): E[exp(x_{n+1} - x_n) | v_n] = e^{r dt} exactly.
# The expectation is taken by quadrature of the oracle's own step functions over their random
# inputs (no formula is retyped): Gauss-Hermite over the quadratic branch's Z_V, adaptive
# quadrature over the exponential branch's uniform U (split at the zero-mass point, found by
# bisection on the step itself), and Gauss-Hermite over the asset Gaussian Z.
# ---------------------------------------------------------------------------------------------
GH_X, GH_W = np.polynomial.hermite_e.hermegauss(60)
GH_W = GH_W / math.sqrt(2 * math.pi)


def _step_mgf(step, v, kappa, theta, xi, rho, dt, r=0.03):
    def over_z(V):
        return sum(w * math.exp(step(0.0, v, V, r, kappa, theta, xi, rho, dt, z) - r * dt) for z, w in zip(GH_X, GH_W))
    if psi_of(v, kappa, theta, xi, dt) <= 1.5:
        return sum(w * over_z(oracle.qe_variance_step(v, kappa, theta, xi, dt, z1, 0.5)) for z1, w in zip(GH_X, GH_W))
    lo, hi = 0.0, 1.0  # the largest u with V = 0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if oracle.qe_variance_step(v, kappa, theta, xi, dt, 0.0, mid) == 0.0:
            lo = mid
        else:
            hi = mid
    tail, _ = integrate.quad(lambda u: over_z(oracle.qe_variance_step(v, kappa, theta, xi, dt, 0.0, u)), hi, 1.0,
                             epsabs=1e-13, epsrel=1e-12, limit=200)
    return lo * over_z(0.0) + tail


@pytest.mark.parametrize("case", QUAD_CASES + EXP_CASES)
@pytest.mark.parametrize("rho", [-0.7, 0.4])
def test_qe_martingale_correction_is_exact_per_step(case, rho):
    v, kappa, theta, xi, dt = case
    corrected = _step_mgf(oracle.qe_m_logprice_step, v, kappa, theta, xi, rho, dt)
    plain = _step_mgf(oracle.qe_logprice_step, v, kappa, theta, xi, rho, dt)
    # corrected: 1 to rounding (measured |error| <= 7e-16); the uncorrected step misses by
    # 2e-12 .. 1e-3 on these cases, so the check would see a dropped or wrong term
    assert abs(corrected - 1.0) <= 1e-13, (case, rho, corrected)
    assert abs(plain - 1.0) > 100 * max(abs(corrected - 1.0), 1e-15), (case, rho, plain)


def test_qe_log_mgf_domain_and_deterministic_limit():
    v, kappa, theta, xi, dt = QUAD_CASES[0]
    val, ok = oracle.qe_log_mgf(v, kappa, theta, xi, dt, 1e6)   # 2 A a >= 1: no moment
    assert not ok and val == 0.0
    v, kappa, theta, xi, dt = EXP_CASES[0]
    val, ok = oracle.qe_log_mgf(v, kappa, theta, xi, dt, 1e9)   # A >= beta: no moment
    assert not ok
    m = theta + (0.03 - theta) * math.exp(-kappa * dt)
    val, ok = oracle.qe_log_mgf(0.03, kappa, theta, 0.0, dt, 0.7)  # xi = 0: V = m
    assert ok and val == pytest.approx(0.7 * m, rel=1e-15)


def test_qe_m_gbm_limit_is_the_plain_scheme_bit_for_bit():
    base = dict(S0=100.0, K=100.0, T=1.0, r=0.02, kappa=1.5, theta=0.04, xi=0.0, rho=0.0, v0=0.04,
                payoff=oracle.EURO_CALL, steps=16, paths=512, seed=3)
    a = oracle.simulate(oracle.Option(**base, scheme=oracle.SCHEME_QE))
    b = oracle.simulate(oracle.Option(**base, scheme=oracle.SCHEME_QE_M))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_qe_m_discounted_asset_is_a_martingale():
    """Per-step exactness makes E[e^{-rT} S_T] = S0 (tower property): a coarse grid
    and a large vol-of-vol, 2^20 paths, within 3 SE."""
    o = oracle.Option(S0=100.0, K=100.0, T=2.0, r=0.03, kappa=0.5, theta=0.04, xi=0.9, rho=-0.9, v0=0.04,
                      payoff=oracle.EURO_CALL, steps=8, paths=1 << 20, seed=21, scheme=oracle.SCHEME_QE_M)
    xT, _, _ = oracle.simulate(o)
    d = math.exp(-o.r * o.T) * o.S0 * np.exp(xT)
    assert abs(d.mean() - o.S0) <= 3 * d.std(ddof=1) / math.sqrt(d.size), d.mean()


def test_bk_has_no_forward_mode_greeks():
    for scheme in (oracle.SCHEME_BK,):
        o = oracle.Option(S0=100.0, K=100.0, T=1.0, r=0.02, kappa=1.5, theta=0.04, xi=0.3, rho=-0.7, v0=0.04,
                          payoff=oracle.EURO_CALL, steps=4, paths=64, seed=1, scheme=scheme)
        with pytest.raises(RuntimeError):
            oracle.greeks(o)


# ---------------------------------------------------------------------------------------------
# Truncated Gaussian (TG) variance step: V = max(mu + sigma Z, 0) moment-matched to the CIR law.
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("case", QUAD_CASES + EXP_CASES)
def test_tg_step_matches_cir_moments_exactly(case):
    """E[V] and Var[V] of the oracle's TG step, by adaptive quadrature over its Gaussian input
    split at the truncation point (found by bisection on the step itself), equal the exact CIR
    conditional moments to 1e-10 relative -- in both psi regimes QE separates."""
    v, kappa, theta, xi, dt = case
    f = lambda z: oracle.tg_variance_step(v, kappa, theta, xi, dt, z)
    lo, hi = -40.0, 40.0  # the largest z with V = 0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) == 0.0:
            lo = mid
        else:
            hi = mid
    pdf = stats.norm.pdf
    m1, _ = integrate.quad(lambda z: f(z) * pdf(z), hi, np.inf, epsabs=1e-15, epsrel=1e-13, limit=200)
    m2, _ = integrate.quad(lambda z: f(z) ** 2 * pdf(z), hi, np.inf, epsabs=1e-17, epsrel=1e-13, limit=200)
    mean, var = cir_moments(v, kappa, theta, xi, dt)
    assert m1 == pytest.approx(mean, rel=1e-10), (case, m1, mean)
    assert m2 - m1 * m1 == pytest.approx(var, rel=1e-9), (case, m2 - m1 * m1, var)


def test_tg_r_is_monotone_and_deterministic_limit():
    psis = np.geomspace(1e-3, 50.0, 60)
    rs = np.array([oracle.tg_r(p) for p in psis])
    # r ~ 1 / sqrt(psi) for small psi (nearly no truncation); r(50) = -1.81
    assert np.all(np.diff(rs) < 0) and rs[0] == pytest.approx(1 / math.sqrt(1e-3), rel=1e-3) and rs[-1] < -1.5
    m = 0.04 + (0.03 - 0.04) * math.exp(-1.5 / 64)
    assert oracle.tg_variance_step(0.03, 1.5, 0.04, 0.0, 1 / 64, 0.7) == pytest.approx(m, rel=1e-15)


def test_european_tg_within_3se_of_cf():
    """The TG scheme (QE's log-price step) prices the C1 call and the K=110 put (64 steps)
    within 3 SE + the discretisation allowance of the CF price."""
    C1 = dict(S0=100.0, K=100.0, T=1.0, r=0.02, kappa=1.5, theta=0.04, xi=0.3, rho=-0.7, v0=0.04)
    from oracle import heston_cf
    for payoff, K, price in ((oracle.EURO_CALL, 100.0, heston_cf.call_price), (oracle.EURO_PUT, 110.0, heston_cf.put_price)):
        d = dict(C1, K=K)
        o = oracle.Option(**d, payoff=payoff, steps=64, paths=1 << 19, seed=43, scheme=oracle.SCHEME_TG)
        p, se, _ = oracle.price_european(o)
        cf = price(d["S0"], d["K"], d["T"], d["r"], d["kappa"], d["theta"], d["xi"], d["rho"], d["v0"])
        assert abs(p - cf) < 3 * se + 0.01, (payoff, p, cf, se)
