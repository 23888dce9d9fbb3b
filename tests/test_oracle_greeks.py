"""Pins of the oracle's forward-mode pathwise Greeks: central finite differences
of the oracle's own price with common random numbers (a different computation:
no tangents), the Black-Scholes limit, and finite differences of the
characteristic-function price."""
import math

import numpy as np
import pytest

import oracle
from oracle import black_scholes as bs
from oracle import heston_cf

C1 = dict(S0=100.0, K=100.0, T=1.0, r=0.02, kappa=1.5, theta=0.04, xi=0.3, rho=-0.7, v0=0.04)


@pytest.mark.parametrize("payoff,K", [(oracle.EURO_CALL, 100.0), (oracle.EURO_PUT, 110.0)])
@pytest.mark.parametrize("scheme", [oracle.SCHEME_QE, oracle.SCHEME_FTE])
def test_forward_mode_matches_crn_finite_differences(payoff, K, scheme):
    """Per-path FD with h = 1e-4 |p| agrees with the pathwise tangent except on the
    few paths whose payoff kink falls inside the bump: within 3 SE of the per-path
    FD.  QE at these parameters stays in its (smooth) quadratic branch, so there
    the agreement is also tight in relative terms; full-truncation Euler has the
    max(v, 0) kink and sqrt(v) near v = 0, which FD smooths over."""
    opt = oracle.Option(**dict(C1, K=K), payoff=payoff, steps=32, paths=40000, seed=4, scheme=scheme)
    _, _, g, gse = oracle.greeks(opt)
    fd, fdse = oracle.fd_greeks(opt)
    for i, name in enumerate(oracle.GREEK_NAMES):
        assert abs(g[i] - fd[i]) < 3 * fdse[i] + 1e-3 * abs(fd[i]) + 1e-9, (name, g[i], fd[i], fdse[i])
        if scheme == oracle.SCHEME_QE:
            assert g[i] == pytest.approx(fd[i], rel=2e-3, abs=2e-3 * fdse[i] + 1e-6), name


def test_greeks_primal_equals_pricing_run():
    """The tangent run's primal is the pricing run bit for bit (same branches)."""
    opt = oracle.Option(**C1, steps=16, paths=4000, seed=6)
    p_tan, se_tan, _, _ = oracle.greeks(opt)
    p, se, _ = oracle.price_european(opt)
    assert p_tan == p and se_tan == se


def test_black_scholes_limit_greeks():
    """xi = 0, rho = 0, v0 = theta = sigma^2: delta -> N(d1); rho -> K T e^{-rT} N(d2);
    and moving v0 and theta together by eps shifts sigma^2 by eps, so
    d/dv0 + d/dtheta = vega_sigma / (2 sigma)."""
    s2 = 0.04
    opt = oracle.Option(**dict(C1, xi=0.0, rho=0.0, v0=s2, theta=s2), steps=16, paths=1 << 18, seed=8)
    _, _, g, gse = oracle.greeks(opt)
    sig = math.sqrt(s2)
    assert abs(g[0] - bs.call_delta(100, 100, 1, 0.02, sig)) < 4 * gse[0]
    assert abs(g[3] - bs.call_rho(100, 100, 1, 0.02, sig)) < 4 * gse[3]
    tot = g[1] + g[2]
    assert abs(tot - bs.vega_sigma(100, 100, 1, 0.02, sig) / (2 * sig)) < 4 * math.hypot(gse[1], gse[2])


def test_european_greeks_against_cf_finite_differences():
    """The pathwise Monte Carlo Greeks estimate the derivatives of the model price,
    which FD on the smooth CF price gives directly: within 3 SE + a bias allowance."""
    opt = oracle.Option(**C1, steps=64, paths=1 << 18, seed=9)
    _, _, g, gse = oracle.greeks(opt)
    base = dict(C1)
    allowance = {"S0": 0.005, "v0": 1.0, "theta": 1.0, "r": 0.5, "kappa": 0.05, "xi": 0.2, "rho": 0.2}
    for i, name in enumerate(oracle.GREEK_NAMES):
        h = 1e-4 * abs(base[name])
        up = dict(base, **{name: base[name] + h})
        dn = dict(base, **{name: base[name] - h})
        cf_d = (heston_cf.call_price(**up) - heston_cf.call_price(**dn)) / (2 * h)
        assert abs(g[i] - cf_d) < 3 * gse[i] + allowance[name], (name, g[i], cf_d, gse[i])


def test_american_greeks_against_fixed_exercise_finite_differences():
    """American put: pathwise Greeks hold the exercise times tau from the LSM run
    fixed.  FD with common random numbers of the cash flows stopped at the same tau
    must agree within 3 SE of the per-path FD (tight: same tau, only the payoff kink
    differs).  The price is the LSM price bit for bit."""
    opt = oracle.Option(**dict(C1, K=110.0), payoff=oracle.AMER_PUT, steps=25, paths=1 << 15, seed=10)
    price, se, g, gse = oracle.greeks(opt)
    res = oracle.price_american(opt)
    assert price == res.price
    fd, fdse = oracle.fixed_tau_fd_greeks(opt, res.tau)
    assert g[0] < 0  # put delta
    for i, name in enumerate(oracle.GREEK_NAMES):
        assert abs(g[i] - fd[i]) < 3 * fdse[i] + 1e-3 * abs(fd[i]) + 1e-9, (name, g[i], fd[i], fdse[i])


def test_american_greeks_against_full_lsm_finite_differences():
    """FD of the full LSM price re-fits every regression, so exercise decisions flip
    under the bump; by the envelope argument those flips cancel to first order in
    expectation but add noise that grows like 1/h, and the in-sample LSM policy is
    only near-optimal, so the two estimators differ by more than their standard
    errors (a known bias, reported rather than hidden).  With a 1% bump the FD must
    agree with the fixed-tau pathwise Greeks in sign and to within a loose band;
    delta, the best-determined Greek, to 5%."""
    opt = oracle.Option(**dict(C1, K=110.0), payoff=oracle.AMER_PUT, steps=25, paths=1 << 16, seed=10)
    _, _, g, gse = oracle.greeks(opt)
    fd, _ = oracle.fd_greeks(opt, rel_bump=1e-2)
    for i, name in enumerate(oracle.GREEK_NAMES):
        assert abs(g[i] - fd[i]) < 0.5 * abs(g[i]) + 10 * gse[i] + 0.2, (name, g[i], fd[i], gse[i])
    assert abs(g[0] - fd[0]) < 0.05 * abs(fd[0])


def test_greeks_at_given_stopping_indices():
    """The fixed-policy Greeks: with every path stopped at N they are the European
    put's Greeks bit for bit; with every path stopped at 0 the value is the intrinsic
    K - S0 with delta -1 and no other sensitivity; at an arbitrary policy the value
    is the mean of the stopped cash flows and the Greeks agree with common-random-
    number finite differences of those cash flows (tau fixed); indices outside 0..N
    are rejected."""
    base = dict(C1, K=110.0, steps=20, paths=1 << 13, seed=12)
    amer = oracle.Option(**base, payoff=oracle.AMER_PUT)
    N, P = base["steps"], base["paths"]
    v, se, g, gse = oracle.greeks_at_tau(amer, np.full(P, N))
    pe, see, ge, gsee = oracle.greeks(oracle.Option(**base, payoff=oracle.EURO_PUT))
    assert v == pe and se == see
    assert np.array_equal(g, ge) and np.array_equal(gse, gsee)
    v0, se0, g0, _ = oracle.greeks_at_tau(amer, np.zeros(P))
    assert v0 == pytest.approx(base["K"] - base["S0"], abs=1e-12) and se0 == 0.0
    assert g0[0] == -1.0 and np.all(g0[1:] == 0.0)
    tau = np.random.default_rng(3).integers(1, N + 1, P)
    v, se, g, gse = oracle.greeks_at_tau(amer, tau)
    sv = oracle.stopped_values(amer, tau)
    assert v == pytest.approx(sv.mean(), rel=1e-13) and se == pytest.approx(sv.std(ddof=1) / math.sqrt(P), rel=1e-9)
    fd, fdse = oracle.fixed_tau_fd_greeks(amer, tau)
    for i, name in enumerate(oracle.GREEK_NAMES):
        assert abs(g[i] - fd[i]) < 3 * fdse[i] + 1e-3 * abs(fd[i]) + 1e-9, (name, g[i], fd[i], fdse[i])
    bad = tau.copy()
    bad[5] = N + 1
    with pytest.raises(RuntimeError):
        oracle.greeks_at_tau(amer, bad)
