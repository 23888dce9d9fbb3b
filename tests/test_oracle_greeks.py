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
@pytest.mark.parametrize("scheme", [oracle.SCHEME_QE, oracle.SCHEME_FTE, oracle.SCHEME_QE_M, oracle.SCHEME_TG])
def test_forward_mode_matches_crn_finite_differences(payoff, K, scheme):
    """Per-path FD with h = 1e-4 |p| agrees with the pathwise tangent except on the
    few paths whose payoff kink falls inside the bump: within 3 SE of the per-path
    FD.  QE at these parameters stays in its (smooth) quadratic branch, and the
    truncated Gaussian step is smooth away from V = 0 (r(psi) is the solved root, so
    the tangent's implicit derivative meets FD of the root itself), so there the
    agreement is also tight in relative terms; full-truncation Euler has the
    max(v, 0) kink and sqrt(v) near v = 0, which FD smooths over.  The truncated Gaussian
    step reaches variances just above zero, where sqrt(K3 v + K4 V) of the next log-price
    step curves sharply: the central difference there takes a 1e-6 bump (at 1e-4 its
    second-order error alone is several times the tight bar)."""
    opt = oracle.Option(**dict(C1, K=K), payoff=payoff, steps=32, paths=40000, seed=4, scheme=scheme)
    _, _, g, gse = oracle.greeks(opt)
    fd, fdse = oracle.fd_greeks(opt, rel_bump=1e-6 if scheme == oracle.SCHEME_TG else 1e-4)
    for i, name in enumerate(oracle.GREEK_NAMES):
        assert abs(g[i] - fd[i]) < 3 * fdse[i] + 1e-3 * abs(fd[i]) + 1e-9, (name, g[i], fd[i], fdse[i])
    if scheme == oracle.SCHEME_FTE:
        return
    # The tight pin.  At a 1e-4 bump the difference quotient of a path whose payoff kink lies
    # inside the bump is not its pathwise derivative; such paths are O(h) of the sample and move
    # the estimate by ~3e-4 (rho of the call).  At a 1e-6 bump they are 100 times rarer, the
    # remaining truncation error is O(h^2), and FP64 rounding of the difference is ~1e-10: the
    # smooth schemes then agree with their tangents to ~1e-7 of the Greek's scale
    # |fd| + s_fd; the truncated Gaussian step, whose next log-price step curves sharply just
    # above V = 0, to ~1e-4.
    fd, fdse = oracle.fd_greeks(opt, rel_bump=1e-6)
    tight = 3e-4 if scheme == oracle.SCHEME_TG else 1e-6
    for i, name in enumerate(oracle.GREEK_NAMES):
        assert abs(g[i] - fd[i]) <= tight * (abs(fd[i]) + fdse[i]), (name, g[i], fd[i], fdse[i])


def test_martingale_corrected_greeks_exponential_branch_and_american():
    """The martingale-corrected scheme where QE mostly takes its exponential branch (xi 0.8,
    low kappa theta): the tangent of K0* = -ln E[exp(A V)] - (K1 + K3 / 2) v through the
    exponential-branch moment p + beta (1 - p) / (beta - A) agrees with CRN differences of
    the oracle's own price; and an American put's Greeks with its exercise indices fixed agree
    with fixed-index differences."""
    opt = oracle.Option(**dict(C1, K=100.0, kappa=0.5, theta=0.02, xi=0.8, v0=0.02), payoff=oracle.EURO_PUT,
                        steps=16, paths=40000, seed=8, scheme=oracle.SCHEME_QE_M)
    _, _, g, gse = oracle.greeks(opt)
    fd, fdse = oracle.fd_greeks(opt)
    for i, name in enumerate(oracle.GREEK_NAMES):
        assert abs(g[i] - fd[i]) < 3 * fdse[i] + 1e-3 * abs(fd[i]) + 1e-9, (name, g[i], fd[i], fdse[i])
    amer = oracle.Option(**dict(C1, K=110.0), payoff=oracle.AMER_PUT, steps=25, paths=1 << 15, seed=10,
                         scheme=oracle.SCHEME_QE_M)
    price, _, g, _ = oracle.greeks(amer)
    res = oracle.price_american(amer)
    assert price == res.price
    fd, fdse = oracle.fixed_tau_fd_greeks(amer, res.tau)
    for i, name in enumerate(oracle.GREEK_NAMES):
        assert abs(g[i] - fd[i]) < 3 * fdse[i] + 1e-3 * abs(fd[i]) + 1e-9, (name, g[i], fd[i], fdse[i])


def test_martingale_corrected_greeks_where_the_moment_never_exists():
    """kappa 4, theta 0.3, xi 2, rho 0.9 on 3-year steps: E[exp(A V) | v] does not exist from any
    v (whichever branch the step takes), so every step keeps the plain constant C0 = r dt + K0
    and the corrected scheme is plain QE: its prices and tangents equal QE's bit for bit, for a
    European put (with d/dT and gamma) and an American put.  A fallback that dropped K0's tangent,
    or differentiated the non-existent moment, would break the equality."""
    kappa, theta, xi, rho, dt = 4.0, 0.3, 2.0, 0.9, 3.0
    A = 0.5 * dt * (kappa * rho / xi - 0.5) + rho / xi + 0.25 * dt * (1.0 - rho * rho)  # K2 + K4 / 2
    for v in np.concatenate([[0.0], np.geomspace(1e-8, 20.0, 200)]):
        assert not oracle.qe_log_mgf(v, kappa, theta, xi, dt, A)[1], v
    base = dict(S0=100.0, K=100.0, T=2 * dt, r=0.02, kappa=kappa, theta=theta, xi=xi, rho=rho, v0=0.3, steps=2,
                paths=8000, seed=7)
    for payoff, fn in ((oracle.EURO_PUT, oracle.greeks_ext), (oracle.AMER_PUT, oracle.greeks)):
        a = fn(oracle.Option(**base, payoff=payoff, scheme=oracle.SCHEME_QE))
        b = fn(oracle.Option(**base, payoff=payoff, scheme=oracle.SCHEME_QE_M))
        assert a[0] == b[0] and a[1] == b[1]
        assert np.array_equal(a[2], b[2], equal_nan=True) and np.array_equal(a[3], b[3], equal_nan=True)


def test_truncated_gaussian_greeks_american_fixed_indices():
    """An American put under the truncated Gaussian step: the tangents with the exercise
    indices of the pricing run held fixed agree with fixed-index central differences (1e-6
    bump, as for the European pins: the step reaches variances just above zero)."""
    amer = oracle.Option(**dict(C1, K=110.0), payoff=oracle.AMER_PUT, steps=25, paths=1 << 15, seed=10,
                         scheme=oracle.SCHEME_TG)
    price, _, g, _ = oracle.greeks(amer)
    res = oracle.price_american(amer)
    assert price == res.price
    fd, fdse = oracle.fixed_tau_fd_greeks(amer, res.tau, rel_bump=1e-6)
    for i, name in enumerate(oracle.GREEK_NAMES):
        assert abs(g[i] - fd[i]) < 3 * fdse[i] + 1e-3 * abs(fd[i]) + 1e-9, (name, g[i], fd[i], fdse[i])


def test_greeks_primal_equals_pricing_run():
    """The tangent run's primal is the pricing run bit for bit (same branches)."""
    for scheme in (oracle.SCHEME_QE, oracle.SCHEME_QE_M):
        opt = oracle.Option(**C1, steps=16, paths=4000, seed=6, scheme=scheme)
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


# ---------------------------------------------------------------------------------------------
# d/dT (steps fixed) and gamma
# ---------------------------------------------------------------------------------------------
def test_black_scholes_gamma_and_dT_against_numerical_derivatives():
    """The closed forms themselves, against central differences of the BS prices."""
    S0, K, T, r, s = 100.0, 95.0, 1.3, 0.03, 0.25
    h = 1e-3
    for price, dT in ((bs.call, bs.call_dT), (bs.put, bs.put_dT)):
        assert dT(S0, K, T, r, s) == pytest.approx((price(S0, K, T + h, r, s) - price(S0, K, T - h, r, s)) / (2 * h),
                                                   rel=1e-6)
        g = (price(S0 + h, K, T, r, s) - 2 * price(S0, K, T, r, s) + price(S0 - h, K, T, r, s)) / h**2
        assert bs.gamma(S0, K, T, r, s) == pytest.approx(g, rel=1e-5)


@pytest.mark.parametrize("scheme", [oracle.SCHEME_QE, oracle.SCHEME_FTE])
@pytest.mark.parametrize("payoff,K", [(oracle.EURO_CALL, 100.0), (oracle.EURO_PUT, 110.0)])
def test_gbm_limit_gamma_and_dT(scheme, payoff, K):
    """xi = 0, rho = 0, v0 = theta: geometric Brownian motion sampled exactly at any step count
    (QE) or by Euler with a constant variance (also exact in distribution), so the estimators of
    gamma and of d/dT agree with Black-Scholes within 3 SE."""
    d = dict(C1, K=K, xi=0.0, rho=0.0)
    o = oracle.Option(**d, payoff=payoff, steps=16, paths=1 << 18, seed=8, scheme=scheme)
    _, _, g, gse = oracle.greeks_ext(o)
    sig = math.sqrt(d["theta"])
    args = (d["S0"], K, d["T"], d["r"], sig)
    dT = bs.call_dT(*args) if payoff == oracle.EURO_CALL else bs.put_dT(*args)
    assert abs(g[7] - dT) < 3 * gse[7], (g[7], dT, gse[7])
    assert abs(g[8] - bs.gamma(*args)) < 3 * gse[8], (g[8], bs.gamma(*args), gse[8])


def test_heston_gamma_and_dT_against_cf_differences():
    """Heston C1 call (64 steps): gamma against the second central difference of the CF price
    in S0 and d/dT against its central difference in T, within 3 SE + the QE bias allowance
    scaled to each Greek (the discretisation bias of the price, 0.01, over the bump)."""
    def cf(**kw):
        d = dict(C1, **kw)
        return heston_cf.call_price(d["S0"], d["K"], d["T"], d["r"], d["kappa"], d["theta"], d["xi"], d["rho"], d["v0"])
    o = oracle.Option(**C1, payoff=oracle.EURO_CALL, steps=64, paths=1 << 19, seed=5)
    _, _, g, gse = oracle.greeks_ext(o)
    h = 0.5
    gam = (cf(S0=100.0 + h) - 2 * cf() + cf(S0=100.0 - h)) / h**2
    dT = (cf(T=1.0 + 1e-3) - cf(T=1.0 - 1e-3)) / 2e-3
    assert abs(g[8] - gam) < 3 * gse[8] + 2e-4, (g[8], gam, gse[8])
    assert abs(g[7] - dT) < 3 * gse[7] + 0.02, (g[7], dT, gse[7])


@pytest.mark.parametrize("scheme", [oracle.SCHEME_QE, oracle.SCHEME_FTE])
def test_dT_against_crn_finite_differences(scheme):
    """d/dT with the step count fixed is the derivative of the discretised price: central FD of
    the oracle's own price in T with common random numbers (the draws are keyed by step and
    path, not by time) agrees within 3 SE of the per-path FD; for an American put with the
    exercise indices held fixed, the FD of the stopped cash flows."""
    o = oracle.Option(**dict(C1, K=110.0), payoff=oracle.EURO_PUT, steps=32, paths=40000, seed=4, scheme=scheme)
    _, _, g, gse = oracle.greeks_ext(o)
    h = 1e-4
    up = oracle.simulate(o.replace(T=o.T + h))[0]
    dn = oracle.simulate(o.replace(T=o.T - h))[0]
    pu = math.exp(-o.r * (o.T + h)) * np.maximum(o.K - o.S0 * np.exp(up), 0.0)
    pd = math.exp(-o.r * (o.T - h)) * np.maximum(o.K - o.S0 * np.exp(dn), 0.0)
    d = (pu - pd) / (2 * h)
    assert abs(g[7] - d.mean()) < 3 * d.std(ddof=1) / math.sqrt(d.size) + 1e-3 * abs(d.mean()), (g[7], d.mean())
    if scheme == oracle.SCHEME_QE:
        am = o.replace(payoff=oracle.AMER_PUT)
        tau = oracle.price_american(am).tau
        _, _, ga, _ = oracle.greeks_at_tau_ext(am, tau)
        d = (oracle.stopped_values(am.replace(T=am.T + h), tau) - oracle.stopped_values(am.replace(T=am.T - h), tau)) / (2 * h)
        assert abs(ga[7] - d.mean()) < 3 * d.std(ddof=1) / math.sqrt(d.size) + 1e-3 * abs(d.mean()), (ga[7], d.mean())


def test_no_likelihood_ratio_gamma_for_a_stopping_rule():
    """With exercise indices decided on the simulated paths, the likelihood-ratio weight would
    re-weight each path together with a stopping decision made on its own trajectory: the
    result is not the policy's gamma (0.075 against 0.019 from central differences of the
    fixed-policy delta on this case), so the oracle reports NaN for American options and for
    given stopping indices; d/dT with the indices fixed stays defined."""
    am = oracle.Option(**dict(C1, K=110.0), payoff=oracle.AMER_PUT, steps=25, paths=1 << 14, seed=10)
    _, _, g, gse = oracle.greeks_ext(am)
    assert math.isnan(g[8]) and math.isfinite(g[7])
    tau = oracle.price_american(am).tau
    _, _, g, _ = oracle.greeks_at_tau_ext(am, tau)
    assert math.isnan(g[8]) and math.isfinite(g[7])


def test_extended_greeks_extend_the_seven():
    """The first 7 values of the extended call are the 7 Greeks bit for bit; the t_0-exercised
    American option has dT = gamma = 0; |rho| = 1 leaves gamma undefined (NaN)."""
    o = oracle.Option(**C1, payoff=oracle.EURO_PUT, steps=16, paths=4000, seed=6)
    p7, se7, g7, gse7 = oracle.greeks(o)
    p9, se9, g9, gse9 = oracle.greeks_ext(o)
    assert (p7, se7) == (p9, se9) and np.array_equal(g7, g9[:7]) and np.array_equal(gse7, gse9[:7])
    deep = oracle.Option(**dict(C1, K=200.0), payoff=oracle.AMER_PUT, steps=8, paths=2000, seed=2)
    _, _, g, _ = oracle.greeks_ext(deep)
    assert g[0] == -1.0 and g[7] == 0.0 and g[8] == 0.0
    _, _, g, _ = oracle.greeks_ext(o.replace(rho=-1.0))
    assert math.isnan(g[8])
