"""Pins of the oracle's basket risk Greeks (per-asset vegas in v0 and theta, correlation
sensitivities) against what does not use its tangents: numpy differences of the Cholesky
factor, the single-option Greeks when only asset 0 carries weight, central differences of
the oracle's own price with common random numbers, the GBM limit's semi-closed form (where
the scheme's log-prices are exactly Gaussian with a trapezoid-rule integrated variance), and
fixed-policy differences of an American basket's stopped cash flows."""
import math

import numpy as np
import pytest

import oracle
from oracle import basket_gbm as bg

C3 = ((1.0, 0.6, -0.3), (0.6, 1.0, 0.2), (-0.3, 0.2, 1.0))


def basket3(**kw):
    base = dict(S0=(100.0, 90.0, 110.0), w=(0.4, 0.35, 0.25), kappa=(1.5, 2.0, 1.0), theta=(0.04, 0.06, 0.03),
                xi=(0.3, 0.5, 0.25), rho=(-0.7, -0.5, -0.3), v0=(0.04, 0.05, 0.035), corr=C3, K=100.0)
    base.update(kw)
    return oracle.Basket(**base)


def bump(b: oracle.Basket, what: str, i: int, j: int, h: float) -> oracle.Basket:
    if what == "corr":
        C = [list(r) for r in b.corr]
        C[i][j] += h
        C[j][i] += h
        return b.replace(corr=tuple(tuple(r) for r in C))
    vals = list(getattr(b, what))
    vals[i] += h
    return b.replace(**{what: tuple(vals)})


def crn_difference(b, what, i, j, h, tau=None):
    """Per-path central difference of the discounted (stopped) cash flow: (mean, SE)."""
    def cash(bb):
        if tau is None:
            return oracle.basket_simulate(bb)[2]
        return oracle.basket_stopped_values(bb, tau)
    fd = (cash(bump(b, what, i, j, h)) - cash(bump(b, what, i, j, -h))) / (2 * h)
    return fd.mean(), fd.std(ddof=1) / math.sqrt(fd.size)


def test_cholesky_derivative_against_numpy_differences():
    rng = np.random.default_rng(5)
    A = rng.normal(size=(5, 5))
    S = A @ A.T + 5 * np.eye(5)
    C = S / np.sqrt(np.outer(np.diag(S), np.diag(S)))
    for i in range(1, 5):
        for j in range(i):
            L, dL = oracle.corr_cholesky_tan(C, i, j)
            np.testing.assert_allclose(L, np.linalg.cholesky(C), rtol=0, atol=1e-14)
            E = np.zeros((5, 5))
            E[i, j] = E[j, i] = 1.0
            h = 1e-6
            fd = (np.linalg.cholesky(C + h * E) - np.linalg.cholesky(C - h * E)) / (2 * h)
            np.testing.assert_allclose(dL, fd, rtol=0, atol=1e-8)
            # lower triangular, and the rows above i do not see C_ij
            assert np.all(np.triu(dL, 1) == 0.0) and np.all(dL[:i, :] == 0.0)
    with pytest.raises(ValueError):
        oracle.corr_cholesky_tan(C, 2, 2)


@pytest.mark.parametrize("scheme", [oracle.SCHEME_QE, oracle.SCHEME_FTE, oracle.SCHEME_QE_M, oracle.SCHEME_TG])
def test_asset_zero_vegas_are_the_single_option_greeks(scheme):
    """Weight on asset 0 only: asset 0 follows the single option's path bit for bit (its
    correlated normal is 1.0 z2_0), so its vegas are the single option's d/dv0 and d/dtheta to
    rounding of the final products; the other assets' vegas and every correlation
    sensitivity are exactly 0 (the first row of L does not move with an off-diagonal C_ij)."""
    b = basket3(w=(1.0, 0.0, 0.0), paths=6000, steps=24, seed=3, scheme=scheme)
    _, _, vv, _, vt, _, dc, _ = oracle.basket_risk_greeks(b)
    single = oracle.Option(S0=100.0, K=100.0, T=1.0, r=0.02, kappa=1.5, theta=0.04, xi=0.3, rho=-0.7, v0=0.04,
                           payoff=oracle.EURO_CALL, steps=24, paths=6000, seed=3, scheme=scheme)
    _, _, g, _ = oracle.greeks(single)
    assert vv[0] == pytest.approx(g[1], rel=1e-12) and vt[0] == pytest.approx(g[2], rel=1e-12), (vv[0], g[1], vt[0], g[2])
    assert np.all(vv[1:] == 0.0) and np.all(vt[1:] == 0.0) and np.all(dc == 0.0)


@pytest.mark.parametrize("scheme", [oracle.SCHEME_QE, oracle.SCHEME_QE_M, oracle.SCHEME_TG, oracle.SCHEME_FTE])
@pytest.mark.parametrize("payoff", [oracle.EURO_CALL, oracle.EURO_PUT])
def test_risk_greeks_against_crn_differences(scheme, payoff):
    """Heston, three correlated assets: every vega and correlation sensitivity against the
    central difference of the oracle's own price on the same paths.  At a 1e-6 bump the payoff
    kink lies inside the bump on very few paths, so for the smooth schemes the two agree to
    1e-5 of |fd| + s_fd; full-truncation Euler (the max(v, 0) kink) within 3 SE of the
    difference."""
    b = basket3(paths=12000, steps=16, seed=4, scheme=scheme, payoff=payoff)
    _, _, vv, vvs, vt, vts, dc, dcs = oracle.basket_risk_greeks(b)
    checks = [("v0", i, 0, vv[i], vvs[i], 1e-6 * b.v0[i]) for i in range(3)]
    checks += [("theta", i, 0, vt[i], vts[i], 1e-6 * b.theta[i]) for i in range(3)]
    checks += [("corr", i, j, dc[i, j], dcs[i, j], 1e-6) for i in range(3) for j in range(i)]
    for what, i, j, g, gse, h in checks:
        fd, fdse = crn_difference(b, what, i, j, h)
        if scheme == oracle.SCHEME_FTE:
            assert abs(g - fd) < 3 * fdse + 1e-3 * abs(fd) + 1e-9, (what, i, j, g, fd, fdse)
        else:
            assert abs(g - fd) <= 1e-5 * (abs(fd) + fdse), (what, i, j, g, fd, fdse)
    assert np.all(dc == dc.T) and np.all(np.diag(dc) == 0.0)


@pytest.mark.parametrize("call", [True, False])
def test_gbm_limit_against_semi_closed_form(call):
    """xi = 0 and v0 = theta: the variance is deterministic and constant, the scheme's
    log-prices are exactly Gaussian with variance Sigma_i = sum_n (v_n + v_{n+1}) dt / 2 and
    correlation C_01, so the price is the two-asset semi-closed form at sigma_i^2 = Sigma_i / T.
    d Sigma_i / d v0_i = sum_n (E^n + E^{n+1}) dt / 2 and d Sigma_i / d theta_i =
    sum_n (2 - E^n - E^{n+1}) dt / 2 with E = e^{-kappa_i dt} (the correlation of the two
    log-prices is stationary in the variance profiles at proportional profiles), and
    d price / d C_01 is the semi-closed form's derivative in its correlation.  The Monte Carlo
    vegas and correlation sensitivity lie within 4 SE of those."""
    sig = (0.2, 0.3)
    kappa = (1.5, 0.8)
    N, T = 8, 1.0
    b = oracle.Basket(S0=(100.0, 90.0), w=(0.6, 0.4), kappa=kappa, theta=tuple(s * s for s in sig),
                      v0=tuple(s * s for s in sig), xi=(0.0, 0.0), rho=(0.0, 0.0), corr=((1.0, 0.5), (0.5, 1.0)),
                      K=95.0, T=T, paths=1 << 18, steps=N, seed=21,
                      payoff=oracle.EURO_CALL if call else oracle.EURO_PUT)
    _, _, vv, vvs, vt, vts, dc, dcs = oracle.basket_risk_greeks(b)
    dt = T / N

    def price(s1, s2, rho):
        return bg.european(100.0, 90.0, 0.6, 0.4, 95.0, T, 0.02, s1, s2, rho, call=call)

    for i in range(2):
        E = math.exp(-kappa[i] * dt)
        dS_dv0 = sum((E ** n + E ** (n + 1)) * dt / 2 for n in range(N))
        dS_dth = sum((2.0 - E ** n - E ** (n + 1)) * dt / 2 for n in range(N))
        h = 1e-4 * sig[i]
        up = list(sig); up[i] += h
        dn = list(sig); dn[i] -= h
        dp_dsig = (price(up[0], up[1], 0.5) - price(dn[0], dn[1], 0.5)) / (2 * h)
        dp_dSigma = dp_dsig / (2.0 * sig[i] * T)  # sigma_i = sqrt(Sigma_i / T)
        assert abs(vv[i] - dp_dSigma * dS_dv0) < 4 * vvs[i], (i, vv[i], dp_dSigma * dS_dv0, vvs[i])
        assert abs(vt[i] - dp_dSigma * dS_dth) < 4 * vts[i], (i, vt[i], dp_dSigma * dS_dth, vts[i])
    h = 1e-4
    dp_drho = (price(0.2, 0.3, 0.5 + h) - price(0.2, 0.3, 0.5 - h)) / (2 * h)
    assert abs(dc[0, 1] - dp_drho) < 4 * dcs[0, 1], (dc[0, 1], dp_drho, dcs[0, 1])


def test_american_basket_risk_greeks_hold_the_policy_fixed():
    """An American basket put: with its own Longstaff-Schwartz exercise indices (tau NULL) the
    price is the LSM price and the Greeks are those at the indices the LSM pass returns; each
    agrees with fixed-index central differences of the stopped cash flows on the same paths."""
    b = basket3(paths=8000, steps=12, seed=6, payoff=oracle.AMER_PUT, K=105.0)
    res = oracle.basket_price_american(b)
    p, se, vv, vvs, vt, vts, dc, dcs = oracle.basket_risk_greeks(b)
    assert p == res.price and se == res.std_err
    tau = np.zeros(b.paths, dtype=np.int32) if res.exercised_at_t0 else res.tau
    q = oracle.basket_risk_greeks(b, tau=tau)
    assert np.array_equal(q[2], vv) and np.array_equal(q[4], vt) and np.array_equal(q[6], dc)
    checks = [("v0", i, 0, vv[i], 1e-6 * b.v0[i]) for i in range(3)]
    checks += [("theta", i, 0, vt[i], 1e-6 * b.theta[i]) for i in range(3)]
    checks += [("corr", i, j, dc[i, j], 1e-6) for i in range(3) for j in range(i)]
    for what, i, j, g, h in checks:
        fd, fdse = crn_difference(b, what, i, j, h, tau=tau)
        assert abs(g - fd) <= 1e-5 * (abs(fd) + fdse), (what, i, j, g, fd, fdse)
