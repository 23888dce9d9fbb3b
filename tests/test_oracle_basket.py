"""Pins of the oracle's correlated-basket functions against what the mathematics fixes:
reductions to the single-asset oracle, the GBM limit (closed forms for the log-return
covariance and the geometric basket, a semi-closed form for the two-asset arithmetic basket
that is itself pinned by 2-D quadrature of the definition, a two-asset binomial lattice for
the Bermudan basket), martingale and parity identities, and finite differences."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import ndtr

import oracle
from oracle import basket_gbm as bg
from oracle import black_scholes as bs
from oracle import crr

C3 = ((1.0, 0.6, -0.3), (0.6, 1.0, 0.2), (-0.3, 0.2, 1.0))


def basket3(**kw):
    base = dict(S0=(100.0, 90.0, 110.0), w=(0.4, 0.35, 0.25), kappa=(1.5, 2.0, 1.0), theta=(0.04, 0.06, 0.03),
                xi=(0.3, 0.5, 0.25), rho=(-0.7, -0.5, -0.3), v0=(0.04, 0.05, 0.035), corr=C3, K=100.0)
    base.update(kw)
    return oracle.Basket(**base)


def gbm(b: oracle.Basket, sig):
    """The xi = 0 limit: constant variance sigma_i^2 (v0 = theta), correlation C."""
    d = b.assets
    return b.replace(xi=(0.0,) * d, v0=tuple(s * s for s in sig), theta=tuple(s * s for s in sig))


def test_corr_cholesky_against_numpy_and_rejects_indefinite():
    rng = np.random.default_rng(3)
    for d in (1, 3, 8, 32):
        A = rng.standard_normal((d, d + 4))
        S = A @ A.T
        C = S / np.sqrt(np.outer(np.diag(S), np.diag(S)))
        L = oracle.corr_cholesky(C)
        np.testing.assert_allclose(L, np.linalg.cholesky(C), rtol=1e-12, atol=1e-13)
        assert np.allclose(np.triu(L, 1), 0.0)
    assert oracle.corr_cholesky([[1.0, 1.2], [1.2, 1.0]]) is None
    assert oracle.corr_cholesky([[1.0, 0.9, 0.9], [0.9, 1.0, -0.9], [0.9, -0.9, 1.0]]) is None


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_asset_zero_is_the_single_asset_path(scheme):
    """Asset 0 draws the single-asset words (counter word 3 = 0) and its correlated normal
    is L_00 z2_0 = z2_0, so a basket with weights e_0 is the single-asset option bit for
    bit, whatever the other assets and the correlations are."""
    b = basket3(w=(1.0, 0.0, 0.0), paths=3000, steps=20, scheme=scheme, K=95.0, payoff=oracle.EURO_PUT)
    o = oracle.Option(S0=100.0, K=95.0, T=1.0, r=0.02, kappa=1.5, theta=0.04, xi=0.3, rho=-0.7, v0=0.04,
                      payoff=oracle.EURO_PUT, steps=20, paths=3000, scheme=scheme)
    xT, vT, pay = oracle.basket_simulate(b)
    rx, rv, rp = oracle.simulate(o)
    assert np.array_equal(xT[:, 0], rx) and np.array_equal(vT[:, 0], rv) and np.array_equal(pay, rp)
    assert oracle.basket_price_european(b) == oracle.price_european(o)[:2]
    # the other assets do move, and differently
    assert np.abs(xT[:, 1] - xT[:, 0]).min() > 0.0


def test_gbm_limit_log_return_moments():
    """xi = 0: ln S_T,i - ln S0_i = (r - sigma_i^2/2) T + sigma_i sqrt(T) (L Z)_i exactly, so
    the sample means and covariances match the closed forms (a transposed or wrong factor
    changes Cov = T sigma_i sigma_j C_ij)."""
    sig = (0.2, 0.3, 0.15)
    b = gbm(basket3(paths=1 << 17, steps=4, seed=11), sig)
    xT, _, _ = oracle.basket_simulate(b)
    P = xT.shape[0]
    T, r = b.T, b.r
    s = np.array(sig)
    mean_ref = (r - 0.5 * s * s) * T
    sd = s * math.sqrt(T)
    assert np.all(np.abs(xT.mean(0) - mean_ref) < 4 * sd / math.sqrt(P))
    cov = np.cov(xT.T)
    ref = T * np.outer(s, s) * np.array(C3)
    se = np.sqrt((ref ** 2 + np.outer(np.diag(ref), np.diag(ref))) / P)
    assert np.all(np.abs(cov - ref) < 4 * se), (cov, ref)


def test_gbm_limit_geometric_basket_closed_form():
    """The geometric basket prod S_i^{a_i} (a = w / sum w) of correlated GBMs is lognormal:
    its call is Black's formula with the mean and variance of sum a_i ln S_T,i."""
    sig = (0.25, 0.2, 0.3)
    b = gbm(basket3(paths=1 << 17, steps=2, seed=5), sig)
    xT, _, _ = oracle.basket_simulate(b)
    a = np.array(b.w) / sum(b.w)
    s = np.array(sig)
    S0 = np.array(b.S0)
    lnG = (a * (np.log(S0) + xT)).sum(1)
    K = 98.0
    pay = math.exp(-b.r * b.T) * np.maximum(np.exp(lnG) - K, 0.0)
    m = float((a * (np.log(S0) + (b.r - 0.5 * s * s) * b.T)).sum())
    v = float(b.T * a @ (np.outer(s, s) * np.array(C3)) @ a)
    F = math.exp(m + 0.5 * v)
    d1 = (math.log(F / K) + 0.5 * v) / math.sqrt(v)
    ref = math.exp(-b.r * b.T) * (F * ndtr(d1) - K * ndtr(d1 - math.sqrt(v)))
    assert abs(pay.mean() - ref) < 3 * pay.std(ddof=1) / math.sqrt(pay.size), (pay.mean(), ref)


def test_semi_closed_form_two_asset_basket_is_pinned():
    """The Gauss-Hermite conditional-Black price equals 2-D adaptive quadrature of the
    definition, reduces to Black-Scholes for w1 = 0, rho = 0, and obeys put-call parity."""
    S1, S2, w1, w2, K, T, r, s1, s2, rho = 100, 90, 0.6, 0.4, 95, 1.0, 0.02, 0.2, 0.3, 0.5
    sq = math.sqrt(T)

    def f(z2, z1):
        a = S1 * math.exp((r - 0.5 * s1 * s1) * T + s1 * sq * z1)
        b = S2 * math.exp((r - 0.5 * s2 * s2) * T + s2 * sq * (rho * z1 + math.sqrt(1 - rho * rho) * z2))
        return max(w1 * a + w2 * b - K, 0.0) * math.exp(-0.5 * (z1 * z1 + z2 * z2)) / (2 * math.pi)

    quad, _ = integrate.dblquad(f, -9, 9, -9, 9, epsabs=1e-9, epsrel=1e-10)
    assert bg.european(S1, S2, w1, w2, K, T, r, s1, s2, rho) == pytest.approx(math.exp(-r * T) * quad, abs=1e-5)
    assert bg.european(100, 100, 0.0, 1.0, 105, T, r, 0.2, 0.3, 0.0) == pytest.approx(
        bs.call(100, 105, T, r, 0.3), rel=1e-10)
    c = bg.european(S1, S2, w1, w2, K, T, r, s1, s2, rho, call=True)
    p = bg.european(S1, S2, w1, w2, K, T, r, s1, s2, rho, call=False)
    assert c - p == pytest.approx(w1 * S1 + w2 * S2 - K * math.exp(-r * T), rel=1e-12)


def test_lattice_is_pinned():
    """The BEG lattice: European value converges to the semi-closed form; with w2 = 0 the
    Bermudan put matches the one-asset CRR tree; American >= European."""
    args = (100, 90, 0.6, 0.4, 95, 1.0, 0.02, 0.2, 0.3, 0.5)
    e = bg.bermudan(*args, dates=50, sub=8, call=True, european_only=True)
    assert e == pytest.approx(bg.european(*args), rel=3e-4)
    one = bg.bermudan(100, 100, 1.0, 0.0, 110, 1.0, 0.02, 0.2, 0.3, 0.4, dates=50, sub=16)
    assert one == pytest.approx(crr.bermudan(100, 110, 1.0, 0.02, 0.2, 50, sub=16), rel=2e-3)
    am = bg.bermudan(*args, dates=50, sub=8)
    assert am > bg.bermudan(*args, dates=50, sub=8, european_only=True)


@pytest.mark.parametrize("call", [True, False])
def test_gbm_two_asset_price_and_greeks_against_semi_closed_form(call):
    """xi = 0, two assets: the Monte Carlo price, pathwise deltas and pathwise-LR gammas
    (cross-gamma included) lie within 4 SE of the semi-closed form and its differences."""
    sig = (0.2, 0.3)
    b = gbm(oracle.Basket(S0=(100.0, 90.0), w=(0.6, 0.4), corr=((1.0, 0.5), (0.5, 1.0)), K=95.0, paths=1 << 18,
                          steps=8, seed=21, payoff=oracle.EURO_CALL if call else oracle.EURO_PUT), sig)
    p, se, dl, dls, g, gs = oracle.basket_greeks(b)
    args = (100, 90, 0.6, 0.4, 95, 1.0, 0.02, 0.2, 0.3, 0.5)
    ref = bg.european(*args, call=call)
    rd, rg = bg.greeks(*args, call=call)
    assert abs(p - ref) < 4 * se, (p, ref, se)
    assert np.all(np.abs(dl - rd) < 4 * dls), (dl, rd, dls)
    assert np.all(np.abs(g - rg) < 4 * gs), (g, rg, gs)
    assert g[0, 1] == g[1, 0]


def test_single_asset_basket_gamma_is_black_scholes():
    sig = 0.25
    b = gbm(oracle.Basket(S0=(100.0,), w=(1.0,), kappa=(1.5,), theta=(0.04,), xi=(0.3,), rho=(-0.7,), v0=(0.04,),
                          corr=((1.0,),), K=105.0, paths=1 << 18, steps=16, seed=2), (sig,))
    _, _, dl, dls, g, gs = oracle.basket_greeks(b)
    assert abs(dl[0] - bs.call_delta(100, 105, 1.0, 0.02, sig)) < 4 * dls[0]
    assert abs(g[0, 0] - bs.gamma(100, 105, 1.0, 0.02, sig)) < 4 * gs[0, 0]


def test_pathwise_put_call_parity():
    """h_call - h_put = B_T - K on every path, so the discounted means differ by
    e^{-rT} (mean B_T - K) to rounding."""
    b = basket3(paths=20000, steps=16)
    xT, _, pc = oracle.basket_simulate(b.replace(payoff=oracle.EURO_CALL))
    _, _, pp = oracle.basket_simulate(b.replace(payoff=oracle.EURO_PUT))
    BT = (np.array(b.w) * np.array(b.S0) * np.exp(xT)).sum(1)
    np.testing.assert_allclose(pc - pp, math.exp(-b.r * b.T) * (BT - b.K), rtol=0, atol=1e-11)


def test_martingale_corrected_assets_are_martingales():
    """Under the martingale-corrected scheme every asset's discounted price has mean S0_i,
    with correlated drivers (the correction is per asset and the correlation does not move
    the means)."""
    b = basket3(paths=1 << 17, steps=8, seed=9, scheme=oracle.SCHEME_QE_M, xi=(0.9, 0.7, 0.5))
    xT, _, _ = oracle.basket_simulate(b)
    disc = math.exp(-b.r * b.T) * np.array(b.S0) * np.exp(xT)
    se = disc.std(0, ddof=1) / math.sqrt(disc.shape[0])
    assert np.all(np.abs(disc.mean(0) - np.array(b.S0)) < 3 * se), (disc.mean(0), se)


def test_heston_deltas_and_gammas_against_crn_differences():
    """Heston, three correlated assets: pathwise deltas equal the central differences of the
    oracle's own price with common random numbers (a tight check: same paths, the bump only
    moves S0), and the pathwise-LR gammas agree with central differences of the pathwise
    deltas within 4 combined SE."""
    b = basket3(paths=1 << 16, steps=32, seed=4)
    p, se, dl, dls, g, gs = oracle.basket_greeks(b)
    S0 = np.array(b.S0)
    for i in range(3):
        h = 1e-4 * S0[i]
        up = list(S0); up[i] += h
        dn = list(S0); dn[i] -= h
        _, _, pu = oracle.basket_simulate(b.replace(S0=tuple(up)))
        _, _, pd = oracle.basket_simulate(b.replace(S0=tuple(dn)))
        fd = (pu - pd) / (2 * h)
        assert abs(dl[i] - fd.mean()) < 4 * fd.std(ddof=1) / math.sqrt(fd.size) + 1e-9, (i, dl[i], fd.mean())
    for j in range(3):
        h = 0.01 * S0[j]
        up = list(S0); up[j] += h
        dn = list(S0); dn[j] -= h
        _, _, du, dus, _, _ = oracle.basket_greeks(b.replace(S0=tuple(up)))
        _, _, dd, dds, _, _ = oracle.basket_greeks(b.replace(S0=tuple(dn)))
        fd = (du - dd) / (2 * h)
        fd_se = np.hypot(dus, dds) / (2 * h)
        for i in range(3):
            assert abs(g[i, j] - fd[i]) < 4 * math.hypot(gs[i, j], fd_se[i]), (i, j, g[i, j], fd[i])


def test_gamma_is_nan_for_perfect_spot_vol_correlation():
    b = basket3(rho=(-1.0, -0.5, -0.3), paths=4000, steps=8)
    _, _, dl, _, g, _ = oracle.basket_greeks(b)
    assert np.all(np.isfinite(dl)) and np.isnan(g[0, 0]) and np.isnan(g[0, 1])
    assert np.isfinite(g[1, 2])


def test_generic_cholesky_solve():
    """Against numpy least squares (full rank), the same fitted values with duplicated
    columns, and bit-equal to the 6x6 solver at nb = 6."""
    rng = np.random.default_rng(8)
    X = rng.standard_normal((400, 10))
    y = rng.standard_normal(400)
    beta, rank = oracle.chol_solve(X.T @ X, X.T @ y)
    assert rank == 10
    np.testing.assert_allclose(beta, np.linalg.lstsq(X, y, rcond=None)[0], rtol=1e-9, atol=1e-12)
    Xd = X.copy()
    Xd[:, 7] = Xd[:, 2]
    beta, rank = oracle.chol_solve(Xd.T @ Xd, Xd.T @ y)
    assert rank == 9
    ls = np.linalg.lstsq(Xd, y, rcond=None)[0]
    np.testing.assert_allclose(Xd @ beta, Xd @ ls, rtol=1e-9, atol=1e-10)
    X6 = X[:, :6]
    G, bv = X6.T @ X6, X6.T @ y
    b6 = np.zeros(6)
    import ctypes
    oracle._L().ref_chol6_solve(oracle._ptr(np.ascontiguousarray(G), ctypes.c_double),
                                oracle._ptr(np.ascontiguousarray(bv), ctypes.c_double),
                                oracle._ptr(b6, ctypes.c_double))
    assert np.array_equal(oracle.chol_solve(G, bv)[0], b6)


def test_basket_states_match_terminal_values():
    b = basket3(paths=2000, steps=12)
    X, V = oracle.basket_states(b)
    xT, vT, _ = oracle.basket_simulate(b)
    S = np.array(b.w) * np.array(b.S0) * np.exp(xT)
    B0 = float(np.dot(b.w, b.S0))
    np.testing.assert_allclose(X[-1], np.log(S.sum(1) / B0), rtol=0, atol=1e-13)
    np.testing.assert_allclose(V[-1], (S * np.maximum(vT, 0)).sum(1) / S.sum(1), rtol=1e-13)


def test_basket_lsm_one_asset_gbm_against_crr():
    """d = 1, xi = 0: the basket LSM (cubic basis; the variance columns are collinear and
    dropped) is within 3 SE plus a 1% policy allowance of the CRR Bermudan put."""
    sig = 0.2
    b = gbm(oracle.Basket(S0=(100.0,), w=(1.0,), kappa=(1.5,), theta=(0.04,), xi=(0.3,), rho=(0.0,), v0=(0.04,),
                          corr=((1.0,),), K=110.0, payoff=oracle.AMER_PUT, steps=50, paths=1 << 17, seed=17), (sig,))
    res = oracle.basket_price_american(b)
    tree = crr.bermudan(100.0, 110.0, 1.0, 0.02, sig, 50, sub=40)
    assert abs(res.price - tree) < 3 * res.std_err + 0.01 * tree, (res.price, tree)
    assert res.lsm_flags & 2


def test_basket_lsm_two_asset_gbm_against_lattice():
    """d = 2, xi = 0: the basket LSM put is within 3 SE plus a 1% policy allowance of the
    two-asset lattice's Bermudan put (exercise at the same 50 dates)."""
    sig = (0.2, 0.3)
    b = gbm(oracle.Basket(S0=(100.0, 90.0), w=(0.6, 0.4), corr=((1.0, 0.5), (0.5, 1.0)), K=105.0,
                          payoff=oracle.AMER_PUT, steps=50, paths=1 << 17, seed=3), sig)
    res = oracle.basket_price_american(b)
    lat = bg.bermudan(100, 90, 0.6, 0.4, 105, 1.0, 0.02, 0.2, 0.3, 0.5, dates=50, sub=8)
    euro = bg.european(100, 90, 0.6, 0.4, 105, 1.0, 0.02, 0.2, 0.3, 0.5, call=False)
    assert abs(res.price - lat) < 3 * res.std_err + 0.01 * lat, (res.price, lat)
    assert lat > euro + 0.05  # early exercise is worth something here


def test_basket_american_consistency():
    """Heston, three assets: the LSM price is the mean of its own stopped cash flows, at
    least the European price, and the pathwise deltas at the fixed exercise indices have the
    put's sign; gamma is not estimated for a stopping rule."""
    b = basket3(payoff=oracle.AMER_PUT, K=105.0, steps=40, paths=1 << 15, seed=6)
    res = oracle.basket_price_american(b)
    assert not res.exercised_at_t0 and res.tau.min() >= 1 and res.tau.max() <= 40
    sv = oracle.basket_stopped_values(b, res.tau)
    assert sv.mean() * math.exp(0.0) == pytest.approx(res.price, rel=1e-12)
    eu, se = oracle.basket_price_european(b.replace(payoff=oracle.EURO_PUT))
    assert res.price > eu - 3 * se
    p, _, dl, _, g, _ = oracle.basket_greeks(b)
    assert p == res.price and np.all(dl < 0) and np.all(np.isnan(g))
    v, _, dl2, _, _, _ = oracle.basket_greeks(b, tau=res.tau)
    assert v == pytest.approx(res.price, rel=1e-12) and np.array_equal(dl, dl2)
