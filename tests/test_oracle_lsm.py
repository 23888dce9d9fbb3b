"""Pins of the oracle's Longstaff-Schwartz pricing: the 6x6 solve against
numpy's SVD least squares, a brute-force numpy restatement on a small case,
the GBM limit against a binomial tree, and no-arbitrage bounds."""
import math

import numpy as np
import pytest

import oracle
from oracle import crr, heston_cf

C2 = dict(S0=100.0, K=110.0, T=1.0, r=0.02, kappa=1.5, theta=0.04, xi=0.3, rho=-0.7, v0=0.04)


def test_chol6_solve_matches_lstsq_full_rank():
    rng = np.random.default_rng(0)
    for _ in range(50):
        Phi = rng.normal(size=(40, 6)) * rng.uniform(0.1, 10, size=6)
        y = rng.normal(size=40)
        beta, rank = oracle.chol6_solve(Phi.T @ Phi, Phi.T @ y)
        ref = np.linalg.lstsq(Phi, y, rcond=None)[0]
        assert rank == 6
        assert np.allclose(Phi @ beta, Phi @ ref, rtol=1e-9, atol=1e-9)


def test_chol6_solve_drops_dependent_columns():
    """Duplicated / zero columns are dropped and the fitted values still equal the
    least-squares projection onto the column span."""
    rng = np.random.default_rng(1)
    for dup in ([0, 1, 2, 0, 1, 2], [0, 1, 2, 3, 3, 3]):
        base = rng.normal(size=(30, 6))
        Phi = base[:, dup].copy()
        Phi[:, 5] *= 2.0
        y = rng.normal(size=30)
        beta, rank = oracle.chol6_solve(Phi.T @ Phi, Phi.T @ y)
        ref = np.linalg.lstsq(Phi, y, rcond=None)[0]
        assert rank == np.linalg.matrix_rank(Phi)
        assert np.allclose(Phi @ beta, Phi @ ref, atol=1e-9)
    beta, rank = oracle.chol6_solve(np.zeros((6, 6)), np.zeros(6))
    assert rank == 0 and not beta.any()


def _numpy_lsm(opt):
    """Longstaff-Schwartz written again with numpy: states from the oracle's step
    functions, regression by numpy lstsq (SVD) on the literal basis
    {1, S, S^2, v, S v, v^2}."""
    N, P = opt.steps, opt.paths
    dt = opt.T / N
    w = oracle.rng_words(opt.seed, opt.stream, 0, P, 0, N)
    S = np.zeros((N + 1, P))
    V = np.zeros((N + 1, P))
    for p in range(P):
        x, v = 0.0, opt.v0
        S[0, p], V[0, p] = opt.S0, v
        for n in range(N):
            z1, z2 = oracle.box_muller(oracle.uniform(w[p, n, 0]), oracle.uniform(w[p, n, 1]))
            vn = oracle.qe_variance_step(v, opt.kappa, opt.theta, opt.xi, dt, z1, oracle.uniform(w[p, n, 2]))
            x = oracle.qe_logprice_step(x, v, vn, opt.r, opt.kappa, opt.theta, opt.xi, opt.rho, dt, z2)
            v = vn
            S[n + 1, p], V[n + 1, p] = opt.S0 * math.exp(x), v
    h = lambda s: np.maximum(opt.K - s, 0.0)
    cash = h(S[N])
    when = np.full(P, N)
    for n in range(N - 1, 0, -1):
        disc = np.exp(-opt.r * dt * (when - n))
        y = cash * disc
        itm = h(S[n]) > 0
        if itm.sum() < 6:
            continue
        s, v = S[n, itm], V[n, itm]
        Phi = np.stack([np.ones_like(s), s, s * s, v, s * v, v * v], axis=1)
        beta = np.linalg.lstsq(Phi, y[itm], rcond=None)[0]
        ex = h(s) > Phi @ beta
        idx = np.where(itm)[0][ex]
        cash[idx] = h(S[n, idx])
        when[idx] = n
    value = np.mean(cash * np.exp(-opt.r * dt * when))
    return max(h(np.array([opt.S0]))[0], value), when


def test_lsm_matches_numpy_restatement_small_case():
    opt = oracle.Option(**C2, payoff=oracle.AMER_PUT, steps=4, paths=256, seed=7)
    ref_price, ref_when = _numpy_lsm(opt)
    res = oracle.price_american(opt, nthreads=2)
    assert res.price == pytest.approx(ref_price, rel=1e-10)
    assert np.array_equal(res.tau, ref_when)


def test_lsm_gbm_limit_against_binomial_bermudan():
    """xi = 0, rho = 0, v0 = theta = sigma^2: GBM Bermudan put with exercise at the N
    Monte Carlo dates.  LSM is within 3 SE plus a 1% policy-bias allowance of the tree.
    The collinear variance columns exercise the column-drop rule."""
    sig2, N = 0.04, 50
    opt = oracle.Option(**dict(C2, xi=0.0, rho=0.0, v0=sig2, theta=sig2), payoff=oracle.AMER_PUT,
                        steps=N, paths=1 << 17, seed=17)
    res = oracle.price_american(opt)
    tree = crr.bermudan(100.0, 110.0, 1.0, 0.02, math.sqrt(sig2), N, sub=40)
    assert abs(res.price - tree) < 3 * res.std_err + 0.01 * tree, (res.price, tree)
    assert res.lsm_flags & 2  # columns were dropped


def test_binomial_tree_converges_to_black_scholes():
    from oracle import black_scholes as bs
    e = crr.bermudan(100, 110, 1.0, 0.02, 0.2, 100, sub=20, european=True)
    assert e == pytest.approx(bs.put(100, 110, 1.0, 0.02, 0.2), abs=2e-3)
    am = crr.bermudan(100, 110, 1.0, 0.02, 0.2, 100, sub=20)
    assert am > e


def test_american_put_bounds():
    """American >= European (CF) and >= intrinsic; an American call without dividends
    is worth the European call (same paths, up to a small policy error)."""
    opt = oracle.Option(**C2, payoff=oracle.AMER_PUT, steps=50, paths=1 << 16, seed=7)
    res = oracle.price_american(opt)
    euro = heston_cf.put_price(100, 110, 1.0, 0.02, 1.5, 0.04, 0.3, -0.7, 0.04)
    assert res.price > euro - 3 * res.std_err
    assert res.price >= 10.0
    assert res.tau.min() >= 1 and res.tau.max() <= 50
    call = opt.replace(K=100.0, payoff=oracle.AMER_CALL)
    am = oracle.price_american(call)
    eu, se, _ = oracle.price_european(call.replace(payoff=oracle.EURO_CALL))
    assert abs(am.price - eu) < 3 * se + 0.02 * eu


def test_lsm_flags_and_t0_exercise():
    """Deep out-of-the-money put: fewer than 6 ITM paths somewhere (flag bit 0).
    Deep in-the-money put with a high rate: intrinsic value wins at t_0."""
    opt = oracle.Option(**dict(C2, K=40.0), payoff=oracle.AMER_PUT, steps=10, paths=64, seed=3)
    assert oracle.price_american(opt).lsm_flags & 1
    deep = oracle.Option(**dict(C2, K=250.0, r=0.2), payoff=oracle.AMER_PUT, steps=10, paths=4096, seed=3)
    res = oracle.price_american(deep)
    assert res.exercised_at_t0 and res.price == pytest.approx(150.0)


def test_lsm_thread_count_independent():
    opt = oracle.Option(**C2, payoff=oracle.AMER_PUT, steps=12, paths=3000, seed=2)
    a = oracle.price_american(opt, nthreads=1)
    b = oracle.price_american(opt, nthreads=5)
    assert a.price == b.price and np.array_equal(a.tau, b.tau)


def test_oracle_outputs_consistent():
    """The exported path states end at the terminal values of `simulate`, and the
    exported regression coefficients reproduce the oracle's own exercise decisions
    at the first regression date (no later date has changed the cash flows yet)."""
    opt = oracle.Option(**C2, payoff=oracle.AMER_PUT, steps=12, paths=3000, seed=21)
    X, V = oracle.path_states(opt)
    xT, vT, _ = oracle.simulate(opt)
    assert np.array_equal(X[-1], xT) and np.array_equal(V[-1], vT)
    res = oracle.price_american(opt)
    N = opt.steps
    S = opt.S0 * np.exp(X[N - 2])
    h = np.maximum(opt.K - S, 0.0)
    a = (S - opt.K) / opt.K
    c = (np.maximum(V[N - 2], 0.0) - opt.theta) / opt.theta
    phi = np.stack([np.ones_like(a), a, a * a, c, a * c, c * c], axis=1)
    ex = (h > 0) & (h > phi @ res.beta[N - 1])
    # paths exercised at N-1 are exactly those; later (earlier-date) decisions may override
    assert np.all(res.tau[ex] <= N - 1)
    assert np.all(res.tau[(h > 0) & ~ex] != N - 1)
