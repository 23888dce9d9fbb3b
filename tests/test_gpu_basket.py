"""GPU parity for correlated baskets: the HIP path through the C ABI against the FP64 oracle
on the same seeded inputs.

Tolerances (FP32 on the GPU, FP64 in the oracle, as for single options):
  * per-path log-prices: median |dx| <= 1e-5, max <= 3e-4 (QE's branch choice can differ on
    near-tie draws, which moves a handful of paths further); per-path variances: relative
    error (with a floor of 1e-3 theta_i) median <= 3e-6, p99 <= 5e-5;
  * prices: |dprice| <= 1e-4 B_0 at equal paths, standard errors to 1e-3 relative;
  * deltas: |d delta| <= 1e-4 max(|delta|, s) with s the per-path standard deviation;
    cross-gammas: |d gamma| <= 1e-3 max(|gamma|, s) (the scores are FP32 sums over the steps);
  * American baskets: the GPU's exercise policy valued by the oracle on its FP64 paths matches
    the GPU price to 1e-4 B_0; the two in-sample LSM prices agree within 3 SE.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2402_12111_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def ob(b: dict, **kw) -> oracle.Basket:
    d = dict(b)
    d.update(kw)
    return oracle.Basket(**d)


def b0(b: dict) -> float:
    return float(np.dot(b["w"], b["S0"]))


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_basket_terminal_values_per_path(S, scheme):
    b = W.basket(5, paths=5000, steps=32)  # 5000 paths: a ragged last block
    say("basket paths scheme", scheme)
    xT, vT, pay = S.debug_basket_paths(b, scheme)
    rx, rv, rp = oracle.basket_simulate(ob(b, scheme=scheme))
    dx = np.abs(xT - rx)
    assert np.median(dx) < 1e-5 and dx.max() < 3e-4, (np.median(dx), dx.max())
    # variance of every asset, relative to max(|v|, 1e-3 theta_i): measured median <= 5e-7,
    # p99 <= 1.2e-5, max 1.6e-3 (Euler, where v crosses 0 on a few paths)
    rv = np.asarray(rv, dtype=np.float64)
    rel = np.abs(vT.astype(np.float64) - rv) / np.maximum(np.abs(rv), 1e-3 * np.asarray(b["theta"])[None, :])
    assert np.median(rel) < 3e-6 and np.quantile(rel, 0.99) < 5e-5 and rel.max() < 5e-3, (
        np.median(rel), np.quantile(rel, 0.99), rel.max())
    assert np.abs(pay - rp).max() < 2e-3


def test_asset_zero_is_the_single_asset_gpu_path(S):
    """Weights e_0: asset 0 draws the single-asset words and its correlated normal is
    1.0 * z2_0, so its GPU path equals the single-option GPU path bit for bit."""
    b = W.basket(4, paths=3000, steps=40)
    b["w"] = (1.0, 0.0, 0.0, 0.0)
    single = W.option(S0=b["S0"][0], K=b["K"], kappa=b["kappa"][0], theta=b["theta"][0], xi=b["xi"][0],
                      rho=b["rho"][0], v0=b["v0"][0], steps=40, paths=3000, seed=b["seed"])
    xT, vT, pay = S.debug_basket_paths(b)
    sx, sv, sp = S.debug_paths(single)
    assert np.array_equal(xT[:, 0], sx) and np.array_equal(vT[:, 0], sv) and np.array_equal(pay, sp)


@pytest.mark.parametrize("d,paths", [(1, 6000), (4, 6000), (8, 6000), (13, 6000), (32, 6000), (13, 60000),
                                     (32, 60000), (13, 110000), (32, 110000), (32, 140000)])
@pytest.mark.parametrize("payoff", [0, 1])
def test_basket_european_price_every_tile(S, d, paths, payoff):
    """A single asset and every compiled asset tile and lane count: baskets of more than 8 assets
    with too few paths to fill the chip at one path per lane run the split kernel (tiles 16 and
    32) with 16 lanes per path at 6,000 paths (32 for 32 assets), 8 at 60,000 and 4 at 110,000
    (on 256 CUs); fewer
    assets run one path per lane (tiles 4 and 8), and 140,000 paths of 32 assets fill the chip at
    one path per lane (tile 32)."""
    b = W.basket(d, paths=paths, steps=16, payoff=payoff)
    say("basket european d", d, "payoff", payoff)
    g = S.basket_price(b)
    r, se = oracle.basket_price_european(ob(b))
    assert abs(g.price - r) <= 1e-4 * b0(b), (g.price, r)
    assert g.std_err == pytest.approx(se, rel=1e-3)


@pytest.mark.parametrize("scheme,d", [(0, 4), (1, 4), (2, 4), (3, 4), (0, 10)])
def test_basket_greeks_european(S, scheme, d):
    """d = 4 at one path per lane, d = 10 with several lanes per path (the split kernel)."""
    b = W.basket(d, paths=1 << 16, steps=32)
    say("basket greeks scheme", scheme)
    g = S.basket_greeks(b, scheme)
    p, se, dl, dls, gm, gms = oracle.basket_greeks(ob(b, scheme=scheme))
    P = b["paths"]
    assert abs(g.price - p) <= 1e-4 * b0(b)
    d_scale = np.maximum(np.abs(dl), dls * math.sqrt(P))
    dd = np.abs(np.array(g.delta) - dl)
    say("delta ratio", dd / (1e-4 * d_scale))
    assert (dd <= 1e-4 * d_scale).all(), (g.delta, dl)
    g_scale = np.maximum(np.abs(gm), gms * math.sqrt(P))
    dg = np.abs(np.array(g.gamma) - gm)
    say("gamma ratio", dg / (1e-3 * g_scale))
    assert (dg <= 1e-3 * g_scale).all(), (g.gamma, gm)
    G = np.array(g.gamma)
    assert np.array_equal(G, G.T)
    assert np.allclose(np.array(g.delta_se), dls, rtol=1e-2)


def test_basket_gamma_nan_for_perfect_spot_vol_correlation(S):
    b = W.basket(3, paths=4096, steps=8)
    b["rho"] = (-1.0,) + tuple(b["rho"][1:])
    g = S.basket_greeks(b)
    G = np.array(g.gamma)
    assert np.isnan(G[0, 0]) and np.isnan(G[0, 2]) and np.isfinite(G[1, 2])
    assert all(math.isfinite(x) for x in g.delta)


@pytest.mark.parametrize("scheme,d", [(0, 4), (2, 4), (0, 12)])
def test_basket_american(S, scheme, d):
    """Longstaff-Schwartz on the 10-function basis: the GPU's exercise policy valued by the
    oracle matches the GPU price; the in-sample prices agree within 3 SE; the coefficients of
    the last date match the oracle's where the policies agree; deltas at the GPU's exercise
    indices match the oracle's on the same indices."""
    b = W.basket(d, moneyness=1.1, payoff=2, paths=20000, steps=50)  # d = 12: the split kernel
    say("basket american scheme", scheme, "assets", d)
    g, tau, beta = S.debug_basket_lsm(b, scheme)
    assert beta.shape == (51, 10) and tau.min() >= 1 and tau.max() <= 50
    o = ob(b, scheme=scheme)
    v = oracle.basket_stopped_values(o, tau).mean()
    assert abs(g.price - v) <= 1e-4 * b0(b), (g.price, v)
    ref = oracle.basket_price_american(o)
    say("basket american", g.price, ref.price, g.std_err, "tau agreement", np.mean(tau == ref.tau))
    assert abs(g.price - ref.price) <= 3 * g.std_err
    assert abs(np.mean(tau < 50) - np.mean(ref.tau < 50)) <= 0.01
    np.testing.assert_allclose(beta[49], ref.beta[49], rtol=2e-3, atol=2e-3 * np.abs(ref.beta[49]).max())
    gr = S.basket_greeks(b, scheme)
    assert gr.price == g.price and all(math.isnan(x) for row in gr.gamma for x in row)
    _, _, dl, dls, _, _ = oracle.basket_greeks(o, tau=tau)
    scale = np.maximum(np.abs(dl), dls * math.sqrt(b["paths"]))
    assert (np.abs(np.array(gr.delta) - dl) <= 2e-3 * scale).all(), (gr.delta, dl)


def induction_consistency(b, scheme, tau, beta):
    """Self-consistency of a backward induction on the oracle's FP64 states of the same paths:
    (policy) the exercise index of every path is the first date whose coefficients say exercise
    (h > 0, h > phi . beta, regression valid), else N; (regression) each date's coefficients
    fit, by least squares over that date's in-the-money paths, the cash flows the policy
    realises after the date, valued at the date.  Returns (share of paths whose index the
    coefficients reproduce, largest difference of fitted continuation values relative to the
    RMS cash flow).  Both hold whatever the exercise decisions are, so they check the mechanics
    (date, discount, coefficients used) of inductions that differ path by path."""
    o = ob(b, scheme=scheme)
    N, P = b["steps"], b["paths"]
    X, V = oracle.basket_states(o)
    B0 = b0(b)
    tbar = float(np.dot(np.array(b["w"]) * np.array(b["S0"]), b["theta"])) / B0
    Bn = B0 * np.exp(X)
    h = np.maximum(Bn - b["K"], 0.0) if b["payoff"] in (0, 3) else np.maximum(b["K"] - Bn, 0.0)
    a, c = Bn / b["K"] - 1.0, V / tbar - 1.0
    phi = np.stack([np.ones_like(a), a, a * a, c, a * c, c * c, a ** 3, a * a * c, a * c * c, c ** 3])
    dt = b["T"] / N
    valid = np.array([np.any(beta[n] != 0.0) for n in range(N + 1)])
    ex = np.zeros((N, P), dtype=bool)  # row n - 1: exercise at date n
    for n in range(1, N):
        if valid[n]:
            ex[n - 1] = (h[n - 1] > 0.0) & (h[n - 1] > np.tensordot(beta[n], phi[:, n - 1], axes=1))
    first = np.where(ex.any(axis=0), ex.argmax(axis=0) + 1, N)
    share = float(np.mean(first == tau))
    worst = 0.0
    for n in range(1, N):
        if not valid[n]:
            continue
        later = ex[n:]  # dates n + 1 .. N - 1
        tn = np.where(later.any(axis=0), later.argmax(axis=0) + n + 1, N)
        y = h[tn - 1, np.arange(P)] * np.exp(-b["r"] * (tn - n) * dt)
        itm = h[n - 1] > 0.0
        A = phi[:, n - 1, itm].T
        ref, *_ = np.linalg.lstsq(A, y[itm], rcond=None)
        d = np.abs(A @ (beta[n] - ref)).max() / np.sqrt(np.mean(y[itm] ** 2))
        worst = max(worst, float(d))
    return share, worst


@pytest.mark.parametrize("scheme,d,steps", [(0, 4, 50), (2, 12, 30), (0, 3, 2), (0, 3, 1)])
def test_basket_american_per_date_induction(S, scheme, d, steps):
    """One launch per date on the same factor records (forced here; taken by itself for paths
    beyond the cooperative capacity).  Both inductions are self-consistent on the oracle's paths
    (exercise indices from the coefficients, coefficients from the realised cash flows); the
    GPU's exercise policy valued by the oracle matches the GPU price; the in-sample price agrees
    with the oracle's within 3 SE, and with the cooperative induction's within one SE (the two
    group the right-hand-side sums differently, and Longstaff-Schwartz carries a near-tie
    decision at one date into the regressions of the earlier ones, so their exercise indices
    differ path by path); deltas at the GPU's exercise indices match the oracle's on the same
    indices."""
    b = W.basket(d, moneyness=1.1, payoff=2, paths=20000, steps=steps)
    say("basket per-date induction scheme", scheme, "assets", d, "steps", steps)
    coop, tau_c, beta_c = S.debug_basket_lsm(b, scheme)
    S.set_lsm_launch(1)
    try:
        g, tau, beta = S.debug_basket_lsm(b, scheme)
        gr = S.basket_greeks(b, scheme)
    finally:
        S.set_lsm_launch(0)
    for name, t, bt in (("cooperative", tau_c, beta_c), ("per-date", tau, beta)):
        share, worst = induction_consistency(b, scheme, t, bt)
        say(name, "indices reproduced", share, "largest fitted-value difference / rms", worst)
        # the GPU forms the Gram and right-hand sides in FP32 (1.3e-4 measured for the cooperative
        # induction on the 4-asset case); coefficients one date late, a discount one step off or
        # indices one date late give 0.05 to 0.8 on the same case
        assert share > 0.999 and worst < 1e-3, (name, share, worst)
    o = ob(b, scheme=scheme)
    v = oracle.basket_stopped_values(o, tau).mean()
    assert abs(g.price - v) <= 1e-4 * b0(b), (g.price, v)
    ref = oracle.basket_price_american(o)
    say("per-date", g.price, "cooperative", coop.price, "oracle", ref.price, "same index", np.mean(tau == tau_c))
    assert abs(g.price - ref.price) <= max(3 * g.std_err, 1e-4 * b0(b))
    assert abs(g.price - coop.price) <= max(g.std_err, 1e-4 * b0(b))
    assert g.lsm_flags == coop.lsm_flags
    assert gr.price == g.price
    if not g.lsm_flags & 4:
        _, _, dl, dls, _, _ = oracle.basket_greeks(o, tau=tau)
        scale = np.maximum(np.abs(dl), dls * math.sqrt(b["paths"]))
        assert (np.abs(np.array(gr.delta) - dl) <= 2e-3 * scale).all(), (gr.delta, dl)


def test_basket_american_beyond_the_cooperative_capacity(S):
    """1.2 M paths, more than the cooperative launch holds (4 per lane of one 1024-thread block
    per CU): the induction runs one launch per date by itself; the GPU's exercise policy valued
    by the oracle matches the GPU price, and the in-sample prices agree within 3 SE."""
    b = W.basket(2, moneyness=1.1, payoff=2, paths=1_200_000, steps=8)
    g, tau, _ = S.debug_basket_lsm(b)
    o = ob(b)
    v = oracle.basket_stopped_values(o, tau).mean()
    say("basket beyond the cooperative capacity", g.price, v, g.std_err)
    assert abs(g.price - v) <= 1e-4 * b0(b), (g.price, v)
    ref = oracle.basket_price_american(o)
    assert abs(g.price - ref.price) <= 3 * g.std_err, (g.price, ref.price, g.std_err)


def test_basket_american_exercised_at_t0(S):
    """Deep in the money with a high rate: the intrinsic value wins at t_0; deltas are
    h'(B_0) w_i."""
    b = W.basket(3, moneyness=3.0, payoff=2, paths=4096, steps=10, r=0.2)
    g = S.basket_price(b)
    assert g.lsm_flags & 4 and g.price == pytest.approx(b["K"] - b0(b)) and g.std_err == 0.0
    gr = S.basket_greeks(b)
    np.testing.assert_allclose(gr.delta, [-w for w in b["w"]])


def test_split_kernel_paths_equal_the_one_path_per_lane_kernel(S):
    """Few paths and many assets run with several lanes per path (the split kernel).  Every
    asset's step is the same FP32 arithmetic in both kernels, so the terminal values of a
    5,000-path run (split) equal the first 5,000 paths of a 200,000-path run (one path per
    lane) bit for bit; the payoffs differ only in the order of the basket sum."""
    b = W.basket(12, paths=5000, steps=16)
    xs, vs, ps = S.debug_basket_paths(b)
    xl, vl, pl = S.debug_basket_paths(dict(b, paths=200000))
    assert np.array_equal(xs, xl[:5000]) and np.array_equal(vs, vl[:5000])
    # 12 FP32 terms of about 10 summed in another order: a few units of FP32 rounding of B
    np.testing.assert_allclose(ps, pl[:5000], rtol=0, atol=2e-6 * b0(b))


def test_table1_tiny_basket_american(S):
    """The paper's Tiny shape (5 assets, 126 steps, 25,000 paths) as one correlated American
    basket: the GPU's exercise policy valued by the oracle matches its price."""
    b = W.table1_basket("tiny")
    g, tau, _ = S.debug_basket_lsm(b)
    o = oracle.Basket(**b)
    v = oracle.basket_stopped_values(o, tau).mean()
    say("table1 tiny basket", g.price, v, g.std_err)
    assert abs(g.price - v) <= 1e-4 * b0(b)
    ref = oracle.basket_price_american(o)
    assert abs(g.price - ref.price) <= 3 * g.std_err


def test_basket_edge_cases(S):
    """Two paths and one step; identity correlation; deterministic variance (xi = 0 for every
    asset); a zero weight; an American basket with a single step (no regression date, so the
    price is max(h(B_0), e^{-r dt} mean h(B_1)))."""
    cases = [dict(paths=2, steps=1), dict(paths=3000, corr=tuple(tuple(float(i == j) for j in range(3))
                                                                 for i in range(3))),
             dict(paths=3000, xi=(0.0, 0.0, 0.0), rho=(0.0, 0.0, 0.0)), dict(paths=3000, w=(0.5, 0.0, 0.5))]
    for kw in cases:
        b = W.basket(3, steps=kw.pop("steps", 16), **kw)
        g = S.basket_price(b)
        r, _ = oracle.basket_price_european(ob(b))
        say("basket edge", kw.keys(), g.price, r)
        assert abs(g.price - r) <= 1e-4 * b0(b), (kw, g.price, r)
    b = W.basket(3, moneyness=1.1, payoff=2, paths=4000, steps=1)
    g = S.basket_price(b)
    ref = oracle.basket_price_american(ob(b))
    assert abs(g.price - ref.price) <= 1e-4 * b0(b) and g.lsm_flags == ref.lsm_flags | (4 if ref.exercised_at_t0 else 0)
