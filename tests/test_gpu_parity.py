"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs.

Tolerances (the method's floating point is FP32 on the GPU, FP64 in the oracle):
  * Philox words and the dyadic uniforms: bit-exact.
  * Box-Muller normals: |dz| <= 3e-6 (hardware log2 / sqrt ~1 ulp, sin/cos in
    revolutions ~1.3e-7 absolute, times |R| <= 5.77).
  * Prices: |dprice| <= 1e-4 * S0 at equal paths (and the oracle itself is
    within 3 SE of the closed form, checked in the CPU tests).
  * European Greeks: |dg| <= 1e-4 * max(|g|, s_g), s_g the per-path standard
    deviation of the Greek (its natural scale), same estimator in both.
  * American prices and Greeks: exercise decisions taken in FP32 on the GPU and
    FP64 in the oracle differ on near-tie paths, and a flip propagates to earlier
    regressions (see test_american_lsm); Greeks |dg| <= 2e-3 * max(|g|, s_g).
"""
import ctypes
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2402_12111_amd import workloads as W

pytestmark = pytest.mark.gpu

PRICE_TOL = 1e-4  # x S0


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


def relative_error(got, want, theta):
    """|got - want| / max(|want|, 1e-3 theta): relative, with a floor where the variance is 0."""
    want = np.asarray(want, dtype=np.float64)
    return np.abs(np.asarray(got, dtype=np.float64) - want) / np.maximum(np.abs(want), 1e-3 * np.asarray(theta))


def test_rng_words_uniforms_bit_exact(S):
    seed, stream, path0, npaths, step0, nsteps = 0xDEADBEEF12345678, 3, 123456, 700, 250, 6
    say("draws window", seed, stream, path0, npaths, step0, nsteps)
    w, u, z = S.debug_draws(seed, stream, path0, npaths, step0, nsteps)
    ref = oracle.rng_words(seed, stream, path0, npaths, step0, nsteps)
    assert np.array_equal(w, ref)
    ref_u = ((ref[..., :3] >> 9).astype(np.float64) + 0.5) * 2.0**-23
    assert np.array_equal(u.astype(np.float64), ref_u)
    bm = np.array([oracle.box_muller(a, b) for a, b in zip(ref_u[..., 0].ravel(), ref_u[..., 1].ravel())])
    dz = np.abs(z.reshape(-1, 2).astype(np.float64) - bm)
    assert dz.max() <= 3e-6, dz.max()


def test_rng_counter_edges(S):
    """Largest counters the layout allows: path near 2^30, step near 2^16, stream 2^32 - 1."""
    w, _, _ = S.debug_draws(2**64 - 1, 2**32 - 1, (1 << 30) - 5, 5, (1 << 16) - 3, 3)
    assert np.array_equal(w, oracle.rng_words(2**64 - 1, 2**32 - 1, (1 << 30) - 5, 5, (1 << 16) - 3, 3))


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_terminal_values_per_path(S, scheme):
    o = W.option(paths=5000, steps=64)  # ragged: 5000 is not a multiple of the tile
    say("paths", o, "scheme", scheme)
    xT, vT, pay = S.debug_paths(o, scheme)
    rx, rv, rp = oracle.simulate(oracle.Option(**o, scheme=scheme))
    dx = np.abs(xT - rx)
    assert np.median(dx) < 5e-6 and dx.max() < 1e-4, (np.median(dx), dx.max())
    # variance: relative to max(|v|, 1e-3 theta) (v reaches 0 in QE's exponential branch and
    # below it under Euler); measured median 1e-6 (QE), 3e-7 (TG), 1e-7 (FTE), max 8e-5 (TG)
    rel = relative_error(vT, rv, o["theta"])
    assert np.median(rel) < 3e-6 and np.quantile(rel, 0.99) < 2e-5 and rel.max() < 2e-4, (
        np.median(rel), np.quantile(rel, 0.99), rel.max())
    assert np.abs(pay - rp).max() < 2e-3


def test_terminal_values_exponential_branch(S):
    """High vol-of-vol and low kappa * theta put most steps in QE's exponential branch;
    FP32 and FP64 may pick different sides of u <= p on a few near-tie draws.  For the
    truncated Gaussian step the same parameters put psi near 32, where most of the
    Gaussian's mass is truncated at zero."""
    o = W.option(paths=4096, steps=50, kappa=0.5, theta=0.02, xi=0.8, v0=0.01, rho=-0.9, T=2.0)
    for scheme in (0, 2, 3):  # plain and martingale-corrected QE, truncated Gaussian
        xT, vT, pay = S.debug_paths(o, scheme)
        rx, rv, rp = oracle.simulate(oracle.Option(**o, scheme=scheme))
        dx = np.abs(xT - rx)
        assert np.median(dx) < 1e-5, scheme
        assert np.mean(dx > 1e-3) < 2e-3, scheme
        # the variance likewise: near-tie branch choices move a few paths (p99 of the relative
        # error measured 1.2e-5 for QE, 1.7e-5 for TG; most paths agree exactly)
        rel = relative_error(vT, rv, o["theta"])
        assert np.median(rel) < 1e-6 and np.quantile(rel, 0.99) < 5e-5, scheme
        assert np.mean(rel > 1e-3) < 2e-3, scheme


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
@pytest.mark.parametrize("payoff,K", [(0, 100.0), (1, 110.0)])
def test_european_price_c1(S, scheme, payoff, K):
    o = W.option(K=K, payoff=payoff)
    say("european", o, "scheme", scheme)
    g = S.price(o, scheme)
    r, se, _ = oracle.price_european(oracle.Option(**o, scheme=scheme))
    assert abs(g.price - r) <= PRICE_TOL * o["S0"], (g.price, r)
    assert g.std_err == pytest.approx(se, rel=1e-3)
    assert g.paths == o["paths"]


def test_european_edge_cases(S):
    """One step, two paths (the minimum), xi = 0 (deterministic variance), rho = +-1."""
    for kw in (dict(steps=1, paths=2), dict(steps=3, paths=130), dict(xi=0.0, rho=0.0),
               dict(rho=-1.0), dict(rho=1.0), dict(v0=0.0), dict(K=1e-3), dict(K=1e4)):
        o = W.option(paths=kw.pop("paths", 3000), **kw)
        say("edge", o)
        g = S.price(o)
        r, _, _ = oracle.price_european(oracle.Option(**o))
        assert abs(g.price - r) <= PRICE_TOL * o["S0"] + 1e-9 * abs(r), (kw, g.price, r)


def test_price_repeatable_and_batch_equals_single(S):
    opts = W.c3_batch(n=12, path_cap=5000)
    b1 = S.price_batch(opts)
    b2 = S.price_batch(opts)
    singles = [S.price(o) for o in opts]
    for x, y, z in zip(b1, b2, singles):
        assert x.price == y.price == z.price and x.std_err == z.std_err


def test_batch_c3_prefix_against_oracle(S):
    """The c3 set on a 4096-path prefix of every option (counter-based draws make a
    prefix the same paths), 96 options of mixed maturity, strike and step count."""
    opts = W.c3_batch(path_cap=4096)[:96]
    res = S.price_batch(opts)
    worst = 0.0
    for o, g in zip(opts, res):
        r, _, _ = oracle.price_european(oracle.Option(**o))
        worst = max(worst, abs(g.price - r))
        assert abs(g.price - r) <= PRICE_TOL * o["S0"], (o, g.price, r)
    say("c3 prefix worst |dprice|", worst)


def test_batch_mixed_european_american(S):
    opts = [W.option(paths=3000), W.option(K=110.0, payoff=2, steps=20, paths=4000, seed=7),
            W.option(K=95.0, payoff=1, steps=30, paths=2500, stream=5),
            W.option(K=100.0, payoff=3, steps=10, paths=2048, seed=9)]
    res = S.price_batch(opts)
    for o, g in zip(opts, res):
        r, _ = oracle.price(oracle.Option(**o))
        assert abs(g.price - r) <= PRICE_TOL * o["S0"], (o, g.price, r)


def test_batch_american_equals_single(S):
    """American options of a batch share cooperative launches (each option on its own
    blocks, options of one launch shape together while they fit co-resident); every
    option keeps the shape it takes alone, so batch and single results are the same
    bits.  24 paper-shaped options (25,000 paths) need several launches; the others
    add a call, an option exercised at t_0, one with too few in-the-money paths, and
    different path counts and step counts interleaved with European options."""
    opts = W.table1_shaped("large")[:24]
    for o in opts:
        o["steps"] = 40
    opts += [W.option(K=100.0, payoff=3, steps=12, paths=5000, seed=9),
             W.option(K=200.0, payoff=2, steps=8, paths=3000, seed=2),     # deep in the money: t_0
             W.option(K=40.0, payoff=2, steps=16, paths=2000, seed=3),     # almost never in the money
             W.option(paths=3000),
             W.option(K=110.0, payoff=2, steps=25, paths=70000, seed=7)]
    batch = S.price_batch(opts)
    for o, b in zip(opts, batch):
        one = S.price(o)
        assert (b.price, b.std_err, b.lsm_flags) == (one.price, one.std_err, one.lsm_flags), (o, b, one)
    assert batch[25].lsm_flags & 4 and batch[25].price == 200.0 - 100.0
    assert batch[26].lsm_flags & 1
    for i in (0, 13, 24, 28):
        r, _ = oracle.price(oracle.Option(**opts[i]))
        assert abs(batch[i].price - r) <= PRICE_TOL * opts[i]["S0"], (i, batch[i].price, r)


@pytest.mark.parametrize("scheme", [2, 3])
def test_other_schemes_american_and_batch(S, scheme):
    """The martingale-corrected QE and truncated Gaussian schemes through the
    Longstaff-Schwartz path (the spill kernel) and the batch kernel: the American price
    matches the oracle's value of the GPU's exercise policy to 1e-4 S0 and the oracle's
    own LSM price within 3 SE; a batch equals single calls bit for bit."""
    o = W.option(K=110.0, payoff=2, steps=50, paths=20000, seed=7, xi=0.6, rho=-0.8)
    say("scheme", scheme, o)
    g, tau, _ = S.debug_lsm(o, scheme)
    ro = oracle.Option(**o, scheme=scheme)
    assert abs(g.price - oracle.stopped_values(ro, tau).mean()) <= PRICE_TOL * o["S0"]
    ref = oracle.price_american(ro)
    say("american", g.price, ref.price, g.std_err)
    assert abs(g.price - ref.price) <= 3 * g.std_err
    plain = S.price(o, 0)
    assert plain.price != g.price  # the scheme changes the paths
    opts = [W.option(paths=3000 + 500 * i, K=90.0 + 5 * i, stream=i, xi=0.6) for i in range(6)] + [o]
    batch = S.price_batch(opts, scheme)
    for x, y in zip(opts, batch):
        one = S.price(x, scheme)
        assert (one.price, one.std_err) == (y.price, y.std_err)
    for x, y in zip(opts[:6], batch):
        r, _, _ = oracle.price_european(oracle.Option(**x, scheme=scheme))
        assert abs(y.price - r) <= PRICE_TOL * x["S0"], (x, y.price, r)


@pytest.mark.parametrize("case", ["small", "c2_full"])
def test_american_lsm(S, case):
    """Longstaff-Schwartz parity.  The in-sample exercise rule is discontinuous: one
    near-tie decision that FP32 and FP64 round to opposite sides changes that path's
    cash flow, which moves every earlier regression a little and can flip further
    near-ties (on the 20,000-path seed-7 sample any single FP32 rounding of S, h, y or
    the basis flips the same decision in the FP64 oracle itself: 4% of exercise
    indices move and the price by 0.007).  So the checks are: the price to 1e-4 S0;
    the first regression (date N-1, identical inputs up to FP32 rounding) through its
    fitted continuation values; the early-exercise fraction; most exercise indices."""
    if case == "small":
        o = W.option(K=110.0, payoff=2, steps=50, paths=20000, seed=7)
    else:
        o = W.c2_american()
    say("american", case, o)
    g, tau, beta = S.debug_lsm(o)
    ro = oracle.Option(**o)
    ref = oracle.price_american(ro)
    say("price", g.price, ref.price, "tau agreement", np.mean(tau == ref.tau))
    assert abs(g.price - ref.price) <= PRICE_TOL * o["S0"], (g.price, ref.price)
    # the GPU's exercise policy valued on the oracle's FP64 paths
    assert abs(g.price - oracle.stopped_values(ro, tau).mean()) <= PRICE_TOL * o["S0"]
    N = o["steps"]
    X, V = oracle.path_states(ro)
    Sn = o["S0"] * np.exp(X[N - 2])
    itm = o["K"] - Sn > 0
    a = Sn[itm] / o["K"] - 1.0
    c = np.maximum(V[N - 2][itm], 0.0) / o["theta"] - 1.0
    phi = np.stack([np.ones_like(a), a, a * a, c, a * c, c * c], axis=1)
    cont_gpu, cont_ref = phi @ beta[N - 1], phi @ ref.beta[N - 1]
    assert np.abs(cont_gpu - cont_ref).max() <= 1e-3 * np.abs(cont_ref).max(), np.abs(cont_gpu - cont_ref).max()
    assert abs(np.mean(tau < N) - np.mean(ref.tau < N)) <= 0.01
    assert np.mean(tau == ref.tau) >= 0.9
    assert tau.min() >= 1 and tau.max() <= N
    assert (g.lsm_flags & 3) == (ref.lsm_flags & 3)
    assert g.std_err == pytest.approx(ref.std_err, rel=2e-2)


@pytest.mark.parametrize("mode", [0, 1])
def test_american_launch_modes(S, mode):
    """The cooperative persistent induction (mode 0) and one launch per date (mode 1)."""
    o = W.option(K=110.0, payoff=2, steps=40, paths=30000, seed=11)
    S.set_lsm_launch(mode)
    try:
        g = S.price(o)
    finally:
        S.set_lsm_launch(0)
    ref = oracle.price_american(oracle.Option(**o))
    assert abs(g.price - ref.price) <= PRICE_TOL * o["S0"], (mode, g.price, ref.price)


def test_american_cooperative_grid_shapes(S):
    """Small grids make each lane carry several paths (PPL 2..16) and leave ragged tails."""
    o = W.option(K=105.0, payoff=2, steps=30, paths=50001, seed=12)
    ref = oracle.price_american(oracle.Option(**o))
    try:
        for gmax in (8, 40, 256):
            S.set_lsm_launch(0, gmax)
            g = S.price(o)
            assert abs(g.price - ref.price) <= PRICE_TOL * o["S0"], (gmax, g.price, ref.price)
    finally:
        S.set_lsm_launch(0, 64)  # the context's default grid cap


@pytest.mark.parametrize("steps", [2, 3, 4])
def test_american_few_dates(S, steps):
    """Two to four steps: the cooperative induction's requests for dates before the first
    (rows clamped to row 0, their values unused) and its first and last dates coincide or
    nearly so.  Ragged path counts at 1, 2 and 4 paths per lane (grid caps 256, 12, 8), each
    against the oracle's price and its valuation of the GPU's own exercise policy."""
    o = W.option(K=110.0, payoff=2, steps=steps, paths=20000 + 17, seed=9)
    ro = oracle.Option(**o)
    ref = oracle.price_american(ro)
    try:
        for gmax in (256, 12, 8):
            S.set_lsm_launch(0, gmax)
            g, tau, _ = S.debug_lsm(o)
            say("few dates", steps, "grid cap", gmax, g.price, ref.price)
            assert abs(g.price - ref.price) <= PRICE_TOL * o["S0"], (steps, gmax, g.price, ref.price)
            assert abs(g.price - oracle.stopped_values(ro, tau).mean()) <= PRICE_TOL * o["S0"]
            assert tau.min() >= 1 and tau.max() <= steps
    finally:
        S.set_lsm_launch(0, 64)  # the context's default grid cap


@pytest.mark.parametrize("gmax", [256, 40, 13])
def test_american_block_size_keeps_the_bits(S, gmax):
    """An option's paths per block (1024 x 1, 2 or 4: grid caps 256, 40 and 13 at 50,001
    paths, ragged) fix the induction's summation order.  On 1024-thread blocks (mode 4), on
    256-thread blocks with four times the paths per lane (mode 3) and as the planner picks
    (mode 0) the price, its error, the exercise indices and every beta are the same bits; the
    price matches the oracle."""
    o = W.option(K=105.0, payoff=2, steps=30, paths=50001, seed=12)
    runs = []
    try:
        for mode in (4, 3, 0):
            S.set_lsm_launch(mode, gmax)
            g, tau, beta = S.debug_lsm(o)
            say("block size mode", mode, "grid cap", gmax, g.price)
            runs.append((g, tau, beta))
    finally:
        S.set_lsm_launch(0, 64)  # the context's default grid cap
    g0, tau0, beta0 = runs[0]
    for g, tau, beta in runs[1:]:
        assert (g.price, g.std_err, g.lsm_flags) == (g0.price, g0.std_err, g0.lsm_flags)
        assert np.array_equal(tau, tau0) and np.array_equal(beta, beta0)
    ref = oracle.price_american(oracle.Option(**o))
    assert abs(g0.price - ref.price) <= PRICE_TOL * o["S0"], (gmax, g0.price, ref.price)


def test_american_block_size_keeps_the_bits_at_full_size(S):
    """One underlying of the large risk run (2^20 paths x 252 steps, 4096 paths per block):
    1024 threads x 4 paths per lane and 256 threads x 16 give the same bits; two such options
    share one launch (256-thread blocks) in a batch and equal single calls."""
    opts = W.c5_risk(2)
    try:
        S.set_lsm_launch(4)
        a = S.price(opts[0])
        S.set_lsm_launch(3)
        b = S.price(opts[0])
    finally:
        S.set_lsm_launch(0)
    say("full size", a.price, b.price)
    assert (a.price, a.std_err, a.lsm_flags) == (b.price, b.std_err, b.lsm_flags)
    batch = S.price_batch(opts)
    assert (batch[0].price, batch[0].std_err) == (a.price, a.std_err)
    one = S.price(opts[1])
    assert (batch[1].price, batch[1].std_err, batch[1].lsm_flags) == (one.price, one.std_err, one.lsm_flags)


def test_american_degenerate_regressions(S):
    """xi = 0 with v0 = theta: the variance columns are exactly zero and are dropped;
    deep OTM with few paths: dates with fewer than 6 ITM paths; deep ITM: t_0 exercise."""
    for kw in (dict(xi=0.0, rho=0.0, K=110.0), dict(K=40.0, paths=64, steps=10), dict(K=250.0, r=0.2, steps=10)):
        o = W.option(payoff=2, steps=kw.pop("steps", 30), paths=kw.pop("paths", 8192), seed=3, **kw)
        say("degenerate", o)
        g = S.price(o)
        ref = oracle.price_american(oracle.Option(**o))
        assert abs(g.price - ref.price) <= PRICE_TOL * o["S0"], (kw, g.price, ref.price)
        assert (g.lsm_flags & 3) == (ref.lsm_flags & 3)
        assert bool(g.lsm_flags & 4) == ref.exercised_at_t0


def _greek_tol(g, gse, P, rel):
    return rel * np.maximum(np.abs(g), gse * math.sqrt(P))


@pytest.mark.parametrize("payoff,K", [(0, 100.0), (1, 110.0)])
def test_greeks_european_vs_forward_mode(S, payoff, K):
    o = W.option(K=K, payoff=payoff, paths=32768, steps=64, seed=4)
    say("greeks european", o)
    gr = S.greeks(o)
    p, se, g, gse = oracle.greeks(oracle.Option(**o))
    tol = _greek_tol(g, gse, o["paths"], 1e-4)
    d = np.abs(np.array(gr.grads) - g)
    say("greeks", gr.grads, "oracle", g, "ratio", d / tol)
    assert (d <= tol).all(), (d, tol)
    assert abs(gr.price - p) <= PRICE_TOL * o["S0"]
    assert np.allclose(gr.grad_se, gse, rtol=1e-2)


def test_greeks_exponential_branch(S):
    o = W.option(K=100.0, payoff=1, paths=16384, steps=40, kappa=0.5, theta=0.02, xi=0.8, v0=0.01, rho=-0.9,
                 T=2.0, seed=4)
    gr = S.greeks(o)
    _, _, g, gse = oracle.greeks(oracle.Option(**o))
    d = np.abs(np.array(gr.grads) - g)
    assert (d <= _greek_tol(g, gse, o["paths"], 1e-3)).all(), (gr.grads, g)


def test_greeks_american_vs_forward_mode(S):
    o = W.option(K=110.0, payoff=2, paths=32768, steps=50, seed=4)
    gr = S.greeks(o)
    p, se, g, gse = oracle.greeks(oracle.Option(**o))
    d = np.abs(np.array(gr.grads) - g)
    say("greeks american", gr.grads, "oracle", g)
    assert (d <= _greek_tol(g, gse, o["paths"], 2e-3)).all(), (d, _greek_tol(g, gse, o["paths"], 2e-3))
    assert abs(gr.price - p) <= PRICE_TOL * o["S0"]
    # under the GPU's own exercise policy the Greeks are those of a fixed stopping
    # rule, which the oracle differentiates on its FP64 paths: the European bar
    _, tau, _ = S.debug_lsm(o)
    v, _, gt, gtse = oracle.greeks_at_tau(oracle.Option(**o), tau)
    d = np.abs(np.array(gr.grads) - gt)
    tol = _greek_tol(gt, gtse, o["paths"], 1e-4)
    say("same policy ratio", d / tol)
    assert (d <= tol).all(), (d, tol)
    assert abs(gr.price - v) <= PRICE_TOL * o["S0"]


@pytest.mark.parametrize("payoff,K", [(0, 100.0), (1, 110.0)])
def test_extended_greeks_european_vs_oracle(S, payoff, K):
    """d/dT and gamma from the same adjoint sweep against the oracle's forward-mode d/dT and
    its likelihood-ratio gamma on the same paths; the first 7 values are simr_greeks' bit for
    bit."""
    o = W.option(K=K, payoff=payoff, paths=32768, steps=64, seed=4)
    ge = S.greeks_ext(o)
    g7 = S.greeks(o)
    assert ge.grads[:7] == g7.grads and ge.price == g7.price
    p, se, g, gse = oracle.greeks_ext(oracle.Option(**o))
    d = np.abs(np.array(ge.grads) - g)
    tol = _greek_tol(g, gse, o["paths"], 1e-4)
    say("ext greeks", ge.grads[7:], "oracle", g[7:], "ratio", d[7:] / tol[7:])
    assert (d <= tol).all(), (d, tol)
    assert np.allclose(ge.grad_se, gse, rtol=1e-2)


@pytest.mark.parametrize("payoff,K", [(0, 100.0), (1, 110.0)])
def test_fte_greeks_vs_forward_mode(S, payoff, K):
    """Full-truncation Euler: the adjoint sweep against the oracle's forward-mode tangents on
    the same paths (all 9 values: the 7 Greeks, d/dT and gamma); FP32 and FP64 can put a step
    on opposite sides of v = 0, the scheme's kink, so the bar is 1e-3 of each Greek's scale."""
    o = W.option(K=K, payoff=payoff, paths=32768, steps=64, seed=4)
    ge = S.greeks_ext(o, scheme=1)
    p, se, g, gse = oracle.greeks_ext(oracle.Option(**o, scheme=1))
    d = np.abs(np.array(ge.grads) - g)
    tol = _greek_tol(g, gse, o["paths"], 1e-3)
    say("fte greeks ratio", d / tol)
    assert (d <= tol).all(), (d, tol)
    assert abs(ge.price - p) <= PRICE_TOL * o["S0"]


def test_fte_greeks_american_fixed_policy(S):
    o = W.option(K=110.0, payoff=2, paths=32768, steps=50, seed=4)
    ge = S.greeks_ext(o, scheme=1)
    _, tau, _ = S.debug_lsm(o, 1)
    v, _, g, gse = oracle.greeks_at_tau_ext(oracle.Option(**o, scheme=1), tau)
    d = np.abs(np.array(ge.grads[:8]) - g[:8])
    tol = _greek_tol(g[:8], gse[:8], o["paths"], 1e-3)
    assert (d <= tol).all(), (d, tol)
    assert abs(ge.price - v) <= PRICE_TOL * o["S0"] and math.isnan(ge.grads[8])


@pytest.mark.parametrize("payoff,K", [(0, 100.0), (1, 110.0)])
def test_martingale_corrected_greeks_vs_forward_mode(S, payoff, K):
    """Martingale-corrected QE: the adjoint of K0* = -ln E[exp(A V) | v] - K13 v (through A, the
    moments m and s^2 of the variance step and the branch it takes) against the oracle's
    forward-mode tangents on the same paths, all 9 values, at the plain QE bar; the first 7 are
    simr_greeks' bit for bit."""
    o = W.option(K=K, payoff=payoff, paths=32768, steps=64, seed=4)
    say("qe-m greeks", o)
    ge = S.greeks_ext(o, scheme=2)
    g7 = S.greeks(o, scheme=2)
    assert ge.grads[:7] == g7.grads and ge.price == g7.price
    p, se, g, gse = oracle.greeks_ext(oracle.Option(**o, scheme=2))
    d = np.abs(np.array(ge.grads) - g)
    tol = _greek_tol(g, gse, o["paths"], 1e-4)
    say("qe-m greeks", ge.grads, "oracle", g, "ratio", d / tol)
    assert (d <= tol).all(), (d, tol)
    assert abs(ge.price - p) <= PRICE_TOL * o["S0"]
    assert np.allclose(ge.grad_se, gse, rtol=1e-2)


def test_martingale_corrected_greeks_exponential_branch_and_american(S):
    """The exponential-branch moment p + beta (1 - p) / (beta - A) (xi 0.8, low kappa theta: QE
    mostly takes that branch) at the bar of plain QE's exponential-branch test, and an American
    put with the GPU's exercise indices held fixed against the oracle on the same policy."""
    o = W.option(K=100.0, payoff=1, paths=16384, steps=40, kappa=0.5, theta=0.02, xi=0.8, v0=0.01, rho=-0.9,
                 T=2.0, seed=4)
    gr = S.greeks(o, scheme=2)
    _, _, g, gse = oracle.greeks(oracle.Option(**o, scheme=2))
    d = np.abs(np.array(gr.grads) - g)
    say("qe-m exponential branch ratio", d / _greek_tol(g, gse, o["paths"], 1e-3))
    assert (d <= _greek_tol(g, gse, o["paths"], 1e-3)).all(), (gr.grads, g)
    am = W.option(K=110.0, payoff=2, paths=32768, steps=50, seed=4)
    ge = S.greeks_ext(am, scheme=2)
    _, tau, _ = S.debug_lsm(am, 2)
    v, _, g, gse = oracle.greeks_at_tau_ext(oracle.Option(**am, scheme=2), tau)
    tol = _greek_tol(g[:8], gse[:8], am["paths"], 1e-4)
    d = np.abs(np.array(ge.grads[:8]) - g[:8])
    say("qe-m american ratio", d / tol)
    assert (d <= tol).all(), (d, tol)
    assert abs(ge.price - v) <= PRICE_TOL * am["S0"] and math.isnan(ge.grads[8])


def test_martingale_corrected_greeks_where_the_moment_never_exists(S):
    """kappa 4, theta 0.3, xi 2, rho 0.9 on 3-year steps: E[exp(A V) | v] exists from no v, every
    step keeps the plain constant C0, and the corrected scheme's price and Greeks equal plain
    QE's on the GPU bit for bit (European put with d/dT and gamma, American put); the put
    against the oracle at the plain bar."""
    base = dict(K=100.0, T=6.0, kappa=4.0, theta=0.3, xi=2.0, rho=0.9, v0=0.3, steps=2, paths=20000, seed=7)
    for payoff in (1, 2):
        o = W.option(payoff=payoff, **base)
        a, b = S.greeks_ext(o, scheme=0), S.greeks_ext(o, scheme=2)
        assert a.price == b.price and a.std_err == b.std_err
        assert np.array_equal(a.grads, b.grads, equal_nan=True) and np.array_equal(a.grad_se, b.grad_se, equal_nan=True)
    o = W.option(payoff=1, **base)
    ge = S.greeks_ext(o, scheme=2)
    p, se, g, gse = oracle.greeks_ext(oracle.Option(**o, scheme=2))
    d = np.abs(np.array(ge.grads) - g)
    tol = _greek_tol(g, gse, o["paths"], 1e-4)
    say("qe-m fallback ratio", d / tol)
    assert (d <= tol).all(), (d, tol)


@pytest.mark.parametrize("payoff,K", [(0, 100.0), (1, 110.0)])
def test_truncated_gaussian_greeks_vs_forward_mode(S, payoff, K):
    """Truncated Gaussian: the adjoint through the table of mu / m and log2(sigma / m) and of
    their exact derivatives in log2(psi) against the oracle's forward-mode tangents (r(psi)
    differentiated implicitly) on the same paths, all 9 values, at the plain QE bar; the first
    7 are simr_greeks' bit for bit."""
    o = W.option(K=K, payoff=payoff, paths=32768, steps=64, seed=4)
    say("tg greeks", o)
    ge = S.greeks_ext(o, scheme=3)
    g7 = S.greeks(o, scheme=3)
    assert ge.grads[:7] == g7.grads and ge.price == g7.price
    p, se, g, gse = oracle.greeks_ext(oracle.Option(**o, scheme=3))
    d = np.abs(np.array(ge.grads) - g)
    tol = _greek_tol(g, gse, o["paths"], 1e-4)
    say("tg greeks", ge.grads, "oracle", g, "ratio", d / tol)
    assert (d <= tol).all(), (d, tol)
    assert abs(ge.price - p) <= PRICE_TOL * o["S0"]
    assert np.allclose(ge.grad_se, gse, rtol=1e-2)


def test_truncated_gaussian_greeks_truncating_and_american(S):
    """A low Feller ratio (xi 0.8, kappa theta 0.01: the step truncates at zero often and psi
    spans the table) at the bar of plain QE's exponential-branch test, and an American put with
    the GPU's exercise indices held fixed against the oracle on the same policy."""
    o = W.option(K=100.0, payoff=1, paths=16384, steps=40, kappa=0.5, theta=0.02, xi=0.8, v0=0.01, rho=-0.9,
                 T=2.0, seed=4)
    gr = S.greeks(o, scheme=3)
    _, _, g, gse = oracle.greeks(oracle.Option(**o, scheme=3))
    d = np.abs(np.array(gr.grads) - g)
    say("tg truncating ratio", d / _greek_tol(g, gse, o["paths"], 1e-3))
    assert (d <= _greek_tol(g, gse, o["paths"], 1e-3)).all(), (gr.grads, g)
    am = W.option(K=110.0, payoff=2, paths=32768, steps=50, seed=4)
    ge = S.greeks_ext(am, scheme=3)
    _, tau, _ = S.debug_lsm(am, 3)
    v, _, g, gse = oracle.greeks_at_tau_ext(oracle.Option(**am, scheme=3), tau)
    tol = _greek_tol(g[:8], gse[:8], am["paths"], 1e-4)
    d = np.abs(np.array(ge.grads[:8]) - g[:8])
    say("tg american ratio", d / tol)
    assert (d <= tol).all(), (d, tol)
    assert abs(ge.price - v) <= PRICE_TOL * am["S0"] and math.isnan(ge.grads[8])


def test_extended_greeks_american_fixed_policy(S):
    """American put: d/dT with the GPU's exercise indices held fixed against the oracle's on the
    same policy; gamma is not defined for a stopping rule (NaN)."""
    o = W.option(K=110.0, payoff=2, paths=32768, steps=50, seed=4)
    ge = S.greeks_ext(o)
    _, tau, _ = S.debug_lsm(o)
    _, _, g, gse = oracle.greeks_at_tau_ext(oracle.Option(**o), tau)
    tol = _greek_tol(g[:8], gse[:8], o["paths"], 1e-4)
    d = np.abs(np.array(ge.grads[:8]) - g[:8])
    assert (d <= tol).all(), (d, tol)
    assert math.isnan(ge.grads[8]) and math.isnan(g[8])


@pytest.mark.parametrize("ck", [8, 32])
@pytest.mark.parametrize("payoff,K", [(1, 100.0), (2, 110.0)])
@pytest.mark.parametrize("scheme", [0, 2, 3])
def test_greeks_checkpoint_interval_does_not_change_the_result(S, ck, payoff, K, scheme):
    """QE, martingale-corrected QE and truncated Gaussian: the segment length of the reverse
    sweep changes nothing but the grouping of FP64 block sums."""
    o = W.option(K=K, payoff=payoff, paths=8192, steps=70, seed=2)
    a = S.greeks(o, scheme, checkpoint_every=16)
    b = S.greeks(o, scheme, checkpoint_every=ck)
    # the recomputed segments are the forward pass bit for bit and the order in which a block
    # sweeps its paths does not depend on the segment length; 32-step segments sweep in blocks of
    # 512 paths instead of 1024, which regroups only the FP64 block sums
    assert a.price == b.price
    if ck == 8:
        assert a.grads == b.grads
    else:
        assert np.allclose(a.grads, b.grads, rtol=1e-12, atol=0.0), (a.grads, b.grads)


def test_autograd_function(S):
    import torch
    o = S.Option(**W.option(K=100.0, payoff=1, paths=8192, steps=32))
    params = [torch.tensor(getattr(o, n), dtype=torch.float64, requires_grad=True) for n in S.GREEK_NAMES]
    price = S.HestonPrice.apply(*params, o)
    price.backward()
    gr = S.greeks(o)
    assert price.item() == pytest.approx(gr.price)
    for p, g in zip(params, gr.grads):
        assert p.grad.item() == pytest.approx(g)


def test_workspace_too_small_is_rejected(S):
    import ctypes
    L = S.library()
    o = S.Option(**W.option())._c()
    prm = S._Params(0, 0, 0, 0)
    out = S._Result(-1.0, -1.0, -1, -1, 0)
    ws = S.workspace(1 << 20)
    rc = L.simr_price(S.context(), ctypes.byref(o), ctypes.byref(prm), ctypes.byref(out),
                      ctypes.c_void_p(ws.data_ptr()), 1024, S._stream())
    assert rc == -1 and b"workspace" in L.simr_last_error()
    assert out.price == -1.0


def test_broadie_kaya_exact_scheme(S):
    """The Broadie-Kaya exact scheme (FP64 on the device): per-path terminal values against
    the oracle's on the same uniforms (the FP32 state between steps is the only difference),
    European prices at equal paths, and an American put through the write-out and the induction
    (the GPU policy valued by the oracle)."""
    o = W.option(steps=4, paths=3000, seed=31)
    xT, vT, pay = S.debug_paths(o, 4)
    rx, rv, rp = oracle.simulate(oracle.Option(**o, scheme=4))
    dx = np.abs(xT - rx)
    say("bk paths", np.median(dx), dx.max(), np.abs(vT - rv).max())
    assert np.median(dx) < 1e-6 and dx.max() < 1e-4
    assert np.abs(vT - rv).max() < 1e-5
    for payoff, K in ((0, 100.0), (1, 110.0)):
        oo = W.option(K=K, payoff=payoff, steps=2, paths=8192, seed=5)
        g = S.price(oo, 4)
        r, se, _ = oracle.price_european(oracle.Option(**oo, scheme=4))
        assert abs(g.price - r) <= PRICE_TOL * oo["S0"], (payoff, g.price, r)
        assert g.std_err == pytest.approx(se, rel=1e-3)
    am = W.option(K=110.0, payoff=2, steps=8, paths=4096, seed=9)
    g, tau, _ = S.debug_lsm(am, 4)
    ro = oracle.Option(**am, scheme=4)
    assert abs(g.price - oracle.stopped_values(ro, tau).mean()) <= PRICE_TOL * am["S0"]
    ref = oracle.price_american(ro)
    assert abs(g.price - ref.price) <= 3 * g.std_err
    with pytest.raises(S.SimrError):
        S.greeks(o, 4)


def test_exchange_failure_is_reported_and_recovered(S):
    """Failure handling of the cooperative induction, forced from the host: with the exchange
    marked as failed (launch mode 2) every wait gives up at once, the launch completes and the
    call reports SIMR_ENUMERIC, for single options and baskets; the next call in the normal
    mode prices as before."""
    o = W.option(K=110.0, payoff=2, steps=20, paths=8192, seed=7)
    b = W.basket(3, moneyness=1.1, payoff=2, paths=4096, steps=10)
    before = S.price(o)
    S.set_lsm_launch(2)
    try:
        for call in (lambda: S.price(o), lambda: S.greeks(o), lambda: S.basket_price(b)):
            with pytest.raises(S.SimrError) as e:
                call()
            assert e.value.status == -5 and "timed out" in str(e.value)
    finally:
        S.set_lsm_launch(0)
    after = S.price(o)
    assert (after.price, after.std_err) == (before.price, before.std_err)
    assert S.basket_price(b).price > 0


def test_profiling_records_only_the_selected_groups(S):
    """simr_profile_groups: a zero mask or bits beyond the 7 groups are refused; with only the
    induction's group selected, an American price records induction launches and nothing else,
    and the price is the unprofiled one bit for bit."""
    L = S.library()
    L.simr_profile_groups.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
    L.simr_profile_enable.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.simr_profile_read.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64)]
    L.simr_profile_reset.argtypes = [ctypes.c_void_p]
    ctx = S.context()
    assert L.simr_profile_groups(ctx, 0) == -1
    assert L.simr_profile_groups(ctx, 1 << 7) == -1
    o = W.option(K=110.0, payoff=2, steps=16, paths=8192, seed=7)
    want = S.price(o)
    try:
        assert L.simr_profile_reset(ctx) == 0
        assert L.simr_profile_groups(ctx, 1 << 2) == 0
        assert L.simr_profile_enable(ctx, 1) == 0
        got = S.price(o)
        assert L.simr_profile_enable(ctx, 0) == 0
        for g in range(7):
            ms, n = ctypes.c_double(), ctypes.c_int64()
            assert L.simr_profile_read(ctx, g, ctypes.byref(ms), ctypes.byref(n)) == 0
            assert (n.value > 0 and ms.value > 0.0) if g == 2 else n.value == 0, (g, n.value)
        assert got.price == want.price and got.std_err == want.std_err
    finally:
        L.simr_profile_enable(ctx, 0)
        L.simr_profile_groups(ctx, (1 << 7) - 1)
        L.simr_profile_reset(ctx)
