"""Seeded synthetic workloads (input recipes only; no pricing arithmetic).

The paper measures SIMR on its own problem sizes (Sec. 3, Table 1: A assets x T
steps x P = 25k paths) with inputs streamed from the host; neither its data nor
the STAC-A2 inputs are available, so these seeded Heston option sets stand in
for them.  Each option is a plain dict with the keys
    S0 K T r kappa theta xi rho v0 payoff steps paths seed stream
that both the GPU binding and the CPU oracle accept.  Payoff codes:
0 European call, 1 European put, 2 American put, 3 American call.

  c1_european     one European call, 8192 paths x 64 steps, Philox seed 1
  c2_american     American put K=110, 131072 paths x 252 steps, seed 7
  c3_batch        1024 European calls with parameters drawn uniformly
                  (kappa in [0.5,3], theta in [0.02,0.09], xi in [0.1,0.8],
                  rho in [-0.9,0], v0 in [0.01,0.09], K in [70,130],
                  T in {0.25,0.5,1,2}, paths log-uniform in [16384,262144],
                  steps = 252 T) from numpy default_rng(3); seed 3, stream i
  c4_greeks       European put K=100 and American put K=110 on 262144 x 252,
                  seed 4, adjoint checkpoints every 16 steps
  c5_risk         64 American puts (K=110, T=1) whose Heston parameters are
                  drawn from the c3 ranges with default_rng(5); 1,048,576 x 252,
                  seed 5, stream u
  table1_shaped   the paper's Tiny/Small/Medium/Large shapes (5/10/20/30 options
                  x 126/126/252/504 steps x 25,000 paths), American puts with
                  c3-range parameters from default_rng(11)

Baskets (dicts with per-asset tuples S0 w kappa theta xi rho v0, the d x d corr,
and K T r payoff steps paths seed stream):
  basket          d assets with c3-range Heston parameters and spots uniform in
                  [80, 120] from default_rng(seed), equal weights 1/d, a
                  one-factor correlation C_ij = b_i b_j (i != j) with loadings
                  b_i uniform in [0.3, 0.8] (positive definite by construction),
                  the strike at B_0 = sum w_i S0_i (money-ness set by `moneyness`)
  basket_risk     the 8-asset European call (262,144 paths x 252 steps, seed 13)
                  and American put at 1.1 B_0 (131,072 x 252, seed 14)
  table1_basket   the paper's Table 1 asset counts as one correlated basket each
                  (5/10/20/30 assets x 126/126/252/504 steps x 25,000 paths),
                  American puts at 1.1 B_0, seed 11
"""
from __future__ import annotations

import math

import numpy as np

EURO_CALL, EURO_PUT, AMER_PUT, AMER_CALL = 0, 1, 2, 3

HESTON_C1 = dict(S0=100.0, K=100.0, T=1.0, r=0.02, kappa=1.5, theta=0.04, xi=0.3, rho=-0.7, v0=0.04)


def option(**kw) -> dict:
    d = dict(HESTON_C1, payoff=EURO_CALL, steps=64, paths=8192, seed=1, stream=0)
    d.update(kw)
    return d


def c1_european() -> dict:
    return option()


def c2_american() -> dict:
    return option(K=110.0, payoff=AMER_PUT, steps=252, paths=131072, seed=7)


def _draw_heston(rng, n):
    return dict(kappa=rng.uniform(0.5, 3.0, n), theta=rng.uniform(0.02, 0.09, n), xi=rng.uniform(0.1, 0.8, n),
                rho=rng.uniform(-0.9, 0.0, n), v0=rng.uniform(0.01, 0.09, n))


def c3_batch(n: int = 1024, seed: int = 3, path_cap: int | None = None) -> list[dict]:
    """The batched-pricing set.  `path_cap` truncates every path count (a prefix of
    the same paths, since the random numbers are counter-based)."""
    rng = np.random.default_rng(seed)
    h = _draw_heston(rng, n)
    K = rng.uniform(70.0, 130.0, n)
    T = rng.choice(np.array([0.25, 0.5, 1.0, 2.0]), n)
    P = np.rint(np.exp(rng.uniform(math.log(16384), math.log(262144), n))).astype(np.int64)
    out = []
    for i in range(n):
        paths = int(P[i]) if path_cap is None else min(int(P[i]), path_cap)
        out.append(option(K=float(K[i]), T=float(T[i]), kappa=float(h["kappa"][i]), theta=float(h["theta"][i]),
                          xi=float(h["xi"][i]), rho=float(h["rho"][i]), v0=float(h["v0"][i]), payoff=EURO_CALL,
                          steps=int(round(252 * T[i])), paths=paths, seed=3, stream=i))
    return out


def c4_greeks() -> list[dict]:
    return [option(K=100.0, payoff=EURO_PUT, steps=252, paths=262144, seed=4),
            option(K=110.0, payoff=AMER_PUT, steps=252, paths=262144, seed=4)]


def c5_risk(n: int = 64, paths: int = 1 << 20) -> list[dict]:
    rng = np.random.default_rng(5)
    h = _draw_heston(rng, n)
    return [option(K=110.0, T=1.0, kappa=float(h["kappa"][u]), theta=float(h["theta"][u]), xi=float(h["xi"][u]),
                   rho=float(h["rho"][u]), v0=float(h["v0"][u]), payoff=AMER_PUT, steps=252, paths=paths, seed=5,
                   stream=u) for u in range(n)]


TABLE1 = {"tiny": (5, 126), "small": (10, 126), "medium": (20, 252), "large": (30, 504)}


def table1_shaped(size: str, paths: int = 25000) -> list[dict]:
    A, N = TABLE1[size]
    rng = np.random.default_rng(11)
    h = _draw_heston(rng, A)
    return [option(K=110.0, T=N / 252.0, kappa=float(h["kappa"][a]), theta=float(h["theta"][a]),
                   xi=float(h["xi"][a]), rho=float(h["rho"][a]), v0=float(h["v0"][a]), payoff=AMER_PUT, steps=N,
                   paths=paths, seed=11, stream=a) for a in range(A)]


def path_steps(opts) -> int:
    if isinstance(opts, dict):
        opts = [opts]
    return int(sum(o["paths"] * o["steps"] for o in opts))


def basket(d: int = 4, seed: int = 13, moneyness: float = 1.0, **kw) -> dict:
    rng = np.random.default_rng(seed)
    h = _draw_heston(rng, d)
    S0 = rng.uniform(80.0, 120.0, d)
    load = rng.uniform(0.3, 0.8, d)
    C = np.outer(load, load)
    np.fill_diagonal(C, 1.0)
    w = np.full(d, 1.0 / d)
    B0 = float(w @ S0)
    b = dict(S0=tuple(float(x) for x in S0), w=tuple(float(x) for x in w),
             kappa=tuple(float(x) for x in h["kappa"]), theta=tuple(float(x) for x in h["theta"]),
             xi=tuple(float(x) for x in h["xi"]), rho=tuple(float(x) for x in h["rho"]),
             v0=tuple(float(x) for x in h["v0"]), corr=tuple(tuple(float(x) for x in row) for row in C),
             K=moneyness * B0, T=1.0, r=0.02, payoff=EURO_CALL, steps=64, paths=8192, seed=seed, stream=0)
    b.update(kw)
    return b


def basket_risk() -> list[dict]:
    return [basket(8, seed=13, steps=252, paths=262144),
            basket(8, seed=14, moneyness=1.1, payoff=AMER_PUT, steps=252, paths=131072)]


def table1_basket(size: str, paths: int = 25000) -> dict:
    A, N = TABLE1[size]
    return basket(A, seed=11, moneyness=1.1, payoff=AMER_PUT, T=N / 252.0, steps=N, paths=paths)


def asset_path_steps(b: dict) -> int:
    return int(len(b["S0"]) * b["paths"] * b["steps"])
