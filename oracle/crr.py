"""Cox-Ross-Rubinstein binomial trees (TEST INFRASTRUCTURE ONLY).

In the limit xi = 0, rho = 0, v0 = theta = sigma^2 the Heston model is GBM,
and the Longstaff-Schwartz problem becomes a Bermudan option whose exercise
dates are the Monte Carlo dates t_1..t_N (plus t_0 through the max with the
intrinsic value).  This tree prices that Bermudan option with `sub` binomial
steps between consecutive exercise dates (CRR 1979: u = e^{sigma sqrt(h)},
d = 1/u, risk-neutral up-probability (e^{r h} - d)/(u - d)), and prices the
European option with no early exercise for the convergence check against
Black-Scholes.
"""
from __future__ import annotations

import math

import numpy as np


def bermudan(S0, K, T, r, sigma, n_dates, sub=64, put=True, exercise_t0=True, european=False):
    M = n_dates * sub
    h = T / M
    u = math.exp(sigma * math.sqrt(h))
    d = 1.0 / u
    q = (math.exp(r * h) - d) / (u - d)
    disc = math.exp(-r * h)
    j = np.arange(M + 1)
    S = S0 * u ** (M - 2 * j)  # node j at the last level: M-j ups, j downs
    V = np.maximum(K - S, 0.0) if put else np.maximum(S - K, 0.0)
    for level in range(M - 1, -1, -1):
        V = disc * (q * V[:-1] + (1.0 - q) * V[1:])
        if european:
            continue
        if level % sub == 0 and (level > 0 or exercise_t0):
            jj = np.arange(level + 1)
            S = S0 * u ** (level - 2 * jj)
            ex = np.maximum(K - S, 0.0) if put else np.maximum(S - K, 0.0)
            V = np.maximum(V, ex)
    return float(V[0])
