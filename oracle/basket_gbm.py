"""Two correlated geometric Brownian motions: reference values for arithmetic basket
options on B = w1 S1 + w2 S2 (the xi = 0 limit of the correlated Heston basket, where
each asset has the constant variance sigma_i^2 and the log-returns have correlation rho).

TEST INFRASTRUCTURE ONLY.

* :func:`european` -- the European price by one-dimensional Gauss-Hermite quadrature of a
  conditional Black-Scholes price: given the normal Z driving asset 1, ln S2_T is Gaussian
  with mean ln S2 + (r - sigma2^2/2) T + sigma2 sqrt(T) rho Z and variance
  sigma2^2 T (1 - rho^2), so E[(w2 S2_T - (K - w1 S1_T))^+ | Z] is Black's formula (or a
  forward when the effective strike is not positive).  Its first and second differences
  in S1, S2 give reference deltas and (cross-)gammas.
* :func:`bermudan` -- the two-asset binomial lattice of Boyle, Evnine and Gibbs (1989):
  each step moves ln S_i by +-sigma_i sqrt(dt), with the four joint moves weighted so that
  the lattice matches the means, variances and correlation of the log-returns; exercise is
  allowed every `sub` steps (the Monte Carlo dates).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import ndtr


def _black_undiscounted_call(F, k, sd):
    """E[(X - k)^+] for X lognormal with mean F and log-sd sd (k > 0, sd > 0)."""
    d1 = (np.log(F / k) + 0.5 * sd * sd) / sd
    return F * ndtr(d1) - k * ndtr(d1 - sd)


def european(S1, S2, w1, w2, K, T, r, s1, s2, rho, call=True, nodes=256):
    """Price of the European call (or put) on w1 S1_T + w2 S2_T with strike K."""
    x, wts = np.polynomial.hermite_e.hermegauss(nodes)  # weight exp(-x^2 / 2)
    wts = wts / math.sqrt(2.0 * math.pi)
    sqT = math.sqrt(T)
    S1T = S1 * np.exp((r - 0.5 * s1 * s1) * T + s1 * sqT * x)
    sd = s2 * sqT * math.sqrt(max(1.0 - rho * rho, 0.0))
    F2 = S2 * np.exp((r - 0.5 * s2 * s2) * T + s2 * sqT * rho * x + 0.5 * sd * sd)  # E[S2_T | x]
    Kp = K - w1 * S1T  # strike left for w2 S2_T
    fwd = w2 * F2 - Kp  # the conditional value when the option cannot end out of the money
    cond = np.where(Kp <= 0.0, fwd, 0.0)
    pos = Kp > 0.0
    if w2 > 0.0 and sd > 0.0:
        cond[pos] = w2 * _black_undiscounted_call(F2[pos], Kp[pos] / w2, sd)
    else:
        cond[pos] = np.maximum(fwd[pos], 0.0)
    c = math.exp(-r * T) * float(np.dot(wts, cond))
    if call:
        return c
    return c - (w1 * S1 + w2 * S2 - K * math.exp(-r * T))  # put-call parity


def greeks(S1, S2, w1, w2, K, T, r, s1, s2, rho, call=True, rel=1e-3):
    """(delta[2], gamma[2, 2]) by central differences of `european` (bump rel * S_i)."""
    S = np.array([S1, S2], dtype=float)
    h = rel * S

    def f(a, b):
        return european(a, b, w1, w2, K, T, r, s1, s2, rho, call)

    delta = np.array([(f(S1 + h[0], S2) - f(S1 - h[0], S2)) / (2 * h[0]),
                      (f(S1, S2 + h[1]) - f(S1, S2 - h[1])) / (2 * h[1])])
    p0 = f(S1, S2)
    g = np.zeros((2, 2))
    g[0, 0] = (f(S1 + h[0], S2) - 2 * p0 + f(S1 - h[0], S2)) / h[0] ** 2
    g[1, 1] = (f(S1, S2 + h[1]) - 2 * p0 + f(S1, S2 - h[1])) / h[1] ** 2
    g[0, 1] = g[1, 0] = (f(S1 + h[0], S2 + h[1]) - f(S1 + h[0], S2 - h[1])
                         - f(S1 - h[0], S2 + h[1]) + f(S1 - h[0], S2 - h[1])) / (4 * h[0] * h[1])
    return delta, g


def bermudan(S1, S2, w1, w2, K, T, r, s1, s2, rho, dates, sub=20, call=False, european_only=False):
    """Bermudan (exercise at t_n = n T / dates, n = 1..dates, and at t_0) basket option
    on the BEG lattice with `sub` steps per exercise interval."""
    n_steps = dates * sub
    dt = T / n_steps
    sq = math.sqrt(dt)
    m1, m2 = (r - 0.5 * s1 * s1) / s1, (r - 0.5 * s2 * s2) / s2
    p_uu = 0.25 * (1.0 + rho + sq * (m1 + m2))
    p_ud = 0.25 * (1.0 - rho + sq * (m1 - m2))
    p_du = 0.25 * (1.0 - rho + sq * (-m1 + m2))
    p_dd = 0.25 * (1.0 + rho - sq * (m1 + m2))
    if min(p_uu, p_ud, p_du, p_dd) < 0.0:
        raise ValueError("lattice probabilities negative: refine the lattice")
    disc = math.exp(-r * dt)

    def payoff(n):
        k = np.arange(n + 1)
        a = S1 * np.exp(s1 * sq * (2 * k - n))  # asset 1 after k up-moves of n
        b = S2 * np.exp(s2 * sq * (2 * k - n))
        B = w1 * a[:, None] + w2 * b[None, :]
        return np.maximum(B - K, 0.0) if call else np.maximum(K - B, 0.0)

    V = payoff(n_steps)
    for n in range(n_steps - 1, -1, -1):
        # node (i, j) at step n: i up-moves of asset 1, j of asset 2
        V = disc * (p_uu * V[1:, 1:] + p_ud * V[1:, :-1] + p_du * V[:-1, 1:] + p_dd * V[:-1, :-1])
        if not european_only and n % sub == 0:
            V = np.maximum(V, payoff(n))
    return float(V[0, 0])
