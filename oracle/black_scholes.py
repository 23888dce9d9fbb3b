"""Black-Scholes closed forms (TEST INFRASTRUCTURE ONLY).

With xi = 0 the Heston variance is deterministic; with v0 = theta it stays at
theta and the model is geometric Brownian motion with sigma^2 = theta.  These
textbook formulas are the prices and Greeks the Monte Carlo estimators must
reproduce in that limit.
"""
from __future__ import annotations

import math

from scipy.stats import norm


def _d12(S0, K, T, r, sigma):
    d1 = (math.log(S0 / K) + (r + 0.5 * sigma * sigma) * T) / (sigma * math.sqrt(T))
    return d1, d1 - sigma * math.sqrt(T)


def call(S0, K, T, r, sigma):
    d1, d2 = _d12(S0, K, T, r, sigma)
    return S0 * norm.cdf(d1) - K * math.exp(-r * T) * norm.cdf(d2)


def put(S0, K, T, r, sigma):
    d1, d2 = _d12(S0, K, T, r, sigma)
    return K * math.exp(-r * T) * norm.cdf(-d2) - S0 * norm.cdf(-d1)


def call_delta(S0, K, T, r, sigma):
    return norm.cdf(_d12(S0, K, T, r, sigma)[0])


def put_delta(S0, K, T, r, sigma):
    return call_delta(S0, K, T, r, sigma) - 1.0


def vega_sigma(S0, K, T, r, sigma):
    """d price / d sigma (same for calls and puts)."""
    d1, _ = _d12(S0, K, T, r, sigma)
    return S0 * norm.pdf(d1) * math.sqrt(T)


def call_rho(S0, K, T, r, sigma):
    _, d2 = _d12(S0, K, T, r, sigma)
    return K * T * math.exp(-r * T) * norm.cdf(d2)


def put_rho(S0, K, T, r, sigma):
    _, d2 = _d12(S0, K, T, r, sigma)
    return -K * T * math.exp(-r * T) * norm.cdf(-d2)


def gamma(S0, K, T, r, sigma):
    """d2 price / d S0^2 (same for calls and puts)."""
    d1, _ = _d12(S0, K, T, r, sigma)
    return norm.pdf(d1) / (S0 * sigma * math.sqrt(T))


def call_dT(S0, K, T, r, sigma):
    """d price / d T of the call (minus the time decay)."""
    d1, d2 = _d12(S0, K, T, r, sigma)
    return S0 * norm.pdf(d1) * sigma / (2.0 * math.sqrt(T)) + r * K * math.exp(-r * T) * norm.cdf(d2)


def put_dT(S0, K, T, r, sigma):
    """d price / d T of the put; by parity call_dT - r K e^{-rT}."""
    return call_dT(S0, K, T, r, sigma) - r * K * math.exp(-r * T)
