"""Heston (1993) semi-closed-form European prices (TEST INFRASTRUCTURE ONLY).

The characteristic function of ln S_T is written in the form of Albrecher,
Mayer, Schoutens and Tistaert (2007, "The little Heston trap"), which keeps the
complex logarithm on its principal branch for long maturities:

    phi(u) = exp( i u (ln S0 + r T)
                  + (kappa theta / xi^2) [ (kappa - rho xi i u - d) T
                                           - 2 ln((1 - g e^{-d T}) / (1 - g)) ]
                  + (v0 / xi^2) (kappa - rho xi i u - d) (1 - e^{-d T}) / (1 - g e^{-d T}) )
    d = sqrt((rho xi i u - kappa)^2 + xi^2 (i u + u^2))
    g = (kappa - rho xi i u - d) / (kappa - rho xi i u + d)

and the call is  C = S0 P1 - K e^{-rT} P2  with the two exercise probabilities

    P1 = 1/2 + (1/pi) int_0^inf Re[ e^{-i u ln K} phi(u - i) / (i u phi(-i)) ] du
    P2 = 1/2 + (1/pi) int_0^inf Re[ e^{-i u ln K} phi(u) / (i u) ] du.

The put follows from put-call parity.  The paper itself prints no prices; this
closed form is the reference the Monte Carlo estimators converge to.
"""
from __future__ import annotations

import cmath
import math

import numpy as np
from scipy import integrate


def char_fn(u, S0, T, r, kappa, theta, xi, rho, v0):
    """phi(u) = E[exp(i u ln S_T)] for complex u (scalar)."""
    iu = 1j * u
    a = kappa - rho * xi * iu
    d = cmath.sqrt((rho * xi * iu - kappa) ** 2 + xi * xi * (iu + u * u))
    g = (a - d) / (a + d)
    edt = cmath.exp(-d * T)
    c_term = (kappa * theta / (xi * xi)) * ((a - d) * T - 2.0 * cmath.log((1.0 - g * edt) / (1.0 - g)))
    d_term = (v0 / (xi * xi)) * (a - d) * (1.0 - edt) / (1.0 - g * edt)
    return cmath.exp(iu * (math.log(S0) + r * T) + c_term + d_term)


def _probabilities(S0, K, T, r, kappa, theta, xi, rho, v0, upper=None):
    lnK = math.log(K)
    phi_mi = char_fn(-1j, S0, T, r, kappa, theta, xi, rho, v0)  # = S0 e^{rT}

    def f1(u):
        val = cmath.exp(-1j * u * lnK) * char_fn(u - 1j, S0, T, r, kappa, theta, xi, rho, v0) / (1j * u * phi_mi)
        return val.real

    def f2(u):
        val = cmath.exp(-1j * u * lnK) * char_fn(u, S0, T, r, kappa, theta, xi, rho, v0) / (1j * u)
        return val.real

    hi = np.inf if upper is None else upper
    i1, _ = integrate.quad(f1, 0.0, hi, limit=2000, epsabs=1e-11, epsrel=1e-10)
    i2, _ = integrate.quad(f2, 0.0, hi, limit=2000, epsabs=1e-11, epsrel=1e-10)
    return 0.5 + i1 / math.pi, 0.5 + i2 / math.pi


def call_price(S0, K, T, r, kappa, theta, xi, rho, v0):
    p1, p2 = _probabilities(S0, K, T, r, kappa, theta, xi, rho, v0)
    return S0 * p1 - K * math.exp(-r * T) * p2


def put_price(S0, K, T, r, kappa, theta, xi, rho, v0):
    return call_price(S0, K, T, r, kappa, theta, xi, rho, v0) - S0 + K * math.exp(-r * T)


def price(opt) -> float:
    """European price of an :class:`oracle.Option` (payoff 0 = call, 1 = put)."""
    args = (opt.S0, opt.K, opt.T, opt.r, opt.kappa, opt.theta, opt.xi, opt.rho, opt.v0)
    return call_price(*args) if opt.payoff == 0 else put_price(*args)


def call_price_mp(S0, K, T, r, kappa, theta, xi, rho, v0, dps=30):
    """The same integrals evaluated with mpmath at `dps` digits (quadrature check)."""
    import mpmath as mp
    mp.mp.dps = dps
    S0, K, T, r, kappa, theta, xi, rho, v0 = map(mp.mpf, (S0, K, T, r, kappa, theta, xi, rho, v0))
    lnK = mp.log(K)

    def cf(u):
        iu = 1j * u
        a = kappa - rho * xi * iu
        d = mp.sqrt((rho * xi * iu - kappa) ** 2 + xi * xi * (iu + u * u))
        g = (a - d) / (a + d)
        edt = mp.exp(-d * T)
        c_term = (kappa * theta / (xi * xi)) * ((a - d) * T - 2 * mp.log((1 - g * edt) / (1 - g)))
        d_term = (v0 / (xi * xi)) * (a - d) * (1 - edt) / (1 - g * edt)
        return mp.exp(iu * (mp.log(S0) + r * T) + c_term + d_term)

    phi_mi = cf(-1j)
    f1 = lambda u: mp.re(mp.exp(-1j * u * lnK) * cf(u - 1j) / (1j * u * phi_mi))
    f2 = lambda u: mp.re(mp.exp(-1j * u * lnK) * cf(u) / (1j * u))
    p1 = mp.mpf(0.5) + mp.quad(f1, [0, 1, 10, 50, mp.inf]) / mp.pi
    p2 = mp.mpf(0.5) + mp.quad(f2, [0, 1, 10, 50, mp.inf]) / mp.pi
    return float(S0 * p1 - K * mp.exp(-r * T) * p2)
