"""Plain FP64 CPU oracle for the Heston Monte Carlo / Longstaff-Schwartz hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it to check and time the GPU path.  The product never
imports it, and the two share no code.

Contents
  * ``libsimr_oracle.so`` (``simr_oracle.c``): Philox4x32-10, the dyadic uniform
    map, Box-Muller, Andersen's QE variance and log-price steps, full-truncation
    Euler, European pricing, Longstaff-Schwartz, forward-mode pathwise Greeks.
    Every step is written in double precision in the order the method states it.
  * :mod:`oracle.heston_cf` -- the Heston (1993) semi-closed-form price through
    the characteristic function in the Albrecher et al. (2007) form.
  * :mod:`oracle.black_scholes` -- Black-Scholes prices and Greeks (the xi -> 0,
    rho = 0 limit of the model).
  * :mod:`oracle.crr` -- a Cox-Ross-Rubinstein binomial tree for Bermudan puts
    (the GBM limit of the Longstaff-Schwartz problem).
  * Correlated baskets (``ref_basket_*`` in ``simr_oracle.c``, :class:`Basket`): d Heston
    assets with Cholesky-correlated asset drivers, European and Longstaff-Schwartz basket
    prices, pathwise deltas and pathwise-likelihood-ratio (cross-)gammas.
  * :mod:`oracle.basket_gbm` -- the two-asset GBM basket: a semi-closed-form European price
    and the Boyle-Evnine-Gibbs two-asset lattice for Bermudan basket options.

The paper (Klaisoongnoen et al., FPGA'24) names the dataflow stages it runs --
VariancePathQE, LogPricePathQE, AssetPathExponential,
longstaffSchwartzPathReduction, writeLongstaffSchwartzPath (Sec. 5, opening
paragraph) -- and the loop nest over assets, time steps and paths (Sec. 2.1,
Listing 2), but it does not print their equations; those come from the
published methods the stage names refer to (see ``simr_oracle.h``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsimr_oracle.so")
_SRC = os.path.join(_HERE, "simr_oracle.c")

EURO_CALL, EURO_PUT, AMER_PUT, AMER_CALL = 0, 1, 2, 3
SCHEME_QE, SCHEME_FTE, SCHEME_QE_M, SCHEME_TG, SCHEME_BK = 0, 1, 2, 3, 4
GREEK_NAMES_EXT = ("S0", "v0", "theta", "r", "kappa", "xi", "rho", "T", "gamma")
GREEK_NAMES = ("S0", "v0", "theta", "r", "kappa", "xi", "rho")


def build(force: bool = False) -> str:
    """Compiles the oracle with gcc (-O2, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
               "-D_POSIX_C_SOURCE=200809L", "-Wall", "-shared", "-fPIC", _SRC,
               "-o", _LIB_PATH + ".tmp", "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _RefOption(ctypes.Structure):
    _fields_ = [("S0", ctypes.c_double), ("K", ctypes.c_double), ("T", ctypes.c_double),
                ("r", ctypes.c_double), ("kappa", ctypes.c_double), ("theta", ctypes.c_double),
                ("xi", ctypes.c_double), ("rho", ctypes.c_double), ("v0", ctypes.c_double),
                ("payoff", ctypes.c_int32), ("steps", ctypes.c_int32), ("paths", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("stream", ctypes.c_uint32), ("scheme", ctypes.c_int32)]


_lib = None


def _L():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i32p = ctypes.POINTER(ctypes.c_int32)
        optp = ctypes.POINTER(_RefOption)
        _lib.ref_philox4x32_10.argtypes = [u32p, u32p, u32p]
        _lib.ref_uniform.argtypes = [ctypes.c_uint32]
        _lib.ref_uniform.restype = ctypes.c_double
        _lib.ref_box_muller.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp]
        _lib.ref_qe_variance_step.argtypes = [ctypes.c_double] * 7
        _lib.ref_qe_log_mgf.argtypes = [ctypes.c_double] * 6 + [ctypes.POINTER(ctypes.c_int)]
        _lib.ref_qe_log_mgf.restype = ctypes.c_double
        _lib.ref_qe_m_logprice_step.argtypes = [ctypes.c_double] * 10
        _lib.ref_tg_r.argtypes = [ctypes.c_double]
        _lib.ref_tg_r.restype = ctypes.c_double
        _lib.ref_tg_variance_step.argtypes = [ctypes.c_double] * 6
        _lib.ref_tg_variance_step.restype = ctypes.c_double
        _lib.ref_qe_m_logprice_step.restype = ctypes.c_double
        _lib.ref_qe_variance_step.restype = ctypes.c_double
        _lib.ref_qe_logprice_step.argtypes = [ctypes.c_double] * 10
        _lib.ref_qe_logprice_step.restype = ctypes.c_double
        _lib.ref_fte_step.argtypes = [dp, dp] + [ctypes.c_double] * 8
        _lib.ref_rng_words.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int32, ctypes.c_int32, u32p]
        _lib.ref_simulate.argtypes = [optp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, dp, dp, dp]
        _lib.ref_price_european.argtypes = [optp, ctypes.c_int, dp, dp, dp]
        _lib.ref_chol6_solve.argtypes = [dp, dp, dp]
        _lib.ref_chol6_solve.restype = ctypes.c_int
        _lib.ref_price_american.argtypes = [optp, ctypes.c_int, dp, dp, i32p, i32p, i32p]
        _lib.ref_price_american_beta.argtypes = [optp, ctypes.c_int, dp, dp, i32p, i32p, i32p, dp]
        _lib.ref_greeks.argtypes = [optp, ctypes.c_int, dp, dp, dp, dp]
        _lib.ref_greeks_at_tau.argtypes = [optp, i32p, ctypes.c_int, dp, dp, dp, dp]
        _lib.ref_greeks_ext.argtypes = [optp, ctypes.c_int, dp, dp, dp, dp]
        _lib.ref_greeks_at_tau_ext.argtypes = [optp, i32p, ctypes.c_int, dp, dp, dp, dp]
        _lib.ref_stopped_values.argtypes = [optp, i32p, ctypes.c_int, dp]
        _lib.ref_path_states.argtypes = [optp, ctypes.c_int, dp, dp]
        _lib.ref_bk_variance.argtypes = [ctypes.c_double] * 6
        _lib.ref_bk_variance.restype = ctypes.c_double
        for name in ("ref_bk_integrated_variance", "ref_bk_log_cf_re", "ref_bk_log_cf_im"):
            getattr(_lib, name).argtypes = [ctypes.c_double] * 7
            getattr(_lib, name).restype = ctypes.c_double
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 64))


@dataclass
class Option:
    """One option under the Heston model, plus the Monte Carlo set-up."""
    S0: float = 100.0
    K: float = 100.0
    T: float = 1.0
    r: float = 0.02
    kappa: float = 1.5
    theta: float = 0.04
    xi: float = 0.3
    rho: float = -0.7
    v0: float = 0.04
    payoff: int = EURO_CALL
    steps: int = 64
    paths: int = 8192
    seed: int = 1
    stream: int = 0
    scheme: int = SCHEME_QE

    def _c(self) -> _RefOption:
        return _RefOption(self.S0, self.K, self.T, self.r, self.kappa, self.theta, self.xi, self.rho,
                          self.v0, self.payoff, self.steps, self.paths, self.seed, self.stream, self.scheme)

    def replace(self, **kw) -> "Option":
        d = dict(self.__dict__)
        d.update(kw)
        return Option(**d)


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _L().ref_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(out, ctypes.c_uint32))
    return out


def uniform(w: int) -> float:
    return _L().ref_uniform(int(w) & 0xFFFFFFFF)


def box_muller(u0: float, u1: float):
    z1, z2 = ctypes.c_double(), ctypes.c_double()
    _L().ref_box_muller(u0, u1, ctypes.byref(z1), ctypes.byref(z2))
    return z1.value, z2.value


def qe_variance_step(v, kappa, theta, xi, dt, z1, u) -> float:
    return _L().ref_qe_variance_step(v, kappa, theta, xi, dt, z1, u)


def qe_logprice_step(x, v, vnext, r, kappa, theta, xi, rho, dt, z2) -> float:
    return _L().ref_qe_logprice_step(x, v, vnext, r, kappa, theta, xi, rho, dt, z2)



def tg_r(psi: float) -> float:
    """r(psi) of the truncated Gaussian scheme."""
    return _L().ref_tg_r(psi)


def tg_variance_step(v, kappa, theta, xi, dt, z1) -> float:
    """One truncated Gaussian variance transition from v."""
    return _L().ref_tg_variance_step(v, kappa, theta, xi, dt, z1)


def qe_log_mgf(v, kappa, theta, xi, dt, A):
    """(ln E[exp(A V_{n+1}) | v], defined) for the QE variance transition from v."""
    ok = ctypes.c_int()
    val = _L().ref_qe_log_mgf(v, kappa, theta, xi, dt, A, ctypes.byref(ok))
    return val, bool(ok.value)


def qe_m_logprice_step(x, v, vnext, r, kappa, theta, xi, rho, dt, z2) -> float:
    """Martingale-corrected QE log-price transition: returns x_{n+1}."""
    return _L().ref_qe_m_logprice_step(x, v, vnext, r, kappa, theta, xi, rho, dt, z2)

def fte_step(x, v, r, kappa, theta, xi, rho, dt, z1, z2):
    xc, vc = ctypes.c_double(x), ctypes.c_double(v)
    _L().ref_fte_step(ctypes.byref(xc), ctypes.byref(vc), r, kappa, theta, xi, rho, dt, z1, z2)
    return xc.value, vc.value


def rng_words(seed: int, stream: int, path0: int, npaths: int, step0: int, nsteps: int) -> np.ndarray:
    """Philox words, shape (npaths, nsteps, 4), for counter (step, path, stream, 0)."""
    out = np.zeros((npaths, nsteps, 4), dtype=np.uint32)
    _L().ref_rng_words(seed, stream, path0, npaths, step0, nsteps, _ptr(out, ctypes.c_uint32))
    return out


def simulate(opt: Option, path0: int = 0, npaths: int | None = None, nthreads: int | None = None):
    """Terminal (x_T, v_T, discounted European payoff) of paths [path0, path0+npaths)."""
    n = opt.paths - path0 if npaths is None else npaths
    xT = np.zeros(n)
    vT = np.zeros(n)
    pay = np.zeros(n)
    o = opt._c()
    rc = _L().ref_simulate(ctypes.byref(o), path0, n, nthreads or default_threads(),
                           _ptr(xT, ctypes.c_double), _ptr(vT, ctypes.c_double), _ptr(pay, ctypes.c_double))
    if rc:
        raise RuntimeError("ref_simulate failed")
    return xT, vT, pay


def price_european(opt: Option, nthreads: int | None = None):
    """(price, std_err, [sum X, sum X^2])."""
    price, se = ctypes.c_double(), ctypes.c_double()
    sums = np.zeros(2)
    o = opt._c()
    rc = _L().ref_price_european(ctypes.byref(o), nthreads or default_threads(), ctypes.byref(price),
                                 ctypes.byref(se), _ptr(sums, ctypes.c_double))
    if rc:
        raise RuntimeError("ref_price_european failed")
    return price.value, se.value, sums


def path_states(opt: Option, nthreads: int | None = None):
    """(X, V), each shaped (steps, paths): x = ln(S/S0) and v at t_1..t_N."""
    X = np.zeros((opt.steps, opt.paths))
    V = np.zeros((opt.steps, opt.paths))
    o = opt._c()
    if _L().ref_path_states(ctypes.byref(o), nthreads or default_threads(), _ptr(X, ctypes.c_double),
                            _ptr(V, ctypes.c_double)):
        raise RuntimeError("ref_path_states failed")
    return X, V


def chol6_solve(G, b):
    """(beta, rank) of the pivoted-Cholesky least-squares solve of G beta = b."""
    Gc = np.ascontiguousarray(G, dtype=np.float64).reshape(36)
    bc = np.ascontiguousarray(b, dtype=np.float64).reshape(6)
    beta = np.zeros(6)
    rank = _L().ref_chol6_solve(_ptr(Gc, ctypes.c_double), _ptr(bc, ctypes.c_double), _ptr(beta, ctypes.c_double))
    return beta, rank


@dataclass
class AmericanResult:
    price: float
    std_err: float
    tau: np.ndarray = field(repr=False)
    exercised_at_t0: bool
    lsm_flags: int
    beta: np.ndarray = field(default=None, repr=False)  # (steps + 1, 6) regression coefficients


def price_american(opt: Option, nthreads: int | None = None) -> AmericanResult:
    price, se = ctypes.c_double(), ctypes.c_double()
    tau = np.zeros(opt.paths, dtype=np.int32)
    beta = np.zeros((opt.steps + 1, 6))
    ex0, flags = ctypes.c_int32(), ctypes.c_int32()
    o = opt._c()
    rc = _L().ref_price_american_beta(ctypes.byref(o), nthreads or default_threads(), ctypes.byref(price),
                                      ctypes.byref(se), _ptr(tau, ctypes.c_int32), ctypes.byref(ex0),
                                      ctypes.byref(flags), _ptr(beta, ctypes.c_double))
    if rc:
        raise RuntimeError("ref_price_american failed")
    return AmericanResult(price.value, se.value, tau, bool(ex0.value), flags.value, beta)


def greeks(opt: Option, nthreads: int | None = None):
    """(price, std_err, grads[7], grad_se[7]) -- forward-mode pathwise Greeks with
    respect to (S0, v0, theta, r, kappa, xi, rho)."""
    price, se = ctypes.c_double(), ctypes.c_double()
    g = np.zeros(7)
    gse = np.zeros(7)
    o = opt._c()
    rc = _L().ref_greeks(ctypes.byref(o), nthreads or default_threads(), ctypes.byref(price),
                         ctypes.byref(se), _ptr(g, ctypes.c_double), _ptr(gse, ctypes.c_double))
    if rc:
        raise RuntimeError("ref_greeks failed")
    return price.value, se.value, g, gse


def greeks_ext(opt: Option, nthreads: int | None = None):
    """(price, std_err, grads[9], grad_se[9]): the 7 Greeks of `greeks`, then d price / d T
    (steps fixed) and gamma d2 price / d S0^2 (pathwise likelihood-ratio estimator)."""
    price, se = ctypes.c_double(), ctypes.c_double()
    g = np.zeros(9)
    gse = np.zeros(9)
    rc = _L().ref_greeks_ext(ctypes.byref(opt._c()), nthreads or default_threads(), ctypes.byref(price),
                             ctypes.byref(se), _ptr(g, ctypes.c_double), _ptr(gse, ctypes.c_double))
    if rc:
        raise RuntimeError("ref_greeks_ext failed")
    return price.value, se.value, g, gse


def greeks_at_tau_ext(opt: Option, tau, nthreads: int | None = None):
    """`greeks_at_tau` with d/dT and gamma appended (9 values)."""
    t = np.ascontiguousarray(tau, dtype=np.int32)
    if t.shape != (opt.paths,):
        raise ValueError("tau must hold one index per path")
    value, se = ctypes.c_double(), ctypes.c_double()
    g = np.zeros(9)
    gse = np.zeros(9)
    rc = _L().ref_greeks_at_tau_ext(ctypes.byref(opt._c()), _ptr(t, ctypes.c_int32), nthreads or default_threads(),
                                    ctypes.byref(value), ctypes.byref(se), _ptr(g, ctypes.c_double),
                                    _ptr(gse, ctypes.c_double))
    if rc:
        raise RuntimeError("ref_greeks_at_tau_ext failed")
    return value.value, se.value, g, gse


def greeks_at_tau(opt: Option, tau, nthreads: int | None = None):
    """(value, std_err, grads[7], grad_se[7]) of the exercise policy that stops path p
    at tau[p]: the mean discounted stopped cash flow and its forward-mode pathwise
    Greeks with the indices held fixed."""
    t = np.ascontiguousarray(tau, dtype=np.int32)
    if t.shape != (opt.paths,):
        raise ValueError("tau must hold one index per path")
    value, se = ctypes.c_double(), ctypes.c_double()
    g = np.zeros(7)
    gse = np.zeros(7)
    o = opt._c()
    rc = _L().ref_greeks_at_tau(ctypes.byref(o), _ptr(t, ctypes.c_int32), nthreads or default_threads(),
                                ctypes.byref(value), ctypes.byref(se), _ptr(g, ctypes.c_double),
                                _ptr(gse, ctypes.c_double))
    if rc:
        raise RuntimeError("ref_greeks_at_tau failed")
    return value.value, se.value, g, gse


def stopped_values(opt: Option, tau, nthreads: int | None = None) -> np.ndarray:
    """Per-path e^{-r tau dt} h(S_tau) with the exercise indices `tau` held fixed."""
    t = np.ascontiguousarray(tau, dtype=np.int32)
    out = np.zeros(opt.paths)
    o = opt._c()
    if _L().ref_stopped_values(ctypes.byref(o), _ptr(t, ctypes.c_int32), nthreads or default_threads(),
                               _ptr(out, ctypes.c_double)):
        raise RuntimeError("ref_stopped_values failed")
    return out


def fixed_tau_fd_greeks(opt: Option, tau, rel_bump: float = 1e-4, nthreads: int | None = None):
    """Central FD with common random numbers of the mean stopped cash flow, the
    exercise indices held fixed: (grads[7], grad_se[7])."""
    g = np.zeros(7)
    gse = np.zeros(7)
    for i, name in enumerate(GREEK_NAMES):
        p0 = getattr(opt, name)
        h = rel_bump * abs(p0) if p0 != 0 else rel_bump
        d = (stopped_values(opt.replace(**{name: p0 + h}), tau, nthreads)
             - stopped_values(opt.replace(**{name: p0 - h}), tau, nthreads)) / (2 * h)
        g[i] = d.mean()
        gse[i] = d.std(ddof=1) / np.sqrt(d.size)
    return g, gse


def price(opt: Option, nthreads: int | None = None):
    """(price, std_err) for any payoff kind."""
    if opt.payoff in (AMER_PUT, AMER_CALL):
        r = price_american(opt, nthreads)
        return r.price, r.std_err
    p, se, _ = price_european(opt, nthreads)
    return p, se


def fd_greeks(opt: Option, rel_bump: float = 1e-4, nthreads: int | None = None):
    """Central finite differences of the oracle price with common random numbers.
    Bump h = rel_bump * |p| (rel_bump if p == 0).  Returns (grads[7], grad_se[7]);
    the standard error is that of the per-path difference for European options
    and None-like NaN for American ones (their regressions differ per bump)."""
    g = np.zeros(7)
    gse = np.full(7, np.nan)
    for i, name in enumerate(GREEK_NAMES):
        p0 = getattr(opt, name)
        h = rel_bump * abs(p0) if p0 != 0 else rel_bump
        up = opt.replace(**{name: p0 + h})
        dn = opt.replace(**{name: p0 - h})
        if opt.payoff in (AMER_PUT, AMER_CALL):
            g[i] = (price_american(up, nthreads).price - price_american(dn, nthreads).price) / (2 * h)
        else:
            _, _, pu = simulate(up, nthreads=nthreads)
            _, _, pd = simulate(dn, nthreads=nthreads)
            d = (pu - pd) / (2 * h)
            g[i] = d.mean()
            gse[i] = d.std(ddof=1) / np.sqrt(d.size)
    return g, gse


# ---------------------------------------------------------------------------------------------
# Correlated baskets
# ---------------------------------------------------------------------------------------------

MAX_ASSETS = 32
BASKET_NB = 10


class _RefBasket(ctypes.Structure):
    _fields_ = [("assets", ctypes.c_int32), ("payoff", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("scheme", ctypes.c_int32), ("paths", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("stream", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("K", ctypes.c_double), ("T", ctypes.c_double), ("r", ctypes.c_double)] + \
               [(n, ctypes.c_double * MAX_ASSETS) for n in ("w", "S0", "kappa", "theta", "xi", "rho", "v0")] + \
               [("corr", ctypes.c_double * (MAX_ASSETS * MAX_ASSETS))]


@dataclass
class Basket:
    """d Heston assets with correlated asset drivers; the payoff is on B = sum w_i S_i.
    Per-asset fields are sequences of length d; corr is the d x d matrix C."""
    S0: tuple = (100.0, 100.0)
    w: tuple = (0.5, 0.5)
    kappa: tuple = (1.5, 1.5)
    theta: tuple = (0.04, 0.04)
    xi: tuple = (0.3, 0.3)
    rho: tuple = (-0.7, -0.7)
    v0: tuple = (0.04, 0.04)
    corr: tuple = ((1.0, 0.5), (0.5, 1.0))
    K: float = 100.0
    T: float = 1.0
    r: float = 0.02
    payoff: int = EURO_CALL
    steps: int = 64
    paths: int = 8192
    seed: int = 1
    stream: int = 0
    scheme: int = SCHEME_QE

    @property
    def assets(self) -> int:
        return len(self.S0)

    def _c(self) -> _RefBasket:
        d = self.assets
        c = _RefBasket()
        c.assets, c.payoff, c.steps, c.scheme = d, self.payoff, self.steps, self.scheme
        c.paths, c.seed, c.stream = self.paths, self.seed, self.stream
        c.K, c.T, c.r = self.K, self.T, self.r
        for name in ("w", "S0", "kappa", "theta", "xi", "rho", "v0"):
            vals = getattr(self, name)
            if len(vals) != d:
                raise ValueError(f"{name} needs {d} values")
            arr = getattr(c, name)
            for i, x in enumerate(vals):
                arr[i] = float(x)
        C = np.asarray(self.corr, dtype=np.float64)
        if C.shape != (d, d):
            raise ValueError("corr must be d x d")
        for i in range(d):
            for j in range(d):
                c.corr[i * MAX_ASSETS + j] = C[i, j]
        return c

    def replace(self, **kw) -> "Basket":
        from dataclasses import replace as _r
        return _r(self, **kw)


def _LB():
    lib = _L()
    if not hasattr(lib, "_basket_ready"):
        dp = ctypes.POINTER(ctypes.c_double)
        i32p = ctypes.POINTER(ctypes.c_int32)
        bp = ctypes.POINTER(_RefBasket)
        lib.ref_corr_cholesky.argtypes = [ctypes.c_int, dp, dp]
        lib.ref_basket_simulate.argtypes = [bp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, dp, dp, dp]
        lib.ref_basket_price_european.argtypes = [bp, ctypes.c_int, dp, dp]
        lib.ref_basket_states.argtypes = [bp, ctypes.c_int, dp, dp]
        lib.ref_chol_solve.argtypes = [ctypes.c_int, dp, dp, dp]
        lib.ref_chol_solve.restype = ctypes.c_int
        lib.ref_basket_price_american.argtypes = [bp, ctypes.c_int, dp, dp, i32p, i32p, i32p, dp]
        lib.ref_basket_stopped_values.argtypes = [bp, i32p, ctypes.c_int, dp]
        lib.ref_basket_greeks.argtypes = [bp, i32p, ctypes.c_int, dp, dp, dp, dp, dp, dp]
        lib.ref_basket_risk_greeks.argtypes = [bp, i32p, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, dp]
        lib.ref_corr_cholesky_tan.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_int, dp, dp]
        lib._basket_ready = True
    return lib


def corr_cholesky(C):
    """Lower Cholesky factor of C, or None if C is not positive definite."""
    C = np.asarray(C, dtype=np.float64)
    d = C.shape[0]
    full = np.zeros((MAX_ASSETS, MAX_ASSETS))
    full[:d, :d] = C
    L = np.zeros((MAX_ASSETS, MAX_ASSETS))
    if _LB().ref_corr_cholesky(d, _ptr(full, ctypes.c_double), _ptr(L, ctypes.c_double)):
        return None
    return L[:d, :d].copy()


def basket_simulate(b: Basket, path0: int = 0, npaths: int | None = None, nthreads: int | None = None):
    """(xT[P, d], vT[P, d], discounted payoff[P]) of paths [path0, path0 + npaths)."""
    n = b.paths - path0 if npaths is None else npaths
    d = b.assets
    xT = np.zeros((n, d))
    vT = np.zeros((n, d))
    pay = np.zeros(n)
    if _LB().ref_basket_simulate(ctypes.byref(b._c()), path0, n, nthreads or default_threads(),
                                 _ptr(xT, ctypes.c_double), _ptr(vT, ctypes.c_double), _ptr(pay, ctypes.c_double)):
        raise RuntimeError("ref_basket_simulate failed (is corr positive definite?)")
    return xT, vT, pay


def basket_price_european(b: Basket, nthreads: int | None = None):
    p, se = ctypes.c_double(), ctypes.c_double()
    if _LB().ref_basket_price_european(ctypes.byref(b._c()), nthreads or default_threads(), ctypes.byref(p),
                                       ctypes.byref(se)):
        raise RuntimeError("ref_basket_price_european failed")
    return p.value, se.value


def basket_states(b: Basket, nthreads: int | None = None):
    """(X, V), each [N, P]: ln(B_n / B_0) and the value-weighted variance at dates 1..N."""
    X = np.zeros((b.steps, b.paths))
    V = np.zeros((b.steps, b.paths))
    if _LB().ref_basket_states(ctypes.byref(b._c()), nthreads or default_threads(), _ptr(X, ctypes.c_double),
                               _ptr(V, ctypes.c_double)):
        raise RuntimeError("ref_basket_states failed")
    return X, V


def chol_solve(G, bv):
    """(beta, rank) of the pivoted-Cholesky least-squares solve of G beta = b."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    bv = np.ascontiguousarray(bv, dtype=np.float64)
    beta = np.zeros(len(bv))
    rank = _LB().ref_chol_solve(len(bv), _ptr(G, ctypes.c_double), _ptr(bv, ctypes.c_double),
                                _ptr(beta, ctypes.c_double))
    return beta, rank


def basket_price_american(b: Basket, nthreads: int | None = None) -> "AmericanResult":
    p, se = ctypes.c_double(), ctypes.c_double()
    tau = np.zeros(b.paths, dtype=np.int32)
    ex0, flags = ctypes.c_int32(), ctypes.c_int32()
    beta = np.zeros((b.steps + 1) * BASKET_NB)
    if _LB().ref_basket_price_american(ctypes.byref(b._c()), nthreads or default_threads(), ctypes.byref(p),
                                       ctypes.byref(se), _ptr(tau, ctypes.c_int32), ctypes.byref(ex0),
                                       ctypes.byref(flags), _ptr(beta, ctypes.c_double)):
        raise RuntimeError("ref_basket_price_american failed")
    return AmericanResult(p.value, se.value, tau, bool(ex0.value), flags.value,
                          beta.reshape(b.steps + 1, BASKET_NB))


def basket_stopped_values(b: Basket, tau, nthreads: int | None = None) -> np.ndarray:
    t = np.ascontiguousarray(tau, dtype=np.int32)
    out = np.zeros(b.paths)
    if _LB().ref_basket_stopped_values(ctypes.byref(b._c()), _ptr(t, ctypes.c_int32), nthreads or default_threads(),
                                       _ptr(out, ctypes.c_double)):
        raise RuntimeError("ref_basket_stopped_values failed")
    return out


def basket_greeks(b: Basket, tau=None, nthreads: int | None = None):
    """(price, std_err, delta[d], delta_se[d], gamma[d, d], gamma_se[d, d]); see
    ref_basket_greeks."""
    d = b.assets
    p, se = ctypes.c_double(), ctypes.c_double()
    dl, dls = np.zeros(d), np.zeros(d)
    g, gs = np.zeros((d, d)), np.zeros((d, d))
    tp = None
    if tau is not None:
        t = np.ascontiguousarray(tau, dtype=np.int32)
        if t.shape != (b.paths,):
            raise ValueError("tau must hold one index per path")
        tp = _ptr(t, ctypes.c_int32)
    if _LB().ref_basket_greeks(ctypes.byref(b._c()), tp, nthreads or default_threads(), ctypes.byref(p),
                               ctypes.byref(se), _ptr(dl, ctypes.c_double), _ptr(dls, ctypes.c_double),
                               _ptr(g, ctypes.c_double), _ptr(gs, ctypes.c_double)):
        raise RuntimeError("ref_basket_greeks failed")
    return p.value, se.value, dl, dls, g, gs


def corr_cholesky_tan(C, i: int, j: int):
    """(L, dL): the Cholesky factor of C and its derivative when C_ij and C_ji move together."""
    C = np.asarray(C, dtype=np.float64)
    d = C.shape[0]
    full = np.zeros((MAX_ASSETS, MAX_ASSETS))
    full[:d, :d] = C
    L = np.zeros((MAX_ASSETS, MAX_ASSETS))
    dL = np.zeros((MAX_ASSETS, MAX_ASSETS))
    if _LB().ref_corr_cholesky_tan(d, _ptr(full, ctypes.c_double), i, j, _ptr(L, ctypes.c_double),
                                   _ptr(dL, ctypes.c_double)):
        raise ValueError("not positive definite, or not an off-diagonal pair")
    return L[:d, :d].copy(), dL[:d, :d].copy()


def basket_risk_greeks(b: Basket, tau=None, nthreads: int | None = None):
    """(price, std_err, vega_v0[d], se[d], vega_theta[d], se[d], dcorr[d, d], se[d, d]); see
    ref_basket_risk_greeks (dcorr symmetric, 0 on the diagonal)."""
    d = b.assets
    p, se = ctypes.c_double(), ctypes.c_double()
    vv, vvs, vt, vts = np.zeros(d), np.zeros(d), np.zeros(d), np.zeros(d)
    dc, dcs = np.zeros((d, d)), np.zeros((d, d))
    tp = None
    if tau is not None:
        t = np.ascontiguousarray(tau, dtype=np.int32)
        if t.shape != (b.paths,):
            raise ValueError("tau must hold one index per path")
        tp = _ptr(t, ctypes.c_int32)
    if _LB().ref_basket_risk_greeks(ctypes.byref(b._c()), tp, nthreads or default_threads(), ctypes.byref(p),
                                    ctypes.byref(se), _ptr(vv, ctypes.c_double), _ptr(vvs, ctypes.c_double),
                                    _ptr(vt, ctypes.c_double), _ptr(vts, ctypes.c_double),
                                    _ptr(dc, ctypes.c_double), _ptr(dcs, ctypes.c_double)):
        raise RuntimeError("ref_basket_risk_greeks failed")
    return p.value, se.value, vv, vvs, vt, vts, dc, dcs


def bk_variance(v, kappa, theta, xi, dt, u) -> float:
    """Broadie-Kaya: the exact CIR transition from v over dt at the uniform u (inverse CDF)."""
    return _L().ref_bk_variance(v, kappa, theta, xi, dt, u)


def bk_integrated_variance(vu, vt, kappa, theta, xi, dt, u) -> float:
    """Broadie-Kaya: the integrated variance over the step given both endpoints, at the uniform u."""
    return _L().ref_bk_integrated_variance(vu, vt, kappa, theta, xi, dt, u)


def bk_log_cf(a, vu, vt, kappa, theta, xi, dt) -> complex:
    """ln E[exp(i a I) | v_u, v_t] for I the integral of V over one step."""
    L = _L()
    return complex(L.ref_bk_log_cf_re(a, vu, vt, kappa, theta, xi, dt), L.ref_bk_log_cf_im(a, vu, vt, kappa, theta, xi, dt))
