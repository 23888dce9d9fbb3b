"""ctypes binding of ``libsimr.so`` (the C ABI in ``include/simr.h``).

Argument marshalling only: every step of the Monte Carlo path runs in the HIP
kernels behind the C ABI.  PyTorch supplies device memory (the workspace and
debug outputs are ``torch.uint8`` / float tensors on the GPU) and the stream
(``torch.cuda.current_stream()``).  There is no CPU fallback: without the
built library or a gfx950 GPU every call raises.
"""
from __future__ import annotations

import atexit
import ctypes
import os
from dataclasses import dataclass, field, fields

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsimr.so")

EURO_CALL, EURO_PUT, AMER_PUT, AMER_CALL = 0, 1, 2, 3
SCHEME_QE, SCHEME_FTE, SCHEME_QE_M, SCHEME_TG, SCHEME_BK = 0, 1, 2, 3, 4
LSM_FEW_ITM, LSM_DROPPED, LSM_EXERCISE_T0 = 1, 2, 4
GREEK_NAMES_EXT = ("S0", "v0", "theta", "r", "kappa", "xi", "rho", "T", "gamma")
GREEK_NAMES = ("S0", "v0", "theta", "r", "kappa", "xi", "rho")

STATUS = {0: "ok", -1: "invalid argument", -2: "out of host memory", -3: "HIP runtime error",
          -4: "unsupported", -5: "numerical failure"}


class SimrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Option(ctypes.Structure):
    _fields_ = [("S0", ctypes.c_double), ("K", ctypes.c_double), ("T", ctypes.c_double), ("r", ctypes.c_double),
                ("kappa", ctypes.c_double), ("theta", ctypes.c_double), ("xi", ctypes.c_double),
                ("rho", ctypes.c_double), ("v0", ctypes.c_double), ("payoff", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("paths", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("stream_id", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class _Params(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int32), ("checkpoint_every", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("price", ctypes.c_double), ("std_err", ctypes.c_double), ("paths", ctypes.c_int64),
                ("lsm_flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _GreeksResult(ctypes.Structure):
    _fields_ = [("price", ctypes.c_double), ("std_err", ctypes.c_double), ("g", ctypes.c_double * 7),
                ("g_se", ctypes.c_double * 7), ("lsm_flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _GreeksExtResult(ctypes.Structure):
    _fields_ = [("price", ctypes.c_double), ("std_err", ctypes.c_double), ("g", ctypes.c_double * 9),
                ("g_se", ctypes.c_double * 9), ("lsm_flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


MAX_ASSETS = 32
BASKET_NB = 10


class _Basket(ctypes.Structure):
    _fields_ = [("assets", ctypes.c_int32), ("payoff", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("paths", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("stream_id", ctypes.c_uint32), ("reserved1", ctypes.c_uint32),
                ("K", ctypes.c_double), ("T", ctypes.c_double), ("r", ctypes.c_double)] + \
               [(n, ctypes.c_double * MAX_ASSETS) for n in ("w", "S0", "kappa", "theta", "xi", "rho", "v0")] + \
               [("corr", ctypes.c_double * (MAX_ASSETS * MAX_ASSETS))]


class _BasketGreeksResult(ctypes.Structure):
    _fields_ = [("price", ctypes.c_double), ("std_err", ctypes.c_double),
                ("delta", ctypes.c_double * MAX_ASSETS), ("delta_se", ctypes.c_double * MAX_ASSETS),
                ("gamma", ctypes.c_double * (MAX_ASSETS * MAX_ASSETS)),
                ("gamma_se", ctypes.c_double * (MAX_ASSETS * MAX_ASSETS)),
                ("lsm_flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


@dataclass
class Option:
    """One option (an "asset" of the paper's Table 1) with its Monte Carlo set-up."""
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

    @classmethod
    def from_dict(cls, d: dict) -> "Option":
        names = {f.name for f in fields(cls)}
        return cls(**{k: v for k, v in d.items() if k in names})

    def _c(self) -> _Option:
        return _Option(self.S0, self.K, self.T, self.r, self.kappa, self.theta, self.xi, self.rho, self.v0,
                       self.payoff, self.steps, self.paths, self.seed, self.stream, 0)


@dataclass
class Basket:
    """A basket of d correlated Heston assets; the payoff is on B = sum w_i S_i.  Per-asset
    fields are sequences of d values, corr the d x d correlation of the asset drivers."""
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

    @property
    def assets(self) -> int:
        return len(self.S0)

    @classmethod
    def from_dict(cls, d: dict) -> "Basket":
        names = {f.name for f in fields(cls)}
        return cls(**{k: v for k, v in d.items() if k in names})

    def _c(self) -> _Basket:
        n = self.assets
        c = _Basket()
        c.assets, c.payoff, c.steps, c.paths = n, self.payoff, self.steps, self.paths
        c.seed, c.stream_id, c.K, c.T, c.r = self.seed, self.stream, self.K, self.T, self.r
        for name in ("w", "S0", "kappa", "theta", "xi", "rho", "v0"):
            vals = getattr(self, name)
            if len(vals) != n:
                raise ValueError(f"{name} needs {n} values")
            arr = getattr(c, name)
            for i, x in enumerate(vals):
                arr[i] = float(x)
        for i, row in enumerate(self.corr):
            if len(row) != n:
                raise ValueError("corr must be d x d")
            for j, x in enumerate(row):
                c.corr[i * MAX_ASSETS + j] = float(x)
        return c


class _BasketRiskResult(ctypes.Structure):
    _fields_ = [("price", ctypes.c_double), ("std_err", ctypes.c_double)] + \
               [(n, ctypes.c_double * MAX_ASSETS) for n in ("vega_v0", "vega_v0_se", "vega_theta", "vega_theta_se")] + \
               [("dcorr", ctypes.c_double * (MAX_ASSETS * MAX_ASSETS)),
                ("dcorr_se", ctypes.c_double * (MAX_ASSETS * MAX_ASSETS)),
                ("lsm_flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


@dataclass
class BasketRisk:
    price: float
    std_err: float
    vega_v0: list
    vega_v0_se: list
    vega_theta: list
    vega_theta_se: list
    dcorr: list      # d x d, symmetric, 0 on the diagonal
    dcorr_se: list
    lsm_flags: int = 0


@dataclass
class BasketGreeks:
    price: float
    std_err: float
    delta: list
    delta_se: list
    gamma: list   # d x d (NaN for American baskets)
    gamma_se: list
    lsm_flags: int = 0


@dataclass
class Result:
    price: float
    std_err: float
    paths: int
    lsm_flags: int = 0


@dataclass
class GreeksResult:
    price: float
    std_err: float
    grads: list = field(default_factory=list)
    grad_se: list = field(default_factory=list)
    lsm_flags: int = 0

    def as_dict(self):
        return dict(zip(GREEK_NAMES, self.grads))


_lib = None
_ctx = {}
_ws = {}


def library() -> ctypes.CDLL:
    """Loads libsimr.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_2402_12111_amd.build)")
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the SIMR library runs on an MI355X (gfx950) only")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        optp, prmp = ctypes.POINTER(_Option), ctypes.POINTER(_Params)
        L.simr_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
        L.simr_destroy.argtypes = [vp]
        L.simr_workspace_size.argtypes = [vp, ctypes.c_int, optp, ctypes.c_int64, prmp, ctypes.POINTER(sz)]
        L.simr_price.argtypes = [vp, optp, prmp, ctypes.POINTER(_Result), vp, sz, vp]
        L.simr_price_batch.argtypes = [vp, optp, ctypes.c_int64, prmp, ctypes.POINTER(_Result), vp, sz, vp]
        L.simr_greeks.argtypes = [vp, optp, prmp, ctypes.POINTER(_GreeksResult), vp, sz, vp]
        L.simr_greeks_batch.argtypes = [vp, optp, ctypes.c_int64, prmp, ctypes.POINTER(_GreeksResult), vp, sz, vp]
        L.simr_price_noalloc.argtypes = [vp, optp, prmp, ctypes.POINTER(_Result), vp]
        L.simr_debug_draws.argtypes = [vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp]
        L.simr_debug_paths.argtypes = [vp, optp, prmp, vp, vp, vp, vp]
        L.simr_debug_lsm.argtypes = [vp, optp, prmp, ctypes.POINTER(_Result), vp, vp, vp, sz, vp]
        L.simr_set_lsm_launch.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
        bkp = ctypes.POINTER(_Basket)
        L.simr_basket_workspace_size.argtypes = [vp, ctypes.c_int, bkp, prmp, ctypes.POINTER(sz)]
        L.simr_basket_price.argtypes = [vp, bkp, prmp, ctypes.POINTER(_Result), vp, sz, vp]
        L.simr_basket_greeks.argtypes = [vp, bkp, prmp, ctypes.POINTER(_BasketGreeksResult), vp, sz, vp]
        L.simr_basket_risk.argtypes = [vp, bkp, prmp, ctypes.POINTER(_BasketRiskResult), vp, sz, vp]
        L.simr_debug_basket_paths.argtypes = [vp, bkp, prmp, vp, vp, vp, vp, sz, vp]
        L.simr_debug_basket_lsm.argtypes = [vp, bkp, prmp, ctypes.POINTER(_Result), vp, vp, vp, sz, vp]
        L.simr_greeks_ext.argtypes = [vp, optp, prmp, ctypes.POINTER(_GreeksExtResult), vp, sz, vp]
        L.simr_get_tile.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.simr_debug_graph_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.simr_debug_fault.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
        L.simr_set_tile.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
        L.simr_status_string.argtypes = [ctypes.c_int]
        L.simr_status_string.restype = ctypes.c_char_p
        L.simr_last_error.restype = ctypes.c_char_p
        for name in ("simr_create", "simr_destroy", "simr_workspace_size", "simr_price", "simr_price_batch",
                     "simr_greeks", "simr_greeks_batch", "simr_debug_draws", "simr_debug_paths", "simr_debug_lsm", "simr_get_tile",
                     "simr_set_tile", "simr_set_lsm_launch", "simr_greeks_ext", "simr_basket_workspace_size",
                     "simr_basket_price", "simr_basket_greeks", "simr_debug_basket_paths",
                     "simr_debug_basket_lsm", "simr_debug_graph_stats", "simr_price_noalloc",
                     "simr_debug_fault", "simr_basket_risk"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
        # registered after torch's own exit handlers, so it runs before them
        atexit.register(shutdown)
    return _lib


def shutdown():
    """Waits for the device, destroys every context (its graphs, events, pinned staging and
    device table) and drops the cached workspaces, while the HIP runtime is still whole.
    Runs at interpreter exit; calling it earlier is allowed (contexts are made again on use)."""
    if _lib is None:
        return
    try:
        torch.cuda.synchronize()
    except Exception:
        pass
    for dev in list(_ctx):
        _lib.simr_destroy(_ctx.pop(dev))
    _ws.clear()


def _check(status: int):
    if status != 0:
        raise SimrError(status, library().simr_last_error().decode())


def context(device: int | None = None) -> ctypes.c_void_p:
    dev = torch.cuda.current_device() if device is None else device
    if dev not in _ctx:
        h = ctypes.c_void_p()
        _check(library().simr_create(ctypes.byref(h), dev))
        _ctx[dev] = h
    return _ctx[dev]


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _params(scheme: int, checkpoint_every: int = 0) -> _Params:
    return _Params(scheme, checkpoint_every, 0, 0)


def _as_options(opts):
    out = []
    for o in opts:
        out.append(o if isinstance(o, Option) else Option.from_dict(o))
    return out


def workspace(nbytes: int) -> torch.Tensor:
    """A device scratch tensor of at least `nbytes`, reused across calls."""
    dev = torch.cuda.current_device()
    t = _ws.get(dev)
    if t is None or t.numel() < nbytes:
        _ws.pop(dev, None)
        t = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8, device=f"cuda:{dev}")
        _ws[dev] = t
    return t


def workspace_size(op: int, opts, scheme: int = SCHEME_QE, checkpoint_every: int = 0) -> int:
    L = library()
    c_opts = (_Option * len(opts))(*[o._c() for o in _as_options(opts)])
    prm = _params(scheme, checkpoint_every)
    n = ctypes.c_size_t()
    _check(L.simr_workspace_size(context(), op, c_opts, len(opts), ctypes.byref(prm), ctypes.byref(n)))
    return n.value


def price_batch(opts, scheme: int = SCHEME_QE) -> list[Result]:
    """Prices a list of options (Option or dicts) in one call."""
    L = library()
    opts = _as_options(opts)
    n = len(opts)
    c_opts = (_Option * n)(*[o._c() for o in opts])
    prm = _params(scheme)
    need = workspace_size(1, opts, scheme)
    ws = workspace(need)
    res = (_Result * n)()
    _check(L.simr_price_batch(context(), c_opts, n, ctypes.byref(prm), res, ctypes.c_void_p(ws.data_ptr()),
                              ws.numel(), _stream()))
    return [Result(r.price, r.std_err, r.paths, r.lsm_flags) for r in res]


def price(opt, scheme: int = SCHEME_QE) -> Result:
    L = library()
    o = _as_options([opt])[0]
    c_opt = o._c()
    prm = _params(scheme)
    ws = workspace(workspace_size(0, [o], scheme))
    r = _Result()
    _check(L.simr_price(context(), ctypes.byref(c_opt), ctypes.byref(prm), ctypes.byref(r),
                        ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return Result(r.price, r.std_err, r.paths, r.lsm_flags)


def price_noalloc(opt, scheme: int = SCHEME_QE) -> Result:
    """A European option priced by the allocation-free entry point (no workspace: the library's
    static device scratch)."""
    L = library()
    o = _as_options([opt])[0]
    c_opt = o._c()
    prm = _params(scheme)
    r = _Result()
    _check(L.simr_price_noalloc(context(), ctypes.byref(c_opt), ctypes.byref(prm), ctypes.byref(r), _stream()))
    return Result(r.price, r.std_err, r.paths, r.lsm_flags)


def greeks(opt, scheme: int = SCHEME_QE, checkpoint_every: int = 16) -> GreeksResult:
    """Price and the 7 pathwise adjoint Greeks (S0, v0, theta, r, kappa, xi, rho)."""
    L = library()
    o = _as_options([opt])[0]
    c_opt = o._c()
    prm = _params(scheme, checkpoint_every)
    ws = workspace(workspace_size(2, [o], scheme, checkpoint_every))
    r = _GreeksResult()
    _check(L.simr_greeks(context(), ctypes.byref(c_opt), ctypes.byref(prm), ctypes.byref(r),
                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return GreeksResult(r.price, r.std_err, list(r.g), list(r.g_se), r.lsm_flags)


def greeks_batch(opts, scheme: int = SCHEME_QE, checkpoint_every: int = 16) -> list[GreeksResult]:
    """greeks() of every option in one call (one synchronisation; the same results)."""
    L = library()
    opts = _as_options(opts)
    n = len(opts)
    c_opts = (_Option * n)(*[o._c() for o in opts])
    prm = _params(scheme, checkpoint_every)
    ws = workspace(workspace_size(3, opts, scheme, checkpoint_every))
    res = (_GreeksResult * n)()
    _check(L.simr_greeks_batch(context(), c_opts, n, ctypes.byref(prm), res, ctypes.c_void_p(ws.data_ptr()),
                               ws.numel(), _stream()))
    return [GreeksResult(r.price, r.std_err, list(r.g), list(r.g_se), r.lsm_flags) for r in res]


def greeks_ext(opt, scheme: int = SCHEME_QE, checkpoint_every: int = 16) -> GreeksResult:
    """Price, the 7 Greeks, d/dT (steps fixed) and gamma (European options; NaN for American)."""
    L = library()
    o = _as_options([opt])[0]
    c_opt = o._c()
    prm = _params(scheme, checkpoint_every)
    ws = workspace(workspace_size(2, [o], scheme, checkpoint_every))
    r = _GreeksExtResult()
    _check(L.simr_greeks_ext(context(), ctypes.byref(c_opt), ctypes.byref(prm), ctypes.byref(r),
                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return GreeksResult(r.price, r.std_err, list(r.g), list(r.g_se), r.lsm_flags)


def debug_draws(seed: int, stream_id: int, path0: int, npaths: int, step0: int, nsteps: int):
    """(words uint32 as int64 [npaths, nsteps, 4], uniforms [.., 3], normals [.., 2]) from the GPU."""
    L = library()
    dev = torch.device("cuda", torch.cuda.current_device())
    w = torch.empty((npaths, nsteps, 4), dtype=torch.int32, device=dev)
    u = torch.empty((npaths, nsteps, 3), dtype=torch.float32, device=dev)
    z = torch.empty((npaths, nsteps, 2), dtype=torch.float32, device=dev)
    _check(L.simr_debug_draws(context(), seed, stream_id, path0, npaths, step0, nsteps, ctypes.c_void_p(w.data_ptr()),
                              ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(z.data_ptr()), _stream()))
    torch.cuda.synchronize()
    return (w.cpu().numpy().view("uint32"), u.cpu().numpy(), z.cpu().numpy())


def debug_paths(opt, scheme: int = SCHEME_QE):
    """Per-path (x_T, v_T, discounted payoff) of one option, FP32, from the production path code."""
    L = library()
    o = _as_options([opt])[0]
    c_opt = o._c()
    prm = _params(scheme)
    dev = torch.device("cuda", torch.cuda.current_device())
    xT = torch.empty(o.paths, dtype=torch.float32, device=dev)
    vT = torch.empty_like(xT)
    pay = torch.empty_like(xT)
    _check(L.simr_debug_paths(context(), ctypes.byref(c_opt), ctypes.byref(prm), ctypes.c_void_p(xT.data_ptr()),
                              ctypes.c_void_p(vT.data_ptr()), ctypes.c_void_p(pay.data_ptr()), _stream()))
    torch.cuda.synchronize()
    return xT.cpu().numpy(), vT.cpu().numpy(), pay.cpu().numpy()


def debug_lsm(opt, scheme: int = SCHEME_QE):
    """(Result, exercise index per path, FP64 coefficients per date [N+1, 6]) of an American option."""
    L = library()
    o = _as_options([opt])[0]
    c_opt = o._c()
    prm = _params(scheme)
    dev = torch.device("cuda", torch.cuda.current_device())
    ws = workspace(workspace_size(0, [o], scheme))
    tau = torch.empty(o.paths, dtype=torch.int32, device=dev)
    beta = torch.empty((o.steps + 1, 6), dtype=torch.float64, device=dev)
    r = _Result()
    _check(L.simr_debug_lsm(context(), ctypes.byref(c_opt), ctypes.byref(prm), ctypes.byref(r),
                            ctypes.c_void_p(tau.data_ptr()), ctypes.c_void_p(beta.data_ptr()),
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return Result(r.price, r.std_err, r.paths, r.lsm_flags), tau.cpu().numpy(), beta.cpu().numpy()


def _as_basket(b) -> Basket:
    return b if isinstance(b, Basket) else Basket.from_dict(b)


def basket_workspace_size(op: int, b, scheme: int = SCHEME_QE) -> int:
    c_b = _as_basket(b)._c()
    prm = _params(scheme)
    n = ctypes.c_size_t()
    _check(library().simr_basket_workspace_size(context(), op, ctypes.byref(c_b), ctypes.byref(prm),
                                                ctypes.byref(n)))
    return n.value


def basket_price(b, scheme: int = SCHEME_QE) -> Result:
    """Price of a basket (Basket or dict): European, or American by Longstaff-Schwartz."""
    bk = _as_basket(b)
    c_b = bk._c()
    prm = _params(scheme)
    ws = workspace(basket_workspace_size(0, bk, scheme))
    r = _Result()
    _check(library().simr_basket_price(context(), ctypes.byref(c_b), ctypes.byref(prm), ctypes.byref(r),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return Result(r.price, r.std_err, r.paths, r.lsm_flags)


def basket_greeks(b, scheme: int = SCHEME_QE) -> BasketGreeks:
    """Price, deltas and (European) cross-gammas of a basket."""
    bk = _as_basket(b)
    d = bk.assets
    c_b = bk._c()
    prm = _params(scheme)
    ws = workspace(basket_workspace_size(2, bk, scheme))
    r = _BasketGreeksResult()
    _check(library().simr_basket_greeks(context(), ctypes.byref(c_b), ctypes.byref(prm), ctypes.byref(r),
                                        ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    g = [[r.gamma[i * MAX_ASSETS + j] for j in range(d)] for i in range(d)]
    gs = [[r.gamma_se[i * MAX_ASSETS + j] for j in range(d)] for i in range(d)]
    return BasketGreeks(r.price, r.std_err, list(r.delta[:d]), list(r.delta_se[:d]), g, gs, r.lsm_flags)


def basket_risk(b, scheme: int = SCHEME_QE) -> BasketRisk:
    """Price, per-asset vegas in v0 and theta, and correlation sensitivities of a basket of at
    most 8 assets (QE, full-truncation Euler or truncated Gaussian)."""
    bk = _as_basket(b)
    d = bk.assets
    c_b = bk._c()
    prm = _params(scheme)
    ws = workspace(basket_workspace_size(3, bk, scheme))
    r = _BasketRiskResult()
    _check(library().simr_basket_risk(context(), ctypes.byref(c_b), ctypes.byref(prm), ctypes.byref(r),
                                      ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    m = [[r.dcorr[i * MAX_ASSETS + j] for j in range(d)] for i in range(d)]
    ms = [[r.dcorr_se[i * MAX_ASSETS + j] for j in range(d)] for i in range(d)]
    return BasketRisk(r.price, r.std_err, list(r.vega_v0[:d]), list(r.vega_v0_se[:d]), list(r.vega_theta[:d]),
                      list(r.vega_theta_se[:d]), m, ms, r.lsm_flags)


def debug_basket_paths(b, scheme: int = SCHEME_QE):
    """Per-path (x_T [P, d], v_T [P, d], discounted payoff [P]) of a basket, FP32."""
    bk = _as_basket(b)
    c_b = bk._c()
    prm = _params(scheme)
    dev = torch.device("cuda", torch.cuda.current_device())
    ws = workspace(basket_workspace_size(0, bk, scheme))
    xT = torch.empty((bk.paths, bk.assets), dtype=torch.float32, device=dev)
    vT = torch.empty_like(xT)
    pay = torch.empty(bk.paths, dtype=torch.float32, device=dev)
    _check(library().simr_debug_basket_paths(context(), ctypes.byref(c_b), ctypes.byref(prm),
                                             ctypes.c_void_p(xT.data_ptr()), ctypes.c_void_p(vT.data_ptr()),
                                             ctypes.c_void_p(pay.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                             ws.numel(), _stream()))
    return xT.cpu().numpy(), vT.cpu().numpy(), pay.cpu().numpy()


def debug_basket_lsm(b, scheme: int = SCHEME_QE):
    """(Result, exercise index per path, FP64 coefficients [N+1, 10]) of an American basket."""
    bk = _as_basket(b)
    c_b = bk._c()
    prm = _params(scheme)
    dev = torch.device("cuda", torch.cuda.current_device())
    ws = workspace(basket_workspace_size(0, bk, scheme))
    tau = torch.empty(bk.paths, dtype=torch.int32, device=dev)
    beta = torch.empty((bk.steps + 1, BASKET_NB), dtype=torch.float64, device=dev)
    r = _Result()
    _check(library().simr_debug_basket_lsm(context(), ctypes.byref(c_b), ctypes.byref(prm), ctypes.byref(r),
                                           ctypes.c_void_p(tau.data_ptr()), ctypes.c_void_p(beta.data_ptr()),
                                           ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return Result(r.price, r.std_err, r.paths, r.lsm_flags), tau.cpu().numpy(), beta.cpu().numpy()


def set_lsm_launch(mode: int, grid_max: int = 0):
    """0: one cooperative persistent launch for all dates (default); 1: one launch per date;
    2: failure test; 3 and 4: cooperative on 256-thread or 1024-thread blocks only."""
    _check(library().simr_set_lsm_launch(context(), mode, grid_max))


FAULT_OFF, FAULT_ALLOC, FAULT_LAUNCH, FAULT_SYNC = 0, 1, 2, 3


def debug_fault(kind: int, nth: int = 1) -> int:
    """Arms (kind 1 alloc, 2 launch, 3 sync) or disarms (0) host-side fault injection on this
    context; returns the number of faults injected on it so far."""
    fired = ctypes.c_int64()
    _check(library().simr_debug_fault(context(), kind, nth, ctypes.byref(fired)))
    return fired.value


def graph_stats():
    """(graphs captured, launches of captured graphs) of the batch calls on this context."""
    c, n = ctypes.c_int64(), ctypes.c_int64()
    _check(library().simr_debug_graph_stats(context(), ctypes.byref(c), ctypes.byref(n)))
    return c.value, n.value


def get_tile():
    b, p = ctypes.c_int32(), ctypes.c_int32()
    _check(library().simr_get_tile(context(), ctypes.byref(b), ctypes.byref(p)))
    return b.value, p.value


def set_tile(block: int, paths_per_lane: int):
    _check(library().simr_set_tile(context(), block, paths_per_lane))


class HestonPrice(torch.autograd.Function):
    """price = HestonPrice.apply(S0, v0, theta, r, kappa, xi, rho, contract)

    `contract` is an :class:`Option` supplying K, T, payoff, steps, paths and
    seed; the seven model inputs are 0-d tensors.  The forward pass runs
    simr_greeks (the pricing pass with checkpoints and the adjoint sweep in the
    same library call); backward returns grad_output times the adjoint Greeks.
    """

    @staticmethod
    def forward(ctx, S0, v0, theta, r, kappa, xi, rho, contract):
        vals = [float(t) for t in (S0, v0, theta, r, kappa, xi, rho)]
        o = Option(**{**contract.__dict__, **dict(zip(GREEK_NAMES, vals))})
        g = greeks(o)
        ctx.save_for_backward(torch.tensor(g.grads, dtype=torch.float64))
        return torch.tensor(g.price, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        (gr,) = ctx.saved_tensors
        gs = [grad_out * gr[i] for i in range(7)]
        return (*gs, None)
