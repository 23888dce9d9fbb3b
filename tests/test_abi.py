"""The C-ABI library loads on the CPU, exports every function include/simr.h
declares, and rejects invalid arguments before it needs a GPU context (no
compute calls here)."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "simr.h")
LIB = os.path.join(ROOT, "paper_2402_12111_amd", "libsimr.so")

from paper_2402_12111_amd import simr as B  # noqa: E402  (ctypes structs only; no GPU use)


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:simr_status|const char\*)\s+(simr_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libsimr.so not built")
    L = ctypes.CDLL(LIB)
    L.simr_last_error.restype = ctypes.c_char_p
    L.simr_status_string.restype = ctypes.c_char_p
    L.simr_status_string.argtypes = [ctypes.c_int]
    return L


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n


def test_struct_layouts_match_header():
    # sizes implied by the header's field lists (natural alignment, x86-64)
    assert ctypes.sizeof(B._Option) == 9 * 8 + 4 + 4 + 8 + 8 + 4 + 4
    assert ctypes.sizeof(B._Params) == 16
    assert ctypes.sizeof(B._Result) == 32
    assert ctypes.sizeof(B._GreeksResult) == 16 + 14 * 8 + 8
    assert ctypes.sizeof(B._GreeksExtResult) == 16 + 18 * 8 + 8


def good_option(**kw):
    d = dict(S0=100.0, K=100.0, T=1.0, r=0.02, kappa=1.5, theta=0.04, xi=0.3, rho=-0.7, v0=0.04, payoff=0,
             steps=64, paths=8192, seed=1, stream=0)
    d.update(kw)
    return B.Option(**d)._c()


BAD = [dict(S0=0.0), dict(K=-1.0), dict(T=0.0), dict(kappa=0.0), dict(theta=-0.1), dict(v0=-1e-9), dict(xi=-0.1),
       dict(rho=1.0000001), dict(payoff=7), dict(steps=0), dict(paths=1), dict(r=math.nan), dict(S0=math.inf),
       dict(steps=1 << 20), dict(paths=(1 << 30) + 1)]


@pytest.mark.parametrize("bad", BAD)
def test_invalid_options_rejected_before_any_launch(lib, bad):
    o = good_option(**bad)
    prm = B._Params(0, 0, 0, 0)
    nbytes = ctypes.c_size_t(12345)
    rc = lib.simr_workspace_size(None, 0, ctypes.byref(o), ctypes.c_int64(1), ctypes.byref(prm), ctypes.byref(nbytes))
    assert rc == -1 and nbytes.value == 12345
    out = B._Result(-7.0, -7.0, -7, -7, 0)
    rc = lib.simr_price(None, ctypes.byref(o), ctypes.byref(prm), ctypes.byref(out), None, ctypes.c_size_t(0), None)
    assert rc == -1
    assert b"option" in lib.simr_last_error()
    assert (out.price, out.std_err, out.paths, out.lsm_flags) == (-7.0, -7.0, -7, -7)  # untouched


def test_invalid_params_and_reserved_fields(lib):
    o = good_option()
    nbytes = ctypes.c_size_t()
    for prm in (B._Params(5, 0, 0, 0), B._Params(-1, 0, 0, 0), B._Params(0, 7, 0, 0), B._Params(0, 0, 1, 0),
                B._Params(0, 0, 0, 1)):
        assert lib.simr_workspace_size(None, 0, ctypes.byref(o), ctypes.c_int64(1), ctypes.byref(prm),
                                       ctypes.byref(nbytes)) == -1
    o.reserved = 1
    assert lib.simr_workspace_size(None, 0, ctypes.byref(o), ctypes.c_int64(1), ctypes.byref(B._Params()),
                                   ctypes.byref(nbytes)) == -1


def test_valid_arguments_need_a_context(lib):
    o = good_option()
    prm = B._Params(0, 0, 0, 0)
    out = B._Result()
    rc = lib.simr_price(None, ctypes.byref(o), ctypes.byref(prm), ctypes.byref(out), None, ctypes.c_size_t(0), None)
    assert rc == -1 and b"ctx" in lib.simr_last_error()
    gout = B._GreeksResult()
    # Broadie-Kaya Greeks are not implemented: unsupported, not invalid; FTE, martingale-corrected
    # QE and truncated Gaussian Greeks pass validation and then need a context
    rc = lib.simr_greeks(None, ctypes.byref(o), ctypes.byref(B._Params(4, 0, 0, 0)), ctypes.byref(gout),
                         None, ctypes.c_size_t(0), None)
    assert rc == -4
    for scheme in (1, 2, 3):  # FTE, QE-M, TG
        rc = lib.simr_greeks(None, ctypes.byref(o), ctypes.byref(B._Params(scheme, 0, 0, 0)), ctypes.byref(gout),
                             None, ctypes.c_size_t(0), None)
        assert rc == -1 and b"ctx" in lib.simr_last_error()
    # the martingale-corrected, truncated Gaussian and Broadie-Kaya schemes are valid pricing schemes
    for scheme in (2, 3, 4):
        nbytes = ctypes.c_size_t()
        assert lib.simr_workspace_size(None, 0, ctypes.byref(o), ctypes.c_int64(1),
                                       ctypes.byref(B._Params(scheme, 0, 0, 0)), ctypes.byref(nbytes)) == 0
        assert nbytes.value > 0
    # the profiling controls need a context too
    lib.simr_profile_groups.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
    assert lib.simr_profile_groups(None, 1 << 2) == -1 and b"ctx" in lib.simr_last_error()
    assert lib.simr_profile_enable(None, 1) == -1


def test_workspace_sizes_grow_with_the_problem(lib):
    prm = B._Params(0, 0, 0, 0)
    sizes = []
    for op, kw in ((0, {}), (0, dict(paths=1 << 16)), (0, dict(payoff=2, steps=252, paths=131072)),
                   (2, {}), (2, dict(payoff=2, steps=252, paths=131072))):
        o = good_option(**kw)
        n = ctypes.c_size_t()
        assert lib.simr_workspace_size(None, op, ctypes.byref(o), ctypes.c_int64(1), ctypes.byref(prm),
                                       ctypes.byref(n)) == 0
        sizes.append(n.value)
    assert sizes[1] > sizes[0]
    # the American spill holds (x, v) per path and date: at least 8 bytes per path-step
    assert sizes[2] >= 8 * 131072 * 252
    assert sizes[4] >= sizes[2]
    # a batch needs at least what its largest member needs
    opts = (B._Option * 3)(good_option(), good_option(paths=1 << 16), good_option(payoff=2, steps=50, paths=4096))
    n = ctypes.c_size_t()
    assert lib.simr_workspace_size(None, 1, opts, ctypes.c_int64(3), ctypes.byref(prm), ctypes.byref(n)) == 0
    assert n.value >= sizes[1]


def test_status_strings(lib):
    for code, text in ((0, b"ok"), (-1, b"invalid argument"), (-3, b"HIP runtime error"), (-4, b"unsupported")):
        assert lib.simr_status_string(code) == text


def test_basket_struct_layouts_match_header():
    M = B.MAX_ASSETS
    assert M == 32
    assert ctypes.sizeof(B._BasketRiskResult) == 16 + 4 * M * 8 + 2 * M * M * 8 + 8
    assert ctypes.sizeof(B._Basket) == 4 * 4 + 8 + 8 + 4 + 4 + 3 * 8 + 7 * M * 8 + M * M * 8
    assert ctypes.sizeof(B._BasketGreeksResult) == 16 + 2 * M * 8 + 2 * M * M * 8 + 8


def good_basket(**kw):
    from paper_2402_12111_amd import workloads as W
    return B.Basket.from_dict(W.basket(3, **kw))._c()


def basket_rc(lib, b, op=0, prm=None):
    n = ctypes.c_size_t()
    prm = prm or B._Params(0, 0, 0, 0)
    return lib.simr_basket_workspace_size(None, op, ctypes.byref(b), ctypes.byref(prm), ctypes.byref(n)), n.value


def test_basket_arguments_validated_before_any_context(lib):
    assert basket_rc(lib, good_basket())[0] == 0
    bad = []
    b = good_basket(); b.corr[0 * 32 + 1] = 0.9; b.corr[1 * 32 + 0] = 0.2; bad.append(("symmetric", b))
    b = good_basket(); b.corr[1 * 32 + 1] = 0.99; bad.append(("diagonal", b))
    b = good_basket()
    for i, j, c in ((0, 1, 0.9), (0, 2, 0.9), (1, 2, -0.9)):
        b.corr[i * 32 + j] = b.corr[j * 32 + i] = c
    bad.append(("positive definite", b))
    b = good_basket(); b.w[1] = -0.1; bad.append(("weight", b))
    b = good_basket(); b.assets = 33; bad.append(("assets", b))
    b = good_basket(); b.assets = 0; bad.append(("assets", b))
    b = good_basket(); b.reserved0 = 1; bad.append(("reserved", b))
    b = good_basket(); b.kappa[2] = 0.0; bad.append(("kappa", b))
    b = good_basket(); b.corr[0] = math.nan; bad.append(("corr", b))
    for what, b in bad:
        rc, _ = basket_rc(lib, b)
        assert rc == -1, what
        assert what.encode() in lib.simr_last_error(), (what, lib.simr_last_error())
    # American baskets beyond the cooperative capacity are valid (one launch per date); their
    # workspace covers the write-out of 8 B per path-date
    rc, nbytes = basket_rc(lib, good_basket(payoff=2, paths=(1 << 20) + 1))
    assert rc == 0 and nbytes > 8 * ((1 << 20) + 1) * good_basket().steps
    assert basket_rc(lib, good_basket(), op=1)[0] == -1
    assert basket_rc(lib, good_basket(), op=3)[0] == 0  # the risk Greeks' workspace
    assert basket_rc(lib, good_basket(), prm=B._Params(4, 0, 0, 0))[0] == -4  # baskets take no BK
    # valid arguments, then the context is missing
    out = B._Result()
    rc = lib.simr_basket_price(None, ctypes.byref(good_basket()), ctypes.byref(B._Params(3, 0, 0, 0)),
                               ctypes.byref(out), None, ctypes.c_size_t(0), None)
    assert rc == -1 and b"ctx" in lib.simr_last_error()


def test_basket_workspace_sizes():
    import ctypes as C
    lib = C.CDLL(LIB)
    d = 3
    _, eu = basket_rc(lib, good_basket(paths=100000, steps=50))
    _, gr = basket_rc(lib, good_basket(paths=100000, steps=50), op=2)
    _, am = basket_rc(lib, good_basket(paths=100000, steps=50, payoff=2))
    assert gr >= eu + 4 * (1 + 2 * d) * 100000  # the per-path Greeks records
    assert am >= eu + 8 * 100000 * 50           # the basket write-out: 8 B per path and date


def _create_with_env(value):
    """simr_create(&ctx, 0) in a fresh process with SIMR_FAULT_INJECT=value: (status, message,
    whether ctx was written)."""
    import subprocess
    import sys
    code = (
        "import ctypes, sys\n"
        f"L = ctypes.CDLL({LIB!r})\n"
        "L.simr_last_error.restype = ctypes.c_char_p\n"
        "h = ctypes.c_void_p(12345)\n"
        "rc = L.simr_create(ctypes.byref(h), 0)\n"
        "print(rc, h.value == 12345, L.simr_last_error().decode())\n")
    env = dict(os.environ, SIMR_FAULT_INJECT=value)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr
    rc, untouched, msg = r.stdout.strip().split(" ", 2)
    return int(rc), untouched == "True", msg


def test_fault_injection_plan_is_parsed_before_any_hip_call(lib):
    """SIMR_FAULT_INJECT is read by simr_create before it touches HIP: a malformed plan is an
    invalid argument, the create plan fails the call as a HIP error with no HIP call made, and
    either way the context pointer is left untouched."""
    for bad in ("bogus", "launch:0", "launch:x", "sync:3x", "allocs", ""):
        rc, untouched, msg = _create_with_env(bad)
        assert rc == -1 and untouched and "SIMR_FAULT_INJECT" in msg, (bad, rc, msg)
    rc, untouched, msg = _create_with_env("create")
    assert rc == -3 and untouched and "injected create failure" in msg
    # a valid plan for later calls passes the parse; without a GPU the device query then fails
    for ok in ("alloc", "launch:2", "sync:17"):
        rc, untouched, msg = _create_with_env(ok)
        assert untouched and "SIMR_FAULT_INJECT" not in msg, (ok, rc, msg)


def test_fault_arming_needs_a_context(lib):
    fired = ctypes.c_int64(-1)
    assert lib.simr_debug_fault(None, 2, 1, ctypes.byref(fired)) == -1
    assert fired.value == -1 and b"ctx" in lib.simr_last_error()


def test_basket_risk_arguments_checked_before_any_context(lib):
    """More than 8 assets, or a scheme without risk tangents (martingale-corrected QE, exact),
    are unsupported; valid arguments then need a context; outputs stay untouched."""
    out = B._BasketRiskResult()
    out.price = -7.0
    for b, prm, rc_want in ((good_basket(), B._Params(0, 0, 0, 0), -1),
                            (B.Basket.from_dict(__import__("paper_2402_12111_amd.workloads", fromlist=["x"]).basket(9))._c(),
                             B._Params(0, 0, 0, 0), -4),
                            (good_basket(), B._Params(2, 0, 0, 0), -4), (good_basket(), B._Params(4, 0, 0, 0), -4)):
        rc = lib.simr_basket_risk(None, ctypes.byref(b), ctypes.byref(prm), ctypes.byref(out), None,
                                  ctypes.c_size_t(0), None)
        assert rc == rc_want, (rc, rc_want, lib.simr_last_error())
    assert out.price == -7.0


def test_greeks_batch_arguments_and_workspace_before_any_context(lib):
    """simr_greeks_batch checks every option (naming the first bad one) and its scheme before it
    needs a context.  Its workspace (op 3) is the largest single-option Greeks workspace when no
    two American options are adjacent; consecutive American options are sized as groups of at
    most 8 GiB (four of 2^20 paths x 252 steps, 2.1 GB of path states each), which hold the
    adjoint buffers once."""
    prm = B._Params(0, 0, 0, 0)
    members = [good_option(), good_option(payoff=2, steps=252, paths=131072), good_option(paths=1 << 16)]
    opts = (B._Option * 3)(*members)
    out = (B._GreeksResult * 3)()
    rc = lib.simr_greeks_batch(None, opts, ctypes.c_int64(3), ctypes.byref(prm), out, None, ctypes.c_size_t(0), None)
    assert rc == -1 and b"ctx" in lib.simr_last_error()
    rc = lib.simr_greeks_batch(None, opts, ctypes.c_int64(0), ctypes.byref(prm), out, None, ctypes.c_size_t(0), None)
    assert rc == -1
    rc = lib.simr_greeks_batch(None, opts, ctypes.c_int64(3), ctypes.byref(B._Params(4, 0, 0, 0)), out, None,
                               ctypes.c_size_t(0), None)
    assert rc == -4  # Broadie-Kaya Greeks: unsupported
    bad = (B._Option * 3)(members[0], members[1], good_option(paths=1))
    rc = lib.simr_greeks_batch(None, bad, ctypes.c_int64(3), ctypes.byref(prm), out, None, ctypes.c_size_t(0), None)
    assert rc == -1 and b"option 2" in lib.simr_last_error()
    single = []
    for o in members:
        n = ctypes.c_size_t()
        assert lib.simr_workspace_size(None, 2, ctypes.byref(o), ctypes.c_int64(1), ctypes.byref(prm),
                                       ctypes.byref(n)) == 0
        single.append(n.value)
    n = ctypes.c_size_t()
    assert lib.simr_workspace_size(None, 3, opts, ctypes.c_int64(3), ctypes.byref(prm), ctypes.byref(n)) == 0
    assert n.value == max(single)
    assert lib.simr_workspace_size(None, 2, opts, ctypes.c_int64(3), ctypes.byref(prm), ctypes.byref(n)) == -1
    big = good_option(payoff=2, steps=252, paths=1 << 20)
    one = ctypes.c_size_t()
    assert lib.simr_workspace_size(None, 2, ctypes.byref(big), ctypes.c_int64(1), ctypes.byref(prm),
                                   ctypes.byref(one)) == 0
    group = []
    for k in (2, 3, 4, 5):
        many = (B._Option * k)(*([big] * k))
        assert lib.simr_workspace_size(None, 3, many, ctypes.c_int64(k), ctypes.byref(prm), ctypes.byref(n)) == 0
        group.append(n.value)
    spill = 2 * 4 * (1 << 20) * 252
    steps = [group[0] - one.value, group[1] - group[0], group[2] - group[1]]  # one option more each
    assert one.value < group[0] < 2 * one.value and min(steps) >= spill and max(steps) - min(steps) <= 1024
    assert group[2] <= 8 << 30
    assert group[3] == group[2]  # a fifth would pass 8 GiB
