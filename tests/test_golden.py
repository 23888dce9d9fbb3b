"""The fixtures under tests/golden/ (written by tests/golden/make_golden.py from the oracle alone):
the oracle still reproduces them, and each is pinned to something other than the oracle --
the Philox words to rocRAND's host implementation, the characteristic-function price to an
independent quadrature of the same integrals, the Monte Carlo estimates to that price within
their standard errors."""
import math
import os

import pytest

import oracle
from oracle import black_scholes, heston_cf

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def philox_fixture():
    """[(seed, stream, step, path, [w0, w1, w2, w3])] from philox4x32_10.txt."""
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            lhs, rhs = line.split(":")
            seed, stream, step, path = (int(x) for x in lhs.split())
            rows.append((seed, stream, step, path, [int(w, 16) for w in rhs.split()]))
    return rows


def reference_fixture():
    """{name: value} from heston_european_reference.txt."""
    out = {}
    with open(os.path.join(GOLDEN, "heston_european_reference.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, value = line.split()
            out[name] = float(value)
    return out


C1 = dict(S0=100.0, K=100.0, T=1.0, r=0.02, kappa=1.5, theta=0.04, xi=0.3, rho=-0.7, v0=0.04)


def test_philox_fixture_is_the_oracle_and_rocrand(rocrand_kat):
    rows = philox_fixture()
    assert len(rows) >= 10
    expect = rocrand_kat([(seed, stream, step, path) for seed, stream, step, path, _ in rows])
    for (seed, stream, step, path, words), e in zip(rows, expect):
        got = oracle.philox4x32_10([step, path, stream, 0], [seed & 0xFFFFFFFF, seed >> 32])
        assert [int(x) for x in got] == words, (seed, stream, step, path)
        assert [int(x) for x in e] == words, (seed, stream, step, path)


def test_reference_prices():
    ref = reference_fixture()
    args = tuple(C1[k] for k in ("S0", "K", "T", "r", "kappa", "theta", "xi", "rho", "v0"))
    # the stored 30-digit quadrature against the oracle's double-precision one, and parity
    assert heston_cf.call_price(*args) == pytest.approx(ref["cf_call"], abs=1e-9)
    assert ref["cf_put"] == pytest.approx(ref["cf_call"] - 100.0 + 100.0 * math.exp(-0.02), abs=1e-12)
    assert black_scholes.call(100.0, 100.0, 1.0, 0.02, 0.2) == pytest.approx(ref["bs_limit_call_sigma_0.2"],
                                                                          abs=1e-12)
    for scheme, name in ((0, "qe"), (1, "fte")):
        o = oracle.Option(**C1, payoff=0, steps=64, paths=8192, seed=1, scheme=scheme)
        price, se, _ = oracle.price_european(o)
        key = f"mc_{name}_call_8192x64_seed1"
        assert price == pytest.approx(ref[key], rel=1e-13) and se == pytest.approx(ref[key + "_std_err"], rel=1e-12)
        assert abs(ref[key] - ref["cf_call"]) <= 3.0 * ref[key + "_std_err"], (name, ref[key], ref["cf_call"])
