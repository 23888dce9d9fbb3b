"""Writes the fixtures of tests/golden/ from the oracle alone (test infrastructure: nothing here
touches the GPU library).  Run from the repository root:

    python tests/golden/make_golden.py

* philox4x32_10.txt -- Philox4x32-10 words (Salmon et al., SC'11) at the counter layout the
  method uses, (step, path, stream, 0) with key (seed_lo, seed_hi), at ordinary and extreme
  counters and keys.  tests/test_oracle_rng.py checks the same function against rocRAND's
  host implementation; the fixture keeps the words themselves.
* heston_european_reference.txt -- the small European call of the Heston model (S0 = K = 100,
  T = 1, r = 0.02, kappa = 1.5, theta = 0.04, xi = 0.3, rho = -0.7, v0 = 0.04): its price from
  the characteristic function (Heston 1993, in the Albrecher et al. 2007 form) by mpmath
  quadrature at 30 digits, the put by parity, the Black-Scholes limit of the same contract
  (xi -> 0, rho = 0, sigma = 0.2), and the FP64 oracle's Monte Carlo estimate at 8,192 paths x
  64 steps (Philox seed 1) under the quadratic-exponential scheme and under full-truncation
  Euler, with their standard errors.
"""
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import black_scholes, heston_cf  # noqa: E402

PHILOX_CASES = [  # (seed, stream, step, path)
    (0, 0, 0, 0),
    (1, 0, 0, 0),
    (1, 0, 1, 0),
    (1, 0, 0, 1),
    (1, 0, 63, 8191),
    (5, 63, 251, 1048575),
    (7, 0, 251, 131071),
    (4, 1, 0, 262143),
    (3, 1023, 503, 262143),
    ((1 << 32) + 3, 2, 17, 99),
    (0xDEADBEEFCAFEF00D, 12345, 100, 424242),
    ((1 << 64) - 1, (1 << 32) - 1, (1 << 32) - 1, (1 << 30) - 1),
]

C1 = dict(S0=100.0, K=100.0, T=1.0, r=0.02, kappa=1.5, theta=0.04, xi=0.3, rho=-0.7, v0=0.04)


def write_philox(path):
    lines = ["# Philox4x32-10 words written by tests/golden/make_golden.py (the oracle's implementation).",
             "# seed stream step path : w0 w1 w2 w3   (hex words; counter (step, path, stream, 0),",
             "# key (seed & 0xffffffff, seed >> 32))"]
    for seed, stream, step, p in PHILOX_CASES:
        w = oracle.philox4x32_10([step, p, stream, 0], [seed & 0xFFFFFFFF, seed >> 32])
        lines.append("%d %d %d %d : %s" % (seed, stream, step, p, " ".join("%08x" % int(x) for x in w)))
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def write_reference(path):
    args = tuple(C1[k] for k in ("S0", "K", "T", "r", "kappa", "theta", "xi", "rho", "v0"))
    call = heston_cf.call_price_mp(*args, dps=30)
    put = call - C1["S0"] + C1["K"] * math.exp(-C1["r"] * C1["T"])
    bs = float(black_scholes.call(C1["S0"], C1["K"], C1["T"], C1["r"], 0.2))
    rows = [("cf_call", call), ("cf_put", put), ("bs_limit_call_sigma_0.2", bs)]
    for scheme, name in ((0, "qe"), (1, "fte")):
        o = oracle.Option(**C1, payoff=0, steps=64, paths=8192, seed=1, scheme=scheme)
        price, se, _ = oracle.price_european(o)
        rows += [(f"mc_{name}_call_8192x64_seed1", price), (f"mc_{name}_call_8192x64_seed1_std_err", se)]
    lines = ["# Heston European call S0=100 K=100 T=1 r=0.02 kappa=1.5 theta=0.04 xi=0.3 rho=-0.7 v0=0.04,",
             "# written by tests/golden/make_golden.py from the oracle (characteristic-function price by",
             "# mpmath at 30 digits; Monte Carlo by the FP64 oracle).  name value (repr of a double)"]
    lines += ["%s %r" % (k, v) for k, v in rows]
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    oracle.build()
    write_philox(os.path.join(HERE, "philox4x32_10.txt"))
    write_reference(os.path.join(HERE, "heston_european_reference.txt"))
    print("written")
