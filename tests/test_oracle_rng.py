"""Pins of the oracle's random-number steps: Philox4x32-10, the uniform map and
Box-Muller.  Each check is against something other than the oracle itself."""
import numpy as np
from scipy import stats

import oracle


def test_philox_matches_rocrand(rocrand_kat):
    """Bit-exact Philox4x32-10 words against rocRAND over random counters and keys
    (Salmon et al. 2011; counter (step, path, stream, 0), key = seed)."""
    rng = np.random.default_rng(20240302)
    tuples = []
    for _ in range(400):
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        stream = int(rng.integers(0, 2**32, dtype=np.uint64))
        step = int(rng.integers(0, 2**32, dtype=np.uint64))
        path = int(rng.integers(0, 2**30))
        tuples.append((seed, stream, step, path))
    tuples += [(0, 0, 0, 0), (1, 0, 0, 0), (2**64 - 1, 2**32 - 1, 2**32 - 1, 2**30 - 1), (7, 0, 251, 131071)]
    expect = rocrand_kat(tuples)
    for (seed, stream, step, path), e in zip(tuples, expect):
        got = oracle.philox4x32_10([step, path, stream, 0], [seed & 0xFFFFFFFF, seed >> 32])
        assert [int(x) for x in got] == [int(x) for x in e], (seed, stream, step, path)


def test_rng_words_layout(rocrand_kat):
    """The block array of ref_rng_words is indexed [path][step][word] over the requested window."""
    w = oracle.rng_words(seed=7, stream=3, path0=1000, npaths=5, step0=250, nsteps=4)
    tuples = [(7, 3, 250 + n, 1000 + p) for p in range(5) for n in range(4)]
    expect = rocrand_kat(tuples).reshape(5, 4, 4)
    assert np.array_equal(w.astype(np.uint64), expect)


def test_uniform_grid_identity():
    """u = ((w >> 9) + 1/2) 2^-23: 2^24 u is the odd integer 2 (w >> 9) + 1, u lies in
    [2^-24, 1 - 2^-24], and u and 1 - u are exact in float32."""
    rng = np.random.default_rng(5)
    ws = list(rng.integers(0, 2**32, size=2000, dtype=np.uint64)) + [0, 511, 512, 2**32 - 1, 2**31]
    for w in ws:
        u = oracle.uniform(int(w))
        k = u * 2.0**24
        assert k == int(k) and int(k) == 2 * (int(w) >> 9) + 1
        assert 2.0**-24 <= u <= 1 - 2.0**-24
        assert float(np.float32(u)) == u and float(np.float32(1.0 - u)) == 1.0 - u


def test_box_muller_special_values():
    """Unit radius when -2 ln u0 = 1, and the four quarter angles."""
    u0 = np.exp(-0.5)
    for u1, (c, s) in [(0.0, (1, 0)), (0.25, (0, 1)), (0.5, (-1, 0)), (0.75, (0, -1))]:
        z1, z2 = oracle.box_muller(u0, u1)
        assert abs(z1 - c) < 1e-15 and abs(z2 - s) < 1e-15


def test_box_muller_normal_sample():
    """Gaussian variates built from Philox words: moments, independence of the pair,
    and a Kolmogorov-Smirnov test against the standard normal."""
    w = oracle.rng_words(seed=1, stream=0, path0=0, npaths=50000, step0=0, nsteps=2).reshape(-1, 4)
    z = np.array([oracle.box_muller(oracle.uniform(a), oracle.uniform(b)) for a, b in w[:, :2]])
    n = z.shape[0]
    for col in range(2):
        x = z[:, col]
        assert abs(x.mean()) < 4 / np.sqrt(n)
        assert abs(x.var() - 1) < 4 * np.sqrt(2 / n)
        kurt = ((x - x.mean()) ** 4).mean() / x.var() ** 2
        assert abs(kurt - 3) < 4 * np.sqrt(24 / n)
        assert stats.kstest(x, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 4 / np.sqrt(n)
    # the dyadic grid truncates the tail at sqrt(2 * 24 ln 2)
    assert np.abs(z).max() <= np.sqrt(-2 * np.log(2.0**-24)) + 1e-12


def test_box_muller_vectorised_restatement():
    """numpy's own log/cos/sin on the same uniforms give the same normals to 1 ulp-ish."""
    w = oracle.rng_words(seed=9, stream=1, path0=0, npaths=500, step0=0, nsteps=1).reshape(-1, 4)
    u0 = ((w[:, 0] >> 9).astype(np.float64) + 0.5) * 2.0**-23
    u1 = ((w[:, 1] >> 9).astype(np.float64) + 0.5) * 2.0**-23
    r = np.sqrt(-2 * np.log(u0))
    z = np.array([oracle.box_muller(a, b) for a, b in zip(u0, u1)])
    assert np.allclose(z[:, 0], r * np.cos(2 * np.pi * u1), rtol=0, atol=1e-13)
    assert np.allclose(z[:, 1], r * np.sin(2 * np.pi * u1), rtol=0, atol=1e-13)
