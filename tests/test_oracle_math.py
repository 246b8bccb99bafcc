"""Pins of the oracle's random numbers and elementary functions.

Philox4x64-10 is pinned against numpy's independent implementation of the
same published generator; sin/cos/atan2 against the C library.
"""
import math

import numpy as np
import pytest


def _numpy_philox_block(ctr, key):
    # numpy's Philox increments the counter before producing a block, so the
    # block for counter c is the first output of a generator started at c - 1.
    c = [int(v) for v in ctr]
    c[0] -= 1
    for i in range(3):  # borrow
        if c[i] < 0:
            c[i] += 1 << 64
            c[i + 1] -= 1
    g = np.random.Philox(key=np.array([int(k) for k in key], dtype=np.uint64),
                         counter=np.array(c, dtype=np.uint64))
    return g.random_raw(4)


@pytest.mark.parametrize("ctr,key", [
    ([1, 0, 0, 0], [1, 0]),
    ([5, 7, 9, 11], [123, 456]),
    ([0, 2 << 32, 17, 0], [1, 0]),                      # counter borrow path
    ([255, (2 << 32) | (3 << 8) | 2, 12345, 0], [2**64 - 1, 0]),
    ([2**64 - 1, 2**64 - 1, 2**64 - 1, 2**64 - 1], [2**64 - 1, 2**64 - 1]),
])
def test_philox_matches_numpy(oracle_mod, ctr, key):
    out = oracle_mod.philox4x64_10(ctr, key)
    ref = _numpy_philox_block(ctr, key)
    assert [int(v) for v in out] == [int(v) for v in ref]


def test_philox_stream_uniformity(oracle_mod):
    # uniforms built as in the updates: (w >> 11) * 2^-53, over site counters
    words = np.array([oracle_mod.philox4x64_10([n, 2 << 32, 3, 0], [7, 0]) for n in range(20000)])
    u = (words >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    assert u.min() >= 0.0 and u.max() < 1.0
    counts, _ = np.histogram(u.ravel(), bins=64, range=(0, 1))
    expected = u.size / 64
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    # 63 dof: mean 63, sd ~11.2; 5 sd bound
    assert chi2 < 63 + 5 * 11.3
    # serial correlation between neighbouring counters and between words
    x = u[:, 0]
    for other in (u[:, 1], u[:, 2], u[:, 3], np.roll(x, 1)):
        r = np.corrcoef(x, other)[0, 1]
        assert abs(r) < 5 / math.sqrt(len(x))


def _ulps(a, ref):
    return abs(a - ref) / math.ulp(ref) if ref != 0 else abs(a) / 5e-324


def test_sincos_within_one_ulp_of_libm(oracle_mod):
    rng = np.random.default_rng(11)
    xs = np.concatenate([rng.uniform(-4 * math.pi, 4 * math.pi, 20000),
                         np.linspace(-13.0, 13.0, 20001),
                         [k * math.pi / 4 for k in range(-16, 17)],
                         [1e-300, -1e-300, 1e-8, 0.0]])
    for x in xs:
        s, c = oracle_mod.sincos(float(x))
        rs, rc = math.sin(x), math.cos(x)
        # the argument reduction is accurate to ~1e-25 absolute
        assert abs(s - rs) <= math.ulp(rs) + 1e-24, x
        assert abs(c - rc) <= math.ulp(rc) + 1e-24, x


def test_sincos_identities(oracle_mod):
    rng = np.random.default_rng(12)
    for x in rng.uniform(-12.0, 12.0, 2000):
        s, c = oracle_mod.sincos(float(x))
        assert abs(s * s + c * c - 1.0) < 4e-16
        s2, c2 = oracle_mod.sincos(float(-x))
        assert s2 == -s and c2 == c  # odd / even exactly (symmetric reduction)


def test_atan2_within_four_ulp_of_libm(oracle_mod):
    rng = np.random.default_rng(13)
    n = 30000
    ys = rng.normal(size=n) * rng.choice([1e-6, 1e-2, 1.0, 6.0], n)
    xs = rng.normal(size=n) * rng.choice([1e-6, 1e-2, 1.0, 6.0], n)
    worst = 0.0
    for y, x in zip(ys, xs):
        a, r = oracle_mod.atan2(float(y), float(x)), math.atan2(y, x)
        worst = max(worst, _ulps(a, r))
    assert worst <= 4.0
    # exact quadrant landmarks
    assert oracle_mod.atan2(1.0, 1.0) == math.pi / 4
    assert oracle_mod.atan2(1.0, 0.0) == math.pi / 2
    assert oracle_mod.atan2(-1.0, 0.0) == -math.pi / 2
    assert oracle_mod.atan2(0.0, 1.0) == 0.0
    assert abs(oracle_mod.atan2(1e-30, -1.0) - math.pi) <= math.ulp(math.pi)
