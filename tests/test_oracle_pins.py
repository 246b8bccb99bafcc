"""Pins of the oracle's plain correlator and hot start against definitions
computed independently with numpy.

* Plain correlator (Sec. 2.2, the input of Eq. (4)):
  C(r) = L^-3 sum_x P*(x) P(x + r e_x) with P(x) = exp(i sum_t theta_0(x, t)),
  checked on random links, where a shift along y or z, the conjugated
  orientation P(x) P*(x + r e_x), or lines built from a spatial direction all
  give different numbers (on cold or pure-gauge lattices every variant is 1).
* Hot start (Sec. 2.1): theta = pi (2u - 1) with u = (w0 >> 11) 2^-53 and w0
  the first word of Philox4x64-10 at counter (n, 1 << 32 | mu, 0, 0), key
  (seed, 0); the words come from numpy's own Philox implementation.  The
  angles lie in [-pi, pi) and are uniform (Kolmogorov-Smirnov).
"""
import math

import numpy as np
import pytest
from scipy import stats

from tests.inputs import random_links


def _numpy_philox_block(ctr, key):
    # numpy's Philox increments its counter before producing a block: the block
    # of counter c is the first output of a generator started at c - 1
    c = [int(v) for v in ctr]
    c[0] -= 1
    for i in range(3):
        if c[i] < 0:
            c[i] += 1 << 64
            c[i + 1] -= 1
    g = np.random.Philox(key=np.array([int(k) for k in key], dtype=np.uint64),
                         counter=np.array(c, dtype=np.uint64))
    return g.random_raw(4)


def _lines(th, mu=0):
    """Polyakov line phases exp(i sum_t theta_mu(t, z, y, x)), shape (z, y, x)."""
    return np.exp(1j * th[..., mu].sum(axis=0))


def _corr(P, r, axis=2, conj_first=True):
    """L^-3 sum P*(x) P(x + r e) (conj_first) or P(x) P*(x + r e), e along the
    given array axis of P[z, y, x] (2 = x, 1 = y, 0 = z)."""
    Q = np.roll(P, -r, axis=axis)  # Q[..., x] = P[..., x + r]
    return np.mean(np.conj(P) * Q) if conj_first else np.mean(P * np.conj(Q))


@pytest.mark.parametrize("L,T,seed", [(4, 6, 301), (6, 4, 302)])
def test_plain_correlator_matches_numpy_definition(oracle_mod, L, T, seed):
    th = random_links(L, T, seed)
    g = oracle_mod.OracleLattice(L, T, 1.0, 1, hot=False)
    g.set_links(th)
    r_list = list(range(1, L))
    got = g.plain_correlator(r_list)
    P = _lines(th)
    ref = np.array([_corr(P, r) for r in r_list])
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)
    # the Polyakov average of the same lines
    p = g.polyakov()
    assert abs(complex(p[0], p[1]) - P.mean()) < 1e-13


def test_plain_correlator_sees_axis_orientation_and_direction(oracle_mod):
    # on random links every plausible mistake gives a different number (r = L/2
    # is left out: there x + r = x - r, so C(L/2) is real in either orientation)
    L, T = 6, 4
    th = random_links(L, T, 303)
    g = oracle_mod.OracleLattice(L, T, 1.0, 1, hot=False)
    g.set_links(th)
    P = _lines(th)
    for r in (1, 2, 4, 5):
        got = complex(g.plain_correlator([r])[0])
        wrong = {
            "shift along y": _corr(P, r, axis=1),
            "shift along z": _corr(P, r, axis=0),
            "P(x) P*(x + r)": _corr(P, r, conj_first=False),
            "lines of theta_x": _corr(_lines(th, mu=1), r),
            "lines of theta_z": _corr(_lines(th, mu=3), r),
        }
        for name, v in wrong.items():
            assert abs(got - v) > 1e-3, f"r={r}: indistinguishable from {name}"
    # the orientation matters only through the imaginary part, which random links make large
    assert abs(complex(g.plain_correlator([1])[0]).imag) > 1e-3


def test_hot_start_is_pi_2u_minus_1_of_the_philox_word(oracle_mod):
    L, T, seed = 4, 4, 0x1234_5678_9ABC
    g = oracle_mod.OracleLattice(L, T, 1.0, seed, hot=True)
    th = g.get_links().reshape(-1, 4)  # natural site index n = ((t L + z) L + y) L + x
    for n in range(L ** 3 * T):
        for mu in range(4):
            w = _numpy_philox_block([n, (1 << 32) | mu, 0, 0], [seed, 0])
            u = float(int(w[0]) >> 11) * 2.0 ** -53
            assert th[n, mu] == math.pi * (2.0 * u - 1.0), (n, mu)


def test_hot_start_range_and_uniformity(oracle_mod):
    L, T = 8, 8
    g = oracle_mod.OracleLattice(L, T, 1.0, 11, hot=True)
    th = g.get_links().ravel()
    assert th.min() >= -math.pi and th.max() < math.pi
    ks = stats.kstest(th, stats.uniform(loc=-math.pi, scale=2 * math.pi).cdf)
    assert ks.pvalue > 1e-3
    # each direction separately, and distinct seeds give distinct starts
    for mu in range(4):
        a = g.get_links()[..., mu].ravel()
        assert stats.kstest(a, stats.uniform(loc=-math.pi, scale=2 * math.pi).cdf).pvalue > 1e-4
    h = oracle_mod.OracleLattice(L, T, 1.0, 12, hot=True)
    assert np.mean(g.get_links() == h.get_links()) < 1e-3
    # hot-start lattices are disordered: plaquette near 0
    assert abs(g.plaquette()) < 5 / math.sqrt(6 * L ** 3 * T)


def test_oracle_results_do_not_depend_on_the_thread_count(oracle_mod):
    # the class passes and sums run over OpenMP threads; links, accept logs and
    # multilevel results are the same bits with one thread and with all
    runs = []
    n_all = oracle_mod.max_threads()
    try:
        for n in (1, max(n_all, 2)):
            oracle_mod.set_threads(n)
            g = oracle_mod.OracleLattice(6, 8, 1.0, 21, hot=True)
            logs = [g.sweep(1, 3, want_log=True) for _ in range(2)]
            c, f, _ = g.multilevel([4, 2], [2, 2], 1, 3, [1, 2, 3], rf_list=[2])
            runs.append((g.get_links(), logs, c, f, g.plaquette()))
    finally:
        oracle_mod.set_threads(n_all)
    (l1, g1, c1, f1, p1), (l2, g2, c2, f2, p2) = runs
    np.testing.assert_array_equal(l1, l2)
    for a, b in zip(g1, g2):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(c1, c2)
    np.testing.assert_array_equal(f1, f2)
    assert p1 == p2
