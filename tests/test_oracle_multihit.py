"""Pins of the oracle's analytical multihit (Sec. 2.2: the temporal links of
the potential are replaced by their conditional means).

* I_1/I_0 against scipy's Bessel functions;
* the conditional mean of exp(i theta_0) against a direct quadrature over the
  link's angle of exp(-beta S_W), S_W the whole Wilson action Eq. (3);
* in the multilevel correlator: r = 1 keeps the links themselves (bit-equal
  to the plain estimator), and at r >= 2 the multihit estimator agrees with
  the plain one over independent configurations while its spread is smaller.
"""
import numpy as np
import pytest
from scipy import special

AX = {0: 0, 1: 3, 2: 2, 3: 1}  # direction -> axis of th[t][z][y][x]


def multihit_means(th, beta):
    """m(t, z, y, x) = conj(S)/|S| I_1(beta|S|)/I_0(beta|S|) for every temporal link,
    S its staple (numpy, from the definition of the Wilson action)."""
    t0 = th[..., 0]
    S = np.zeros(t0.shape, dtype=complex)
    for nu in (1, 2, 3):
        a = AX[nu]
        tn = th[..., nu]
        fwd = np.roll(tn, -1, axis=0) - np.roll(t0, -1, axis=a) - tn
        bwd = -(np.roll(t0, 1, axis=a) + np.roll(np.roll(tn, -1, axis=0), 1, axis=a) - np.roll(tn, 1, axis=a))
        S += np.exp(1j * fwd) + np.exp(1j * bwd)
    mag = np.abs(S)
    ratio = special.i1e(beta * mag) / special.i0e(beta * mag)
    out = np.zeros_like(S)
    nz = mag > 0
    out[nz] = ratio[nz] * np.conj(S[nz]) / mag[nz]
    return out


def multihit_corr(th, beta, r):
    """One update per level: (1/L^3) sum_x conj(M(x)) M(x + r), M the product over
    all times of the multihit means (r >= 2)."""
    M = multihit_means(th, beta).prod(axis=0)  # [z][y][x]
    return np.mean(np.conj(M) * np.roll(M, -r, axis=2))


@pytest.mark.parametrize("x", [0.0, 1e-9, 1e-3, 0.3, 1.0, 2.5, 6.0, 17.0, 60.0, 250.0])
def test_bessel_ratio_against_scipy(oracle_mod, x):
    ref = special.i1e(x) / special.i0e(x) if x > 0 else 0.0
    got = oracle_mod.bessel_ratio(x)
    assert abs(got - ref) <= 4e-15 * max(abs(ref), 1e-300) + 1e-300, (got, ref)


def test_bessel_ratio_large_argument_expansion(oracle_mod):
    for x in (601.0, 900.0, 5000.0):
        ref = special.i1e(x) / special.i0e(x)
        assert abs(oracle_mod.bessel_ratio(x) - ref) < 1e-12


def test_multihit_mean_is_conditional_mean_of_the_action(oracle_mod):
    L, T, beta = 4, 4, 1.3
    g = oracle_mod.OracleLattice(L, T, beta, 9, hot=True)
    th0 = g.get_links()
    rng = np.random.default_rng(2)
    grid = np.linspace(-np.pi, np.pi, 720, endpoint=False)
    for _ in range(4):
        t, z, y, x = (int(v) for v in rng.integers(0, L, 4))
        n = ((t * L + z) * L + y) * L + x
        # exp(-beta S_W) as the link's angle runs over the circle, all else fixed
        act = np.empty(len(grid))
        th = th0.copy()
        for i, a in enumerate(grid):
            th[t, z, y, x, 0] = a
            g.set_links(th)
            act[i] = g.total_action()
        w = np.exp(-(act - act.min()))  # total_action() is beta S_W
        ref = (w * np.exp(1j * grid)).sum() / w.sum()  # periodic trapezoid: spectrally accurate
        g.set_links(th0)
        got = g.multihit_mean(n)
        assert abs(got - ref) < 1e-12, (got, ref)


def test_multilevel_multihit_r1_unchanged_and_r2_reduced_variance(oracle_mod):
    L, T = 4, 8
    plain, mh = [], []
    for seed in range(40):
        ga = oracle_mod.OracleLattice(L, T, 1.0, 100 + seed, hot=True)
        gb = oracle_mod.OracleLattice(L, T, 1.0, 100 + seed, hot=True)
        for g in (ga, gb):
            for _ in range(10):
                g.sweep(1, 3)
        ca, _, _ = ga.multilevel([2], [20], 1, 3, [1, 2])
        cb, _, _ = gb.multilevel([2], [20], 1, 3, [1, 2], multihit=True)
        assert ca[0] == cb[0]  # r = 1 uses the links themselves
        np.testing.assert_array_equal(ga.get_links(), gb.get_links())  # the chain is not touched
        plain.append(ca[1].real)
        mh.append(cb[1].real)
    plain, mh = np.array(plain), np.array(mh)
    d = mh - plain
    assert abs(d.mean()) < 3 * d.std(ddof=1) / np.sqrt(len(d))
    assert mh.std(ddof=1) < plain.std(ddof=1)


def test_multihit_means_match_numpy_definition(oracle_mod):
    L, T, beta = 4, 6, 0.9
    g = oracle_mod.OracleLattice(L, T, beta, 4, hot=True)
    th = g.get_links()
    m = multihit_means(th, beta)
    for n in (0, 17, 93, 255, 300, L ** 3 * T - 1):
        t, rem = divmod(n, L ** 3)
        z, rem = divmod(rem, L * L)
        y, x = divmod(rem, L)
        assert abs(g.multihit_mean(n) - m[t, z, y, x]) < 1e-13


@pytest.mark.parametrize("levels", [([2], [1]), ([4, 2], [1, 1])])
def test_multihit_single_update_reduces_to_definition(oracle_mod, levels):
    L, T, beta = 4, 8, 1.0
    g = oracle_mod.OracleLattice(L, T, beta, 6, hot=True)
    g.sweep(1, 3)
    c, _, _ = g.multilevel(levels[0], levels[1], 1, 3, [1, 2, 3], multihit=True)
    th = g.get_links()
    from tests.test_oracle_multilevel import plain_corr
    assert abs(c[0] - plain_corr(th, 1)) < 1e-13
    for k, r in enumerate([2, 3], start=1):
        assert abs(c[k] - multihit_corr(th, beta, r)) < 1e-13
