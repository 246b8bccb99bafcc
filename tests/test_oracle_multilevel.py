"""Pins of the oracle's multilevel estimators (Sec. 2.2, Eqs. (8), (9)).

Special cases where the nested averages collapse to the plain definitions
(one update per level; updates that are the identity; a cold lattice); the
nested averages of runs with several updates per level rebuilt in numpy from
the configurations of the same slab-frozen sweeps (two and three levels,
field insertion, multihit lines, the six directions); and a statistical check
that the multilevel estimator and the plain estimator agree.
"""
import math

import numpy as np
import pytest

from tests.test_oracle_multihit import multihit_means

AX = {0: 0, 1: 3, 2: 2, 3: 1}
FIELD_PLANES = [(0, 1), (0, 2), (0, 3), (2, 3), (3, 1), (1, 2)]  # E_x..E_z, B_x..B_z


def polyakov_lines(th):
    """P(x) = exp(i sum_t theta_0(x, t)), indexed [z][y][x]."""
    return np.exp(1j * th[..., 0].sum(axis=0))


def plain_corr(th, r):
    P = polyakov_lines(th)
    return np.mean(np.conj(P) * np.roll(P, -r, axis=2))


def field_ops(th, beta, squared=False):
    """O_c(t, z, y, x) = sqrt(beta) sin(theta_munu) for the six components, or
    with squared=True the Eq. (6) components beta (1 - cos(theta_munu))."""
    out = []
    for mu, nu in FIELD_PLANES:
        p = (th[..., mu] + np.roll(th[..., nu], -1, axis=AX[mu])
             - np.roll(th[..., mu], -1, axis=AX[nu]) - th[..., nu])
        out.append(beta * (1.0 - np.cos(p)) if squared else math.sqrt(beta) * np.sin(p))
    return np.array(out)


def field_identity(th, beta, r, squared=False):
    """(1/V) sum_x0 sum_t P*(x0) P(x0 + r) O(x0 + d, t) for d in both planes."""
    T, L = th.shape[0], th.shape[1]
    P = polyakov_lines(th)
    w = np.conj(P) * np.roll(P, -r, axis=2)          # [z][y][x]
    Osum = field_ops(th, beta, squared).sum(axis=1)  # [c][z][y][x]
    res = np.zeros((2, 6, L, L), dtype=complex)
    for plane, m in enumerate([(r - 1) // 2, r // 2]):
        for dy in range(L):
            for dz in range(L):
                sh = np.roll(np.roll(np.roll(Osum, -m, axis=3), -dy, axis=2), -dz, axis=1)
                res[plane, :, dy, dz] = (w[None] * sh).sum(axis=(1, 2, 3))
    return res / (T * L ** 3)


@pytest.mark.parametrize("levels", [([2], [1]), ([4, 2], [1, 1]), ([4], [1])])
def test_single_update_reduces_to_plain_correlator(oracle_mod, levels):
    L, T = 4, 8
    g = oracle_mod.OracleLattice(L, T, 1.0, 17)
    for _ in range(3):
        g.sweep(1, 2)
    r_list = [1, 2, 3]
    c, _, _ = g.multilevel(levels[0], levels[1], 1, 2, r_list)
    th = g.get_links()
    for k, r in enumerate(r_list):
        assert abs(c[k] - plain_corr(th, r)) < 1e-13


def test_identity_updates_give_plain_correlator(oracle_mod):
    # eps = 0 and no overrelaxation: every update returns the same link
    L, T = 4, 4
    g = oracle_mod.OracleLattice(L, T, 1.0, 5, eps=0.0)
    th = g.get_links()
    c, _, _ = g.multilevel([2], [5], 1, 0, [1, 2])
    np.testing.assert_array_equal(g.get_links(), th)
    for k, r in enumerate([1, 2]):
        assert abs(c[k] - plain_corr(th, r)) < 1e-13


@pytest.mark.parametrize("levels,rf", [(([2], [1]), [2]), (([4, 2], [1, 1]), [1, 2])])
def test_field_single_update_reduces_to_plain_definition(oracle_mod, levels, rf):
    L, T, beta = 4, 8, 1.0
    g = oracle_mod.OracleLattice(L, T, beta, 23)
    g.sweep(1, 1)
    c, f, _ = g.multilevel(levels[0], levels[1], 1, 1, [1, 2], rf_list=rf)
    th = g.get_links()
    for i, r in enumerate(rf):
        ref = field_identity(th, beta, r)
        np.testing.assert_allclose(f[i], ref, atol=1e-13)


def test_cold_lattice_field_vanishes(oracle_mod):
    g = oracle_mod.OracleLattice(4, 4, 1.0, 1, hot=False, eps=0.0)
    c, f, _ = g.multilevel([2], [3], 1, 0, [1, 2], rf_list=[2])
    np.testing.assert_array_equal(c, [1.0, 1.0])
    np.testing.assert_array_equal(f, np.zeros_like(f))


def test_accept_log_length(oracle_mod):
    L, T = 4, 4
    g = oracle_mod.OracleLattice(L, T, 1.0, 1)
    _, _, log = g.multilevel([4, 2], [2, 3], 1, 3, [1], log_cap=10 ** 6)
    n_sweeps = 2 + 2 * 3
    assert len(log) == n_sweeps * 8 * (g.V // 2)
    assert g.pass_id == n_sweeps


@pytest.mark.slow
def test_multilevel_and_plain_estimators_agree(oracle_mod):
    # Both estimate <P*(0) P(r)>; compare at r = 1 on 4^3 x 4, beta = 1.
    L, T, beta = 4, 4, 1.0
    g = oracle_mod.OracleLattice(L, T, beta, 2024)
    for _ in range(30):
        g.sweep(1, 3)
    plain, ml = [], []
    for _ in range(400):
        g.sweep(1, 3)
        plain.append(g.plain_correlator([1])[0].real)
    for _ in range(100):
        for _ in range(2):
            g.sweep(1, 3)
        c, _, _ = g.multilevel([2], [8], 1, 3, [1])
        ml.append(c[0].real)
    plain, ml = np.array(plain), np.array(ml)

    def err(x, b):
        n = len(x) // b
        m = x[: n * b].reshape(n, b).mean(axis=1)
        return m.std(ddof=1) / math.sqrt(n)

    d = abs(plain.mean() - ml.mean())
    e = math.hypot(err(plain, 20), err(ml, 5))
    assert d < 4 * e, (plain.mean(), ml.mean(), e)
    # the multilevel estimate is the less noisy one per unit of measurement
    assert ml.std() < plain.std()


@pytest.mark.parametrize("levels", [([2], [1]), ([4, 2], [1, 1])])
def test_field_squared_single_update_reduces_to_definition(oracle_mod, levels):
    # Eq. (6) components inserted instead of Eq. (5)
    L, T, beta = 4, 8, 1.2
    g = oracle_mod.OracleLattice(L, T, beta, 29)
    g.sweep(1, 2)
    _, f, _ = g.multilevel(levels[0], levels[1], 1, 2, [1, 2, 3], rf_list=[2, 3], field_squared=True)
    th = g.get_links()
    for i, r in enumerate([2, 3]):
        np.testing.assert_allclose(f[i], field_identity(th, beta, r, squared=True), atol=1e-13)


def test_field_squared_means_sum_to_the_plaquette(oracle_mod):
    # sum_c beta (1 - Re P_c) over the six orientations is 6 beta (1 - <plaquette>)
    g = oracle_mod.OracleLattice(4, 6, 0.8, 3)
    g.sweep(1, 3)
    m2 = g.field2_means()
    assert abs(m2.sum() - 6 * 0.8 * (1.0 - g.plaquette())) < 1e-13
    assert np.all(m2 > 0)
    cold = oracle_mod.OracleLattice(4, 4, 1.0, 1, hot=False)
    np.testing.assert_array_equal(cold.field2_means(), np.zeros(6))


@pytest.mark.parametrize("squared", [False, True])
def test_connected_profile_vanishes_for_a_constant_magnetic_field(oracle_mod, squared):
    # Eq. (7).  theta_y(x) = 2 pi x / L puts the same angle on every xy
    # plaquette whatever the temporal links are, so B_z is one constant and
    # B_x = B_y = 0 everywhere.  Identity updates (eps = 0, no OR) keep the
    # configuration, the field profile is then B_z C(r) at every offset and
    # the connected B profile is exactly zero; the E components, made from
    # random temporal links, are not constant and survive the subtraction.
    L, T, beta = 6, 4, 1.3
    rng = np.random.default_rng(5)
    th = np.zeros((T, L, L, L, 4))
    th[..., 0] = rng.uniform(-np.pi, np.pi, size=(T, L, L, L))
    th[..., 2] = ((2 * np.pi * np.arange(L) / L) + np.pi) % (2 * np.pi) - np.pi
    g = oracle_mod.OracleLattice(L, T, beta, 3, hot=False, eps=0.0)
    g.set_links(th)
    r_list, rf = [1, 2, 3], [2, 3]
    fields, corrs, omeans = [], [], []
    for _ in range(2):
        c, f, _ = g.multilevel([2], [2], 1, 0, r_list, rf_list=rf, field_squared=squared)
        fields.append(f)
        corrs.append(c)
        omeans.append(g.field2_means() if squared else g.field_means())
    np.testing.assert_array_equal(g.get_links(), th)
    # C(r) differs between the field separations, so a wrong r index shows
    assert abs(corrs[0][1] - corrs[0][2]) > 1e-3
    conn = oracle_mod.connected_profile(fields, corrs, omeans, r_list, rf)
    assert conn.shape == (2, 2, 6, L, L)
    assert np.abs(conn[:, :, 3:]).max() < 1e-13
    assert np.abs(conn[:, :, :3]).max() > 1e-2
    bz = beta * (1 - math.cos(2 * np.pi / L)) if squared else math.sqrt(beta) * math.sin(2 * np.pi / L)
    assert abs(omeans[0][5] - bz) < 1e-13
    ref = np.broadcast_to(bz * corrs[0][[1, 2], None, None, None], fields[0][:, :, 5].shape)
    np.testing.assert_allclose(fields[0][:, :, 5], ref, atol=1e-13)


def test_connected_profile_of_an_ensemble_uses_ratio_of_means(oracle_mod):
    # Eq. (7) divides the ensemble means, not run by run: with two runs whose
    # field profiles and correlators are proportional the ratio is the common
    # factor; a per-run average of ratios would give a different value here
    L = 2
    f1 = np.full((1, 2, 6, L, L), 2.0 + 0j)
    f2 = np.full((1, 2, 6, L, L), 1.0 + 0j)
    c1, c2 = np.array([1.0 + 0j]), np.array([3.0 + 0j])
    o = [np.arange(6) * 0.1, np.arange(6) * 0.3]
    conn = oracle_mod.connected_profile([f1, f2], [c1, c2], o, [1], [1])
    np.testing.assert_allclose(conn[0, 0, :, 0, 0], 3.0 / 4.0 - np.arange(6) * 0.2, atol=1e-15)


def plain_corr_dir(th, r, axis, sign):
    """L^-3 sum_x P*(x) P(x + sign r e_axis), axis 0, 1, 2 = x, y, z."""
    P = polyakov_lines(th)  # [z][y][x]
    return np.mean(np.conj(P) * np.roll(P, -sign * r, axis=2 - axis))


def plain_corr_sym(th, r):
    return np.mean([plain_corr_dir(th, r, a, s) for a in range(3) for s in (1, -1)])


@pytest.mark.parametrize("levels", [([2], [1]), ([4, 2], [1, 1]), ([4, 2, 1], [1, 1, 1])])
def test_symmetric_correlator_single_update_reduces_to_six_directions(oracle_mod, levels):
    # one update per level: the symmetric multilevel correlator is the plain
    # one averaged over the separations along +-x, +-y, +-z
    L, T = 4, 8
    g = oracle_mod.OracleLattice(L, T, 1.0, 19)
    g.sweep(1, 2)
    r_list = [1, 2, 3]
    c, _, _ = g.multilevel(levels[0], levels[1], 1, 2, r_list, symmetric=True)
    th = g.get_links()
    for k, r in enumerate(r_list):
        assert abs(c[k] - plain_corr_sym(th, r)) < 1e-13
    # and the six directions differ from one another on this configuration
    vals = [plain_corr_dir(th, 2, a, s) for a in range(3) for s in (1, -1)]
    assert np.ptp(np.real(vals)) > 1e-3


def test_symmetric_correlator_identity_updates_and_reality(oracle_mod):
    # identity updates (eps = 0, no OR) keep a random configuration for any
    # number of updates; both orientations make the average real
    L, T = 4, 8
    g = oracle_mod.OracleLattice(L, T, 1.0, 23, hot=True, eps=0.0)
    th = g.get_links()
    c, _, _ = g.multilevel([4, 2], [3, 2], 1, 0, [1, 2, 3], symmetric=True)
    for k, r in enumerate([1, 2, 3]):
        assert abs(c[k] - plain_corr_sym(th, r)) < 1e-13
    g2 = oracle_mod.OracleLattice(L, T, 1.0, 23, hot=True)
    c2, _, _ = g2.multilevel([4, 2], [3, 2], 1, 2, [1, 2, 3], symmetric=True)
    assert np.abs(c2.imag).max() < 1e-15
    g3 = oracle_mod.OracleLattice(L, T, 1.0, 23, hot=True)
    c3, _, _ = g3.multilevel([4, 2], [3, 2], 1, 2, [1, 2, 3])
    assert np.abs(c3.imag).max() > 1e-6  # one orientation alone is not real


def _shift(a, r, e):
    """a at x0 + r e for a[..., z, y, x] (periodic), e a unit vector (ex, ey, ez)."""
    return np.roll(np.roll(np.roll(a, -r * e[0], axis=-1), -r * e[1], axis=-2), -r * e[2], axis=-3)


DIRS6 = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]


def _two_level_by_replay(g, th0, th1, n0, n1, n_metro, n_or, r_list, rf, beta, multihit=False, symmetric=False):
    """C_ML(r) and the field estimator of Eq. (9) at separation rf of a
    two-level run (Sec. 2.2), rebuilt in numpy from the configurations the
    same slab-frozen sweeps produce: level-0 slabs of th0 (n0 updates), each
    followed by n1 updates in slabs of th1; per inner configuration the
    two-link products over each inner slab and the field operators summed over
    its times; inner averages over the n1 configurations, their products over
    the children of each top slab averaged over the n0 iterations; the
    insertion in one child with the other children's plain averages, and in
    one top slab with the other top slabs' averages.  multihit: for r >= 2 the
    correlator lines take the temporal links' multihit means (so also the
    averages that multiply an insertion elsewhere); the slab holding the
    insertion keeps the links themselves.  symmetric: C_ML(r) is the mean of
    the estimates along +-x, +-y, +-z, each with its own nested averages; the
    insertion stays along +x."""
    th = g.get_links()
    T, L = th.shape[0], th.shape[1]
    ns0, nch, ns1 = T // th0, th0 // th1, T // th1
    nr, kf = len(r_list), list(r_list).index(rf)
    dirs = DIRS6 if symmetric else DIRS6[:1]
    nd = len(dirs)
    A = np.zeros((ns0, L, L, L, nd, nr), dtype=complex)
    B = np.zeros((ns0, L, L, L, 2, 6, L, L), dtype=complex)
    for _ in range(n0):
        g.sweep(n_metro, n_or, th_frozen=th0)
        a1 = np.zeros((ns1, L, L, L, nd, nr), dtype=complex)
        b1 = np.zeros((ns1, L, L, L, 2, 6, L, L), dtype=complex)
        for _ in range(n1):
            g.sweep(n_metro, n_or, th_frozen=th1)
            th = g.get_links()
            u = np.exp(1j * th[..., 0])  # [t][z][y][x]
            if multihit:
                mm = multihit_means(th, beta)
            for di, e in enumerate(dirs):
                for k, r in enumerate(r_list):
                    v = mm if multihit and r >= 2 else u
                    tl = np.conj(v) * _shift(v, r, e)
                    a1[..., di, k] += tl.reshape(ns1, th1, L, L, L).prod(axis=1)
            tslab = (np.conj(u) * _shift(u, rf, (1, 0, 0))).reshape(ns1, th1, L, L, L).prod(axis=1)
            osl = field_ops(th, beta).reshape(6, ns1, th1, L, L, L).sum(axis=2)  # [c][slab][z][y][x]
            for plane, m in enumerate([(rf - 1) // 2, rf // 2]):
                for dy in range(L):
                    for dz in range(L):
                        sh = np.roll(np.roll(np.roll(osl, -m, axis=4), -dy, axis=3), -dz, axis=2)
                        b1[..., plane, :, dy, dz] += tslab[..., None] * np.moveaxis(sh, 0, -1)
        a1 /= n1
        b1 /= n1
        a1c = a1.reshape(ns0, nch, L, L, L, nd, nr)
        A += a1c.prod(axis=1)
        b1c = b1.reshape(ns0, nch, L, L, L, 2, 6, L, L)
        for ci in range(nch):
            other = np.ones((ns0, L, L, L), dtype=complex)
            for ch in range(nch):
                if ch != ci:
                    other = other * a1c[:, ch, ..., 0, kf]
            B += b1c[:, ci] * other[..., None, None, None, None]
    A /= n0
    B /= n0
    C = A.prod(axis=0).mean(axis=(0, 1, 2)).mean(axis=0)
    F = np.zeros((2, 6, L, L), dtype=complex)
    for s in range(ns0):
        other = np.ones((L, L, L), dtype=complex)
        for s2 in range(ns0):
            if s2 != s:
                other = other * A[s2, ..., 0, kf]
        F += (B[s] * other[..., None, None, None, None]).sum(axis=(0, 1, 2))
    return C, F / (T * L ** 3)


@pytest.mark.parametrize("multihit,symmetric", [(False, False), (True, False), (False, True), (True, True)])
@pytest.mark.parametrize("levels,n_sub", [([4, 2], [2, 3]), ([8, 2], [3, 2])])
def test_two_level_estimators_rebuilt_from_the_configurations(oracle_mod, levels, n_sub, multihit, symmetric):
    # several updates per level, so that every average is over more than one
    # configuration: the oracle's nested averages (correlator and field
    # insertion) against the same averages taken in numpy from the
    # configurations of the same update sequence
    L, T, beta = 4, 8, 1.0
    r_list, rf = [1, 2, 3], 2
    g1 = oracle_mod.OracleLattice(L, T, beta, 61)
    g2 = oracle_mod.OracleLattice(L, T, beta, 61)
    for g in (g1, g2):
        for _ in range(2):
            g.sweep(1, 2)
    c1, f1, _ = g1.multilevel(levels, n_sub, 1, 2, r_list, rf_list=[rf], multihit=multihit, symmetric=symmetric)
    c2, f2 = _two_level_by_replay(g2, levels[0], levels[1], n_sub[0], n_sub[1], 1, 2, r_list, rf, beta,
                                  multihit=multihit, symmetric=symmetric)
    np.testing.assert_array_equal(g1.get_links(), g2.get_links())
    assert g1.pass_id == g2.pass_id
    np.testing.assert_allclose(c1, c2, rtol=1e-12, atol=0)
    assert np.abs(f1[0] - f2).max() <= 1e-12 * np.abs(f2).max()
    # the estimates are not the plain ones of the final configuration
    assert abs(c1[0] - plain_corr(g1.get_links(), 1)) > 1e-6


def _level_by_replay(g, lev, ths, n_subs, r_list, beta, multihit, dirs):
    """Averages over n_subs[lev] updates in slabs of ths[lev] of the slab
    products: two-link lines over the slab's times at the innermost level,
    else the products of the children's averages (Sec. 2.2).  Returns
    [slab][z][y][x][dir][r]."""
    th = g.get_links()
    T, L = th.shape[0], th.shape[1]
    ns = T // ths[lev]
    acc = np.zeros((ns, L, L, L, len(dirs), len(r_list)), dtype=complex)
    for _ in range(n_subs[lev]):
        g.sweep(1, 2, th_frozen=ths[lev])
        if lev == len(ths) - 1:
            th = g.get_links()
            u = np.exp(1j * th[..., 0])
            if multihit:
                mm = multihit_means(th, beta)
            for di, e in enumerate(dirs):
                for k, r in enumerate(r_list):
                    v = mm if multihit and r >= 2 else u
                    tl = np.conj(v) * _shift(v, r, e)
                    acc[..., di, k] += tl.reshape(ns, ths[lev], L, L, L).prod(axis=1)
        else:
            child = _level_by_replay(g, lev + 1, ths, n_subs, r_list, beta, multihit, dirs)
            nch = ths[lev] // ths[lev + 1]
            acc += child.reshape((ns, nch) + child.shape[1:]).prod(axis=1)
    return acc / n_subs[lev]


@pytest.mark.parametrize("ths,n_subs", [([8, 4, 2], [2, 2, 3]), ([4, 2, 1], [2, 2, 2])])
@pytest.mark.parametrize("multihit,symmetric", [(False, False), (True, True)])
def test_three_level_correlator_rebuilt_from_the_configurations(oracle_mod, multihit, symmetric, ths, n_subs):
    # three levels on 4^3 x 8, every average over more than one
    # configuration: one top slab spanning T, or two top slabs with innermost
    # slabs of one time slice (only temporal links updated there)
    L, T, beta = 4, 8, 1.0
    r_list = [1, 2, 3]
    g1 = oracle_mod.OracleLattice(L, T, beta, 67)
    g2 = oracle_mod.OracleLattice(L, T, beta, 67)
    for g in (g1, g2):
        g.sweep(1, 2)
    c1, _, _ = g1.multilevel(ths, n_subs, 1, 2, r_list, multihit=multihit, symmetric=symmetric)
    dirs = DIRS6 if symmetric else DIRS6[:1]
    A = _level_by_replay(g2, 0, ths, n_subs, r_list, beta, multihit, dirs)
    c2 = A.prod(axis=0).mean(axis=(0, 1, 2)).mean(axis=0)
    np.testing.assert_array_equal(g1.get_links(), g2.get_links())
    np.testing.assert_allclose(c1, c2, rtol=1e-12, atol=0)
