"""Pins of the oracle's action, updates and plain observables.

Each test checks the oracle against something other than itself: a brute-force
recomputation of the whole Wilson action, gauge invariance, exact closed forms
for special configurations, the exact single-link conditional density, or the
strong-coupling expansion.
"""
import math

import numpy as np
import pytest
from scipy import special, stats

from tests.inputs import random_angles, random_gauge, random_links, random_sites

# numpy axis of the shift along mu in theta[t][z][y][x][mu]
AX = {0: 0, 1: 3, 2: 2, 3: 1}


def gauge_transform(th, phi):
    """theta_mu(x) -> theta_mu(x) + phi(x) - phi(x + mu), wrapped to [-pi, pi)."""
    out = th.copy()
    for mu in range(4):
        out[..., mu] = th[..., mu] + phi - np.roll(phi, -1, axis=AX[mu])
    return (out + np.pi) % (2 * np.pi) - np.pi


def site(L, t, x, y, z):
    return ((t * L + z) * L + y) * L + x


def test_local_delta_equals_global_action_difference(oracle_mod):
    L = T = 4
    g = oracle_mod.OracleLattice(L, T, 1.3, 5)
    g.set_links(random_links(L, T, 21))
    sites = random_sites(g.V, 24, 22)
    vals = random_angles(24, 23)
    for k, (n, v) in enumerate(zip(sites, vals)):
        mu = k % 4
        before = g.total_action()
        d = g.local_delta(int(n), mu, float(v))
        th = g.get_links()
        flat = th.reshape(-1, 4)
        old = flat[n, mu]
        flat[n, mu] = v
        g.set_links(th)
        after = g.total_action()
        flat[n, mu] = old
        g.set_links(th)
        # total action ~ beta * 6V ~ 2000; rounding of that sum ~1e-12
        assert abs((after - before) - d) < 1e-10, (n, mu)


def test_local_delta_gauge_invariant(oracle_mod):
    L, T = 4, 6
    g = oracle_mod.OracleLattice(L, T, 1.0, 5)
    th = random_links(L, T, 31)
    phi = random_gauge(L, T, 32)
    g.set_links(th)
    sites = random_sites(g.V, 20, 33)
    vals = random_angles(20, 34)
    d0 = [g.local_delta(int(n), k % 4, float(v)) for k, (n, v) in enumerate(zip(sites, vals))]
    g.set_links(gauge_transform(th, phi))
    phif = phi.reshape(-1)
    d1 = []
    for k, (n, v) in enumerate(zip(sites, vals)):
        mu = k % 4
        t, z, y, x = np.unravel_index(int(n), (T, L, L, L))
        c = [t, x, y, z]
        c[mu] += 1
        m = site(L, c[0] % T, c[1] % L, c[2] % L, c[3] % L)
        d1.append(g.local_delta(int(n), mu, float(v + phif[n] - phif[m])))
    np.testing.assert_allclose(d1, d0, atol=1e-12)


def test_cold_start_observables_exact(oracle_mod):
    g = oracle_mod.OracleLattice(4, 6, 1.0, 1, hot=False)
    assert g.plaquette() == 1.0
    np.testing.assert_array_equal(g.polyakov(), [1.0, 0.0, 1.0])
    np.testing.assert_array_equal(g.plain_correlator([1, 2, 3]), [1.0, 1.0, 1.0])
    np.testing.assert_array_equal(g.field_means(), np.zeros(6))


def test_pure_gauge_observables(oracle_mod):
    L, T = 4, 6
    g = oracle_mod.OracleLattice(L, T, 1.0, 1, hot=False)
    g.set_links(gauge_transform(np.zeros((T, L, L, L, 4)), random_gauge(L, T, 41)))
    assert abs(g.plaquette() - 1.0) < 1e-15
    p = g.polyakov()
    assert abs(p[0] - 1.0) < 1e-14 and abs(p[1]) < 1e-14
    np.testing.assert_allclose(g.plain_correlator([1, 2]), [1.0, 1.0], atol=1e-14)
    np.testing.assert_allclose(g.field_means(), np.zeros(6), atol=1e-15)


def test_constant_links_unit_polyakov(oracle_mod):
    L, T = 4, 4
    g = oracle_mod.OracleLattice(L, T, 1.0, 1, hot=False)
    th = np.zeros((T, L, L, L, 4))
    th[..., :] = [0.3, -1.1, 2.0, 0.7]
    g.set_links(th)
    assert abs(g.plaquette() - 1.0) < 1e-15
    p = g.polyakov()
    assert abs(p[2] - 1.0) < 1e-14
    assert abs(p[0] - math.cos(4 * 0.3)) < 1e-14 and abs(p[1] - math.sin(4 * 0.3)) < 1e-14


@pytest.mark.parametrize("n_flux", [1, 2])
def test_quantised_constant_field(oracle_mod, n_flux):
    # theta_y(x) = 2 pi n x / L: every xy plaquette carries 2 pi n / L,
    # including across the periodic seam; B_z = sqrt(beta) sin(2 pi n / L).
    L, T, beta = 6, 4, 1.7
    g = oracle_mod.OracleLattice(L, T, beta, 1, hot=False)
    th = np.zeros((T, L, L, L, 4))
    xs = np.arange(L)
    th[..., 2] = ((2 * np.pi * n_flux * xs / L) + np.pi) % (2 * np.pi) - np.pi
    g.set_links(th)
    phi = 2 * np.pi * n_flux / L
    assert abs(g.plaquette() - (5 + math.cos(phi)) / 6) < 1e-15
    fm = g.field_means()
    np.testing.assert_allclose(fm, [0, 0, 0, 0, 0, math.sqrt(beta) * math.sin(phi)], atol=1e-14)
    # Eq. (3): only the V xy plaquettes contribute, each beta (1 - cos phi)
    V = L ** 3 * T
    assert abs(g.total_action() - beta * V * (1 - math.cos(phi))) < 1e-11


def test_overrelaxation_conserves_action_and_is_involution(oracle_mod):
    L = T = 4
    g = oracle_mod.OracleLattice(L, T, 1.0, 3)
    th0 = random_links(L, T, 51)
    g.set_links(th0)
    for mu in range(4):
        for p in range(2):
            # local conservation on each updated link
            flat = g.get_links().reshape(-1, 4)
            before_act = g.total_action()
            g.class_pass(mu, p, kind=1)
            after = g.get_links().reshape(-1, 4)
            changed = np.nonzero(after[:, mu] != flat[:, mu])[0]
            assert len(changed) > 0.9 * g.V / 2
            for n in changed[:40]:
                sr, si = g.staple(int(n), mu)
                c0 = math.cos(flat[n, mu]) * sr - math.sin(flat[n, mu]) * si
                c1 = math.cos(after[n, mu]) * sr - math.sin(after[n, mu]) * si
                assert abs(c0 - c1) < 1e-14
            assert abs(g.total_action() - before_act) < 1e-12 * before_act
            # applying the same class pass again restores the links
            g.class_pass(mu, p, kind=1)
            again = g.get_links().reshape(-1, 4)
            d = np.abs(((again[:, mu] - flat[:, mu]) + np.pi) % (2 * np.pi) - np.pi)
            assert d.max() < 1e-14
            g.set_links(after.reshape(th0.shape))


def test_metropolis_proposal_and_beta0_acceptance(oracle_mod):
    # At beta = 0 every proposal is accepted, and theta' - theta must be the
    # counter-based uniform eps*(2u1 - 1) of this link's Philox block.
    L = T = 4
    eps = 0.7
    g = oracle_mod.OracleLattice(L, T, 0.0, 9, eps=eps)
    th0 = g.get_links().reshape(-1, 4)
    g.pass_id = 5
    log = np.zeros(g.V // 2 * 2, dtype=np.uint8)
    g.class_pass(1, 1, kind=0, n_hits=2, pass_id=5, log=log)
    assert (log == 1).all()
    th1 = g.get_links().reshape(-1, 4)
    for n in range(g.V):
        t, z, y, x = np.unravel_index(n, (T, L, L, L))
        if (t + x + y + z) % 2 != 1:
            assert th1[n, 1] == th0[n, 1]
            continue
        expect = th0[n, 1]
        for h in range(2):
            w = oracle_mod.philox4x64_10([n, (2 << 32) | (h << 8) | 1, 5, 0], [9, 0])
            u1 = float(int(w[0]) >> 11) * 2.0 ** -53
            expect = expect + eps * (2 * u1 - 1)
            expect = (expect + math.pi) % (2 * math.pi) - math.pi
        assert abs(th1[n, 1] - expect) < 1e-14


def test_frozen_links_untouched(oracle_mod):
    L, T = 4, 8
    g = oracle_mod.OracleLattice(L, T, 1.0, 4)
    th0 = g.get_links()
    log = g.sweep(2, 1, th_frozen=4, want_log=True)
    th1 = g.get_links()
    for t in range(T):
        for mu in range(4):
            same = np.array_equal(th0[t, ..., mu], th1[t, ..., mu])
            assert same == (mu > 0 and t % 4 == 0), (t, mu)
    # frozen links are marked 2 in the accept log, all others 0/1
    half = g.V // 2
    log = log.reshape(4, 2, half, 2)
    assert set(np.unique(log[0])) <= {0, 1}
    assert (log[1:] != 2).sum() > 0 and (log[1:] == 2).sum() == 3 * (T // 4) * L ** 3 * 2


@pytest.mark.slow
def test_metropolis_samples_von_mises_conditional(oracle_mod):
    # Repeated Metropolis passes on one class leave every other link fixed, so
    # each link of the class is an independent chain whose stationary law is
    # exp(beta |S| cos(theta + alpha)) (Eq. (3)).  Probability-integral
    # transform of theta + alpha must be uniform.
    L = T = 8
    beta = 1.0
    g = oracle_mod.OracleLattice(L, T, beta, 77)
    mu, par = 2, 0
    pit = []
    pid = 0
    for rep in range(3):
        for _ in range(12):
            g.class_pass(mu, par, kind=0, n_hits=10, pass_id=pid)
            pid += 1
        th = g.get_links().reshape(-1, 4)
        for n in range(g.V):
            t, z, y, x = np.unravel_index(n, (T, L, L, L))
            if (t + x + y + z) % 2 != par:
                continue
            sr, si = g.staple(n, mu)
            kappa = beta * math.hypot(sr, si)
            phi = ((th[n, mu] + math.atan2(si, sr)) + np.pi) % (2 * np.pi) - np.pi
            pit.append(stats.vonmises.cdf(phi, kappa))
    pit = np.array(pit)
    res = stats.kstest(pit, "uniform")
    assert res.pvalue > 1e-4, res


@pytest.mark.slow
@pytest.mark.parametrize("beta", [0.0, 0.1])
def test_strong_coupling_plaquette(oracle_mod, beta):
    # <cos theta_p> = I1(beta)/I0(beta) + O(u^5); at beta=0.1 the correction
    # is ~1e-6, far below the statistical error here.
    L = T = 6
    g = oracle_mod.OracleLattice(L, T, beta, 101)
    for _ in range(5):
        g.sweep(1, 1)
    vals = []
    for _ in range(150):
        g.sweep(1, 1)
        vals.append(g.plaquette())
    vals = np.array(vals)
    mean = vals.mean()
    # blocks of 10 for the error (sweeps at this coupling decorrelate fast)
    err = vals.reshape(15, 10).mean(axis=1).std(ddof=1) / math.sqrt(15)
    u = special.i1(beta) / special.i0(beta)
    assert abs(mean - u) < 4 * err + 1e-6, (mean, u, err)
