"""Host analysis (Eqs. (1), (2), (4), (7), (10) and the jackknife) against
closed forms, exact synthetic data and brute-force sums."""
import math

import numpy as np
import pytest
from scipy import special

from paper_1208_0166_amd import analysis as an


def test_potential_inverts_the_correlator():
    r = np.arange(1, 13)
    V = 0.6 + 0.167 * r - math.pi / 12 / r
    C = np.exp(-24 * V) * (1 + 0j)
    np.testing.assert_allclose(an.potential(C, 24), V, rtol=1e-13)


def test_jackknife_of_the_mean_is_the_standard_error():
    x = np.random.default_rng(1).normal(size=(37, 3))
    est, err, loo = an.jackknife(x)
    np.testing.assert_allclose(est, x.mean(axis=0), rtol=1e-14)
    np.testing.assert_allclose(err, x.std(axis=0, ddof=1) / math.sqrt(37), rtol=1e-12)
    assert loo.shape == (37, 3)


def test_jackknife_of_a_nonlinear_estimator_matches_the_delta_method():
    rng = np.random.default_rng(2)
    n = 4000
    x = rng.normal(5.0, 0.5, size=n)
    _, err, _ = an.jackknife(x, np.log)
    # d log(m) = dm / m
    assert abs(err - 0.5 / math.sqrt(n) / 5.0) < 0.05 * err


@pytest.mark.parametrize("c", [None, math.pi / 12])
def test_potential_fit_recovers_exact_parameters(c):
    r = np.arange(3, 13, dtype=float)
    V = 0.61 + 0.1672 * r - (0.27 if c is None else c) / r
    fit = an.fit_potential(r, V, np.full(len(r), 1e-3), c=c)
    assert abs(fit["sigma"] - 0.1672) < 1e-12 and abs(fit["mu"] - 0.61) < 1e-12
    if c is None:
        assert abs(fit["c"] - 0.27) < 1e-11
    assert fit["chi2"] < 1e-15 and fit["dof"] == len(r) - (3 if c is None else 2)


def test_potential_fit_errors_cover_the_truth():
    # over many noisy data sets the sigma pulls are standard normal
    rng = np.random.default_rng(3)
    r = np.arange(3, 13, dtype=float)
    dV = 0.002 * r
    V0 = 0.61 + 0.1672 * r - math.pi / 12 / r
    pulls, chi2 = [], []
    for _ in range(400):
        fit = an.fit_potential(r, V0 + rng.normal(size=len(r)) * dV, dV, c=math.pi / 12)
        pulls.append((fit["sigma"] - 0.1672) / fit["d_sigma"])
        chi2.append(fit["chi2"] / fit["dof"])
    pulls = np.array(pulls)
    assert abs(pulls.mean()) < 0.2 and abs(pulls.std() - 1.0) < 0.1
    assert abs(np.mean(chi2) - 1.0) < 0.1


def test_luscher_coefficient():
    assert abs(an.luscher_coefficient(4) - math.pi / 12) < 1e-16
    assert an.luscher_coefficient(2) == 0.0


@pytest.mark.parametrize("s", [0.7, 2.0, 5.5])
def test_width_of_a_gaussian(s):
    # B = D (or both 0): f is a Gaussian e^{-rho^2/s}, whose second moment is
    # s over the plane and s / 2 along one axis
    for B in (0.0, 0.4, -0.3):
        assert abs(an.width2(1.0, s, B, B) - s) < 1e-10 * s
        assert abs(an.width2(1.0, s, B, B, dims=1) - s / 2) < 1e-8 * s


@pytest.mark.parametrize("B,D", [(0.5, 0.2), (-0.4, 1.3), (2.0, -0.5)])
def test_width_against_the_dilogarithm_closed_form(B, D):
    # int_0^1 g = B/D + (1 - B/D) ln(1 + D) / D,
    # int_0^1 (-ln u) g = B/D + (1 - B/D) (-Li2(-D) / D), Li2(-D) = spence(1 + D)
    s = 3.0
    q = B / D
    den = q + (1 - q) * math.log1p(D) / D
    num = q + (1 - q) * (-special.spence(1 + D) / D)
    assert abs(an.width2(0.2, s, B, D) - s * num / den) < 1e-9


def test_width_against_a_brute_force_plane_sum():
    A, s, B, D = 0.3, 2.5, 0.6, 0.25
    h = 0.02
    x = np.arange(-12, 12, h) + h / 2
    rho2 = x[:, None] ** 2 + x[None, :] ** 2
    f = an.ansatz(rho2, A, s, B, D)
    assert abs((rho2 * f).sum() / f.sum() - an.width2(A, s, B, D)) < 1e-6


def test_transverse_profile_minimal_images_and_planes():
    L = 6
    prof = np.zeros((2, 6, L, L))
    d = np.minimum(np.arange(L), L - np.arange(L))
    prof[0, 0] = d[:, None] ** 2 + d[None, :] ** 2
    prof[1, 0] = 3 * prof[0, 0]
    rho2, vals = an.transverse_profile(prof, 0)
    np.testing.assert_array_equal(rho2, [0, 1, 2, 4, 5, 8, 9, 10, 13, 18])
    np.testing.assert_allclose(vals, 2 * rho2)  # mean of the planes: (1 + 3) / 2 rho^2
    rho2, vals = an.transverse_profile(prof, 0, planes=(0,))
    np.testing.assert_allclose(vals, rho2)


def test_ansatz_fit_recovers_the_width_of_exact_data():
    L = 24
    A, s, B, D = -0.05, 3.0, 0.5, 0.2
    d = np.minimum(np.arange(L), L - np.arange(L))
    rho2 = (d[:, None] ** 2 + d[None, :] ** 2).astype(float)
    prof = np.zeros((2, 6, L, L))
    prof[:, 0] = an.ansatz(rho2, A, s, B, D)
    r2, v = an.transverse_profile(prof, 0)
    p, _ = an.fit_ansatz(r2, v)
    np.testing.assert_allclose(an.ansatz(r2, *p), v, atol=1e-10)
    assert abs(an.width2(*p) - an.width2(A, s, B, D)) < 1e-6


def test_flux_tube_width_of_synthetic_configurations():
    # configurations whose <P*P E_x> is C (i f(rho) + <E_x>) plus noise: the
    # jackknife width recovers w^2 of f within a few errors
    rng = np.random.default_rng(4)
    L, n = 16, 40
    A, s, B, D = 0.08, 2.2, 0.3, 0.1
    d = np.minimum(np.arange(L), L - np.arange(L))
    rho2 = (d[:, None] ** 2 + d[None, :] ** 2).astype(float)
    f = an.ansatz(rho2, A, s, B, D)
    profiles, corrs, omeans = [], [], []
    for _ in range(n):
        c = 0.02 * (1 + 0.1 * rng.normal())
        o = 1e-3 * rng.normal(size=6)
        prof = np.zeros((2, 6, L, L), dtype=complex)
        prof[:, 0] = c * (1j * f + o[0]) + 1e-4 * rng.normal(size=(2, L, L)) * (1 + 1j)
        profiles.append(prof)
        corrs.append(c + 0j)
        omeans.append(o)
    w2, err, p = an.flux_tube_width(profiles, corrs, omeans, comp=0)
    true = an.width2(A, s, B, D)
    assert err > 0 and abs(w2 - true) < 4 * err + 1e-3


def _golden():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_results.json")) as fh:
        return json.load(fh)


def test_luscher_coefficient_matches_the_value_the_paper_quotes():
    # the reading d = 4 in Eq. (1) gives the pi/12 = 0.2618 of Sec. 3.1
    g = _golden()
    assert abs(an.luscher_coefficient(4) - g["luscher_expected"]["value"]) < 5e-5
    assert abs(an.luscher_coefficient(3) - g["luscher_expected"]["value"]) > 0.1
