"""Host analysis of multilevel results (Sec. 3 of arXiv:1208.0166).

* the static potential of Eq. (4), V(r) = -ln C(r) / N_t;
* jackknife errors over independent configurations (Sec. 3.3);
* the string-model fit of Eq. (1), V(r) = mu + sigma r - c / r, with the
  Luscher coefficient c fixed to pi (d - 2) / 24 or free (Sec. 3.1);
* the flux-tube ansatz of Eq. (10) fitted to a transverse profile in the
  mediator plane, and the squared width of Eq. (2) as the second moment of
  the fitted ansatz over the transverse plane (Sec. 3.3).

Plain numpy/scipy on host arrays: the inputs are correlators and connected
profiles read back from the library (u1ml.measure / u1ml.ensemble_read).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize


# ---------------------------------------------------------------------------
# Eq. (4) and jackknife
# ---------------------------------------------------------------------------
def potential(corr, n_t: int):
    """V(r) = -ln C(r) / N_t (Eq. (4)); C is real in expectation, its real
    part is used."""
    return -np.log(np.real(np.asarray(corr))) / float(n_t)


def jackknife(samples, estimator=lambda m: m):
    """Leave-one-out jackknife over the first axis of ``samples``
    ([n_configurations, ...]).  ``estimator`` maps a mean over configurations
    to the quantity of interest.  Returns (estimate on the full mean, error,
    the n leave-one-out estimates); error^2 = (n-1)/n sum_i (q_i - q_bar)^2."""
    x = np.asarray(samples)
    n = x.shape[0]
    if n < 2:
        raise ValueError("jackknife needs at least two configurations")
    full = np.asarray(estimator(x.mean(axis=0)))
    total = x.sum(axis=0)
    loo = np.array([np.asarray(estimator((total - x[i]) / (n - 1))) for i in range(n)])
    err = np.sqrt((n - 1) / n * ((loo - loo.mean(axis=0)) ** 2).sum(axis=0))
    return full, err, loo


# ---------------------------------------------------------------------------
# Eq. (1): V(r) = mu + sigma r - c / r
# ---------------------------------------------------------------------------
def luscher_coefficient(d: int = 4) -> float:
    """pi (d - 2) / 24; d = 4 gives the pi / 12 the paper compares with."""
    return math.pi * (d - 2) / 24.0


def fit_potential(r, V, dV, c=None):
    """Weighted least squares of Eq. (1) over the given points.

    c = None fits mu, sigma and c; a number fixes the Luscher coefficient
    (e.g. luscher_coefficient(4)).  The model is linear in its parameters, so
    the fit is the closed-form normal equations; parameter errors are the
    square roots of the diagonal of (X^T W X)^-1.  Returns a dict with mu,
    sigma, c, their errors (d_mu, d_sigma, d_c; d_c = 0 when fixed), chi2 and
    dof."""
    r = np.asarray(r, dtype=float)
    V = np.asarray(V, dtype=float)
    w = 1.0 / np.asarray(dV, dtype=float) ** 2
    if c is None:
        X = np.stack([np.ones_like(r), r, -1.0 / r], axis=1)
        y = V
    else:
        X = np.stack([np.ones_like(r), r], axis=1)
        y = V + c / r
    A = X.T @ (w[:, None] * X)
    cov = np.linalg.inv(A)
    p = cov @ (X.T @ (w * y))
    resid = y - X @ p
    chi2 = float((w * resid ** 2).sum())
    dof = len(r) - X.shape[1]
    out = {"mu": p[0], "sigma": p[1], "d_mu": math.sqrt(cov[0, 0]), "d_sigma": math.sqrt(cov[1, 1]),
           "chi2": chi2, "dof": dof}
    if c is None:
        out.update(c=p[2], d_c=math.sqrt(cov[2, 2]))
    else:
        out.update(c=float(c), d_c=0.0)
    return out


# ---------------------------------------------------------------------------
# Eqs. (10) and (2): transverse profile, ansatz, width
# ---------------------------------------------------------------------------
def transverse_profile(profile, comp: int, planes=(0, 1)):
    """Flatten one component of the profile of one separation, [2][6][L][L]
    (real), into (rho^2, value) pairs over the mediator plane.

    rho^2 = dy'^2 + dz'^2 with the periodic minimal images dy', dz' of the
    offsets.  The listed planes are averaged (for an even r the two planes sit
    symmetrically about the midpoint of the charges).  Points of equal rho^2
    are averaged too.  Returns (rho2 [n], value [n]) sorted by rho^2."""
    a = np.asarray(profile)
    if a.ndim != 4:
        raise ValueError("pass the profile of one separation, [2][6][L][L]")
    L = a.shape[-1]
    v = np.mean([a[p, comp] for p in planes], axis=0)
    d = np.minimum(np.arange(L), L - np.arange(L))
    rho2 = (d[:, None] ** 2 + d[None, :] ** 2).ravel()
    vals = v.ravel()
    keys = np.unique(rho2)
    means = np.array([vals[rho2 == k].mean() for k in keys])
    return keys.astype(float), means


def ansatz(rho2, A, s, B, D):
    """Eq. (10): A e^{-rho^2/s} (1 + B e^{-rho^2/s}) / (1 + D e^{-rho^2/s})."""
    u = np.exp(-np.asarray(rho2, dtype=float) / s)
    return A * u * (1.0 + B * u) / (1.0 + D * u)


def fit_ansatz(rho2, values, errors=None, p0=None):
    """Least-squares fit of Eq. (10) to (rho^2, value) points.  Returns
    (A, s, B, D) and their covariance."""
    rho2 = np.asarray(rho2, dtype=float)
    values = np.asarray(values, dtype=float)
    if p0 is None:
        A0 = values[0] if values[0] != 0 else 1.0
        # s from the first point below half the central value
        half = np.nonzero(np.abs(values) < 0.5 * abs(A0))[0]
        s0 = rho2[half[0]] / math.log(2.0) if len(half) and rho2[half[0]] > 0 else 1.0
        p0 = (A0, s0, 0.0, 0.0)
    p, cov = optimize.curve_fit(ansatz, rho2, values, p0=p0, sigma=errors,
                                absolute_sigma=errors is not None, maxfev=20000)
    return p, cov


def width2(A, s, B, D, dims: int = 2):
    """Eq. (2) on the fitted ansatz, w^2 = int x^2 f / int f (A cancels).

    dims = 2: over the whole transverse plane, x^2 = rho^2; with
    u = e^{-rho^2/s}, w^2 = s int_0^1 (-ln u) g(u) du / int_0^1 g(u) du,
    g = (1 + B u) / (1 + D u).  dims = 1: along one transverse axis through
    the flux-tube axis, w^2 = int x^2 f(x^2) dx / int f(x^2) dx."""
    del A

    def g(u):
        return (1.0 + B * u) / (1.0 + D * u)

    if dims == 2:
        num = integrate.quad(lambda u: -math.log(u) * g(u) if u > 0 else 0.0, 0.0, 1.0, limit=200)[0]
        den = integrate.quad(g, 0.0, 1.0, limit=200)[0]
        return s * num / den
    if dims == 1:
        def f(x):
            u = math.exp(-x * x / s)
            return u * g(u)
        num = integrate.quad(lambda x: x * x * f(x), 0.0, math.inf, limit=200)[0]
        den = integrate.quad(f, 0.0, math.inf, limit=200)[0]
        return num / den
    raise ValueError("dims must be 1 or 2")


def connected_part(profile, corr_rf, omean, squared: bool = False):
    """Eq. (7) for one field separation: profile [2][6][L][L] (mean
    <P* P O>), corr_rf = mean C(r_f), omean [6] = mean <O_c>.  Returns the
    real array that carries the signal: by charge conjugation <P* P O> is
    imaginary for the Eq. (5) operators and real for the squared components
    of Eq. (6) (squared=True)."""
    conn = np.asarray(profile) / corr_rf - np.asarray(omean, dtype=float)[None, :, None, None]
    return np.real(conn) if squared else np.imag(conn)


def flux_tube_width(profiles, corr_rf, omeans, comp: int = 0, squared: bool = False, planes=(0, 1), p0=None,
                    dims: int = 2):
    """Squared width w^2(r/2) of one field component (Eq. (2)) with its
    jackknife error over configurations.

    profiles [n][2][6][L][L]: each configuration's <P* P O> at one
    separation r; corr_rf [n]: its C(r); omeans [n][6]: its operator means.
    Every jackknife sample forms the connected profile (Eq. (7)) of its
    means, fits Eq. (10) over the mediator plane and integrates Eq. (2).
    Returns (w2, error, ansatz parameters (A, s, B, D) of the full sample)."""
    profiles = np.asarray(profiles)
    n = profiles.shape[0]
    shape = profiles.shape[1:]
    packed = np.concatenate([profiles.reshape(n, -1), np.asarray(corr_rf).reshape(n, 1),
                             np.asarray(omeans, dtype=float).astype(complex)], axis=1)

    def est(m):
        sig = connected_part(m[:-7].reshape(shape), m[-7], np.real(m[-6:]), squared)
        rho2, vals = transverse_profile(sig, comp, planes)
        p, _ = fit_ansatz(rho2, vals, p0=p0)
        return np.array([width2(*p, dims=dims), *p])

    full, err, _ = jackknife(packed, est)
    return float(full[0]), float(err[0]), full[1:]
