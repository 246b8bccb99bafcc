"""FP32-sweep / FP64-accumulate path against the FP64 path, statistically.

The two paths run the same Markov-chain protocol (Sec. 2.1 updates, Sec. 2.2
multilevel measurements) from the same cold start; only their random numbers
and the precision of the link arithmetic differ, so every observable has the
same expectation on both at every point of the protocol.  Independent chains
(one batch per precision, one lattice per chain) give one average per chain
over its measured configurations; the errors are jackknife errors over the
chains.  Compared: the average plaquette of Eq. (3), the Polyakov-loop
modulus |P|, the two-level multilevel correlator <P*(0) P(r)> (real part;
the input of Eq. (4)) and, on request, the E_x insertion of Eq. (9) in the
mediator plane (its imaginary part carries the signal, Eq. (5)).

Host code: every update and measurement runs in the library's kernels.
"""
from __future__ import annotations

import math

import numpy as np

from . import analysis as an
from . import u1ml


def run_chains(precision, L, beta, n_chains, n_therm, n_configs, n_between, levels, n_sub, r_list, seed0,
               stream=None, on_config=None, rf=None):
    """n_chains independent L^4 chains at one precision in one batch (cold
    start, seeds seed0 + i): n_therm sweeps, then n_configs times n_between
    sweeps and one multilevel run.  Returns per-chain, per-configuration
    observables [chain][config][2 + n_r (+ 2)]: plaquette, |P|, Re C_ML(r),
    and with a field separation rf the E_x insertion of Eq. (9) in the
    mediator plane (plane 0): Im <P* P E_x> at the plane's centre and summed
    over the plane (the flux of E_x through it)."""
    b = u1ml.batch_create([L] * n_chains, [L] * n_chains, [beta] * n_chains,
                          [seed0 + i for i in range(n_chains)], start=u1ml.COLD, precision=precision,
                          stream=stream)
    for _ in range(n_therm):
        u1ml.batch_sweep(b, 1, 3)
    n_obs = 2 + len(r_list) + (2 if rf else 0)
    out = np.zeros((n_chains, n_configs, n_obs))
    for k in range(n_configs):
        for _ in range(n_between):
            u1ml.batch_sweep(b, 1, 3)
        u1ml.batch_multilevel(b, levels, n_sub, 1, 3, r_list, rf_list=[rf] if rf else ())
        for i in range(n_chains):
            obs, c, f = u1ml.batch_measure(b, i, correlator=True, field_profile=bool(rf))
            out[i, k, 0] = obs["plaquette"]
            out[i, k, 1] = obs["poly_abs"]
            out[i, k, 2:2 + len(r_list)] = np.real(c)
            if rf:
                ex = f[0, 0, 0]  # [dy][dz] of E_x, plane 0
                out[i, k, -2] = ex[0, 0].imag
                out[i, k, -1] = ex.sum().imag
        if on_config:
            on_config(k)
    b.close()
    return out


def summarize(samples):
    """Mean over configurations per chain, then the mean over chains and its
    jackknife error (chains are independent; configurations of one chain are
    not).  samples: [chain][config][observable]."""
    per_chain = np.asarray(samples).mean(axis=1)
    mean, err, _ = an.jackknife(per_chain)
    return mean, err


def compare(L=24, beta=1.0, n_chains=8, n_therm=200, n_configs=4, n_between=50, levels=(4, 2), n_sub=(10, 20),
            r_list=(1, 2, 3, 4), seed0=2000, stream=None, on_config=None, rf=None):
    """Run both precisions and return one entry per observable:
    {"name", "fp32": [mean, err], "fp64": [mean, err], "rel_dev": |m32 - m64| / |m64|,
     "sigmas": |m32 - m64| / sqrt(err32^2 + err64^2)}."""
    res = {}
    for name, prec in (("fp32", u1ml.FP32), ("fp64", u1ml.FP64)):
        s = run_chains(prec, L, beta, n_chains, n_therm, n_configs, n_between, list(levels), list(n_sub),
                       list(r_list), seed0, stream=stream,
                       on_config=(lambda k, nm=name: on_config(nm, k)) if on_config else None, rf=rf)
        res[name] = summarize(s)
    names = ["plaquette", "poly_abs"] + [f"C_ML(r={r})" for r in r_list]
    if rf:
        names += [f"Im E_x(r={rf}, centre)", f"Im E_x(r={rf}, plane sum)"]
    rows = []
    for j, nm in enumerate(names):
        m32, e32 = float(res["fp32"][0][j]), float(res["fp32"][1][j])
        m64, e64 = float(res["fp64"][0][j]), float(res["fp64"][1][j])
        comb = math.hypot(e32, e64)
        rows.append({"name": nm, "fp32": [m32, e32], "fp64": [m64, e64],
                     "rel_dev": abs(m32 - m64) / abs(m64) if m64 != 0 else float("inf"),
                     "rel_err": comb / abs(m64) if m64 != 0 else float("inf"),
                     "sigmas": abs(m32 - m64) / comb if comb > 0 else (0.0 if m32 == m64 else float("inf"))})
    return rows
