"""The precision split at the paper's size (Sec. 2.1: 24^4, beta = 1) and on
the 48^4 lattice: FP32 sweeps with FP64 accumulation against the FP64 path,
which the parity tests tie bit for bit to the oracle.  Both run the same protocol (cold start,
thermalisation, then configurations separated by sweeps, each measured by a
two-level multilevel run, Sec. 2.2), so every observable has one expectation;
the test asserts agreement within 3 sigma (jackknife over independent chains)
for the plaquette, |P|, the multilevel correlator <P*(0) P(r)> at r = 1..4 and
the E_x insertion at r = 2 (Eq. (9): the FP32 path's field sums carry FP32
sines), and prints the relative deviation of each."""
import sys

import numpy as np
import pytest

from paper_1208_0166_amd import precision

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_fp32_vs_fp64_at_24_beta1_within_3_sigma():
    say("[gpu] 24^4 beta=1: 16 FP32 and 16 FP64 chains, 6 configurations each, multilevel {4,2} x {10,20}")
    rows = precision.compare(L=24, beta=1.0, n_chains=16, n_therm=200, n_configs=6, n_between=50,
                             levels=(4, 2), n_sub=(10, 20), r_list=(1, 2, 3, 4), seed0=2000, rf=2,
                             on_config=lambda name, k: say(f"  {name} configuration {k} done"))
    for row in rows:
        say(f"  {row['name']:>12}: fp32 {row['fp32'][0]:.6e} +- {row['fp32'][1]:.1e}  "
            f"fp64 {row['fp64'][0]:.6e} +- {row['fp64'][1]:.1e}  rel. deviation {row['rel_dev']:.2e}  "
            f"({row['sigmas']:.2f} sigma)")
    for row in rows:
        assert row["sigmas"] < 3.0, row
    by = {r["name"]: r for r in rows}
    # the FP64 side is the confining phase of the paper's workload
    assert 0.55 < by["plaquette"]["fp64"][0] < 0.62
    c = [by[f"C_ML(r={r})"]["fp64"][0] for r in (1, 2, 3, 4)]
    assert 0 < c[0] < 1e-3 and c[1] < c[0]
    # plaquette and |P| are resolved to better than 1 % relative
    assert by["plaquette"]["rel_err"] < 1e-2 and np.isfinite(by["poly_abs"]["rel_err"])
    # the E_x flux through the mediator plane is resolved (its sign fixed by
    # the charges): the comparison is not vacuous
    flux = by["Im E_x(r=2, plane sum)"]
    assert abs(flux["fp64"][0]) > 3 * flux["fp64"][1]


def test_fp32_vs_fp64_at_48_beta1_within_3_sigma():
    # the large-lattice workload (48^4, beta = 1: 85 MB of FP32 links per
    # chain) with its multilevel shape ({4,2} x {20,10}): 16 chains per
    # precision from the same cold start, a short thermalisation and two
    # measured configurations; every observable agrees within 3 sigma
    say("[gpu] 48^4 beta=1: 16 FP32 and 16 FP64 chains, 2 configurations each, multilevel {4,2} x {20,10}")
    rows = precision.compare(L=48, beta=1.0, n_chains=16, n_therm=100, n_configs=2, n_between=40,
                             levels=(4, 2), n_sub=(20, 10), r_list=(1, 2), seed0=4000,
                             on_config=lambda name, k: say(f"  {name} configuration {k} done"))
    for row in rows:
        say(f"  {row['name']:>12}: fp32 {row['fp32'][0]:.6e} +- {row['fp32'][1]:.1e}  "
            f"fp64 {row['fp64'][0]:.6e} +- {row['fp64'][1]:.1e}  rel. deviation {row['rel_dev']:.2e}  "
            f"({row['sigmas']:.2f} sigma)")
    for row in rows:
        assert row["sigmas"] < 3.0, row
    by = {r["name"]: r for r in rows}
    # the plaquette and C_ML(r = 1) are resolved (the comparison is not vacuous)
    assert by["plaquette"]["rel_err"] < 1e-3
    assert 0.5 < by["plaquette"]["fp64"][0] < 0.65
    c1 = by["C_ML(r=1)"]
    assert c1["fp64"][0] > 3 * c1["fp64"][1] and c1["fp32"][0] > 3 * c1["fp32"][1]
