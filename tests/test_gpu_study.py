"""Reduced-statistics physics smoke run of the potential study (Sec. 3.1):
16 FP32 chains of 24^4 at beta = 1, one two-level multilevel run each with
10 x 100 iterations and analytical multihit, V(r) of Eq. (4) with jackknife
errors and the fit of Eq. (1) with the Luscher term fixed to pi/12.

Stated tolerance: the fitted string tension lies within 10 % of the paper's
0.16719(30) (Sec. 3.1, tests/golden/paper_results.json).  The paper's
statistics are 100 configurations of 100 x 1000 iterations; at this smoke
statistics the fit uses the few separations the correlator resolves, and
500 thermalisation sweeps from a cold start leave beta = 1, just below the
transition, not fully equilibrated, so only the magnitude is checked."""
import json
import os
import sys

import pytest

from paper_1208_0166_amd import study

pytestmark = pytest.mark.gpu


def test_reduced_statistics_string_tension(tmp_path):
    print("[gpu] potential study: 16 chains, n1 10, n2 100, 500 sweeps", flush=True)
    out = tmp_path / "potential.json"
    assert study.main(["potential", "--replicas", "16", "--n1", "10", "--n2", "100", "--therm", "500",
                       "--out", str(out)]) == 0
    res = json.loads(out.read_text())
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_results.json")) as fh:
        paper = json.load(fh)["potential_fit_luscher_fixed"]["sigma"]
    fit = res["fits"]["luscher_fixed"]
    print(f"  sigma {fit['sigma']:.4f} +- {fit['d_sigma_jackknife']:.4f} over r = {res['fit_r']}, paper {paper}",
          flush=True)
    sys.stdout.flush()
    assert len(res["fit_r"]) >= 3
    assert abs(fit["sigma"] - paper) < 0.10 * paper
    # V(r) rises with r over the fitted range (confinement)
    V = res["V"]
    k = [res["r"].index(int(r)) for r in res["fit_r"]]
    assert all(V[a] < V[b] for a, b in zip(k, k[1:]))
