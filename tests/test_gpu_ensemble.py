"""Ensembles of multilevel runs on the GPU and the connected profile of
Eq. (7), against the oracle's chain and its connected_profile."""
import sys

import numpy as np
import pytest

from paper_1208_0166_amd import u1ml

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def close_rel(a, b, rel=1e-12):
    scale = max(np.abs(b).max(), 1e-300)
    assert np.abs(a - b).max() <= rel * scale, (np.abs(a - b).max(), scale)


@pytest.mark.parametrize("squared,multihit", [(False, False), (True, False), (False, True)])
def test_ensemble_and_connected_profile_match_oracle(oracle_mod, squared, multihit):
    L, T, beta = 4, 8, 1.1
    r_list, rf = [1, 2, 3], [2, 3]
    say(f"[gpu] ensemble vs oracle squared={squared} multihit={multihit}")
    o = oracle_mod.OracleLattice(L, T, beta, 81, hot=True)
    g = u1ml.init_lattice(L, T, beta, 81)
    u1ml.set_estimator(g, multihit=multihit, field_squared=squared)
    with pytest.raises(u1ml.U1MLError) as e:
        u1ml.ensemble_read(g)
    assert e.value.code == u1ml.ESTATE
    fields, corrs, omeans = [], [], []
    for _ in range(3):
        o.sweep(1, 3)
        u1ml.sweep(g, 1, 3)
        c, f, _ = o.multilevel([4, 2], [2, 2], 1, 3, r_list, rf_list=rf, multihit=multihit, field_squared=squared)
        fields.append(f)
        corrs.append(c)
        omeans.append(o.field2_means() if squared else o.field_means())
        u1ml.multilevel(g, [4, 2], [2, 2], 1, 3, r_list, rf_list=rf)
        u1ml.ensemble_add(g)
    np.testing.assert_array_equal(u1ml.get_links(g), o.get_links())
    n, c_g, f_g, k_g = u1ml.ensemble_read(g, correlator=True, field_profile=True, connected=True)
    assert n == 3
    close_rel(c_g, np.mean(corrs, axis=0))
    close_rel(f_g, np.mean(fields, axis=0))
    close_rel(k_g, oracle_mod.connected_profile(fields, corrs, omeans, r_list, rf))
    # reset empties it; the next add starts a new ensemble
    u1ml.ensemble_reset(g)
    with pytest.raises(u1ml.U1MLError) as e:
        u1ml.ensemble_read(g)
    assert e.value.code == u1ml.ESTATE
    u1ml.ensemble_add(g)
    n, c1, _, _ = u1ml.ensemble_read(g)
    assert n == 1
    close_rel(c1, corrs[-1])


def test_ensemble_rejects_runs_of_another_shape():
    say("[gpu] ensemble shape checks")
    g = u1ml.init_lattice(4, 8, 1.0, 82)
    with pytest.raises(u1ml.U1MLError) as e:
        u1ml.ensemble_add(g)
    assert e.value.code == u1ml.ESTATE
    u1ml.multilevel(g, [2], [2], 1, 2, [1, 2], rf_list=[2])
    u1ml.ensemble_add(g)
    u1ml.multilevel(g, [2], [2], 1, 2, [1, 2, 3], rf_list=[2])
    with pytest.raises(u1ml.U1MLError) as e:
        u1ml.ensemble_add(g)
    assert e.value.code == u1ml.EINVAL
    u1ml.multilevel(g, [2], [2], 1, 2, [1, 2], rf_list=[2])
    u1ml.set_estimator(g, field_squared=True)
    u1ml.multilevel(g, [2], [2], 1, 2, [1, 2], rf_list=[2])
    with pytest.raises(u1ml.U1MLError) as e:
        u1ml.ensemble_add(g)
    assert e.value.code == u1ml.EINVAL
    # runs without field: the correlator mean only
    u1ml.ensemble_reset(g)
    u1ml.multilevel(g, [2], [2], 1, 2, [1, 2])
    u1ml.ensemble_add(g)
    n, c, _, _ = u1ml.ensemble_read(g)
    assert n == 1 and c.shape == (2,)
    with pytest.raises(u1ml.U1MLError) as e:
        u1ml.ensemble_read(g, field_profile=True)
    assert e.value.code == u1ml.ESTATE


def test_batch_ensemble_matches_oracle(oracle_mod):
    Ls, seeds, beta = [4, 6], [83, 84], 1.0
    r_list, rf = [1, 2, 3], [3]
    say("[gpu] batch ensemble vs oracle")
    b = u1ml.batch_create(Ls, [8, 8], [beta, beta], seeds)
    ors = [oracle_mod.OracleLattice(L, 8, beta, s) for L, s in zip(Ls, seeds)]
    runs = [([], [], []) for _ in Ls]
    for _ in range(2):
        u1ml.batch_multilevel(b, [4, 2], [2, 2], 1, 2, r_list, rf_list=rf)
        u1ml.batch_ensemble_add(b)
        for i, o in enumerate(ors):
            c, f, _ = o.multilevel([4, 2], [2, 2], 1, 2, r_list, rf_list=rf)
            runs[i][0].append(f)
            runs[i][1].append(c)
            runs[i][2].append(o.field_means())
    for i, o in enumerate(ors):
        np.testing.assert_array_equal(u1ml.batch_get_links(b, i), o.get_links())
        n, c_g, f_g, k_g = u1ml.batch_ensemble_read(b, i, correlator=True, field_profile=True, connected=True)
        assert n == 2 and f_g.shape == (1, 2, 6, Ls[i], Ls[i])
        close_rel(c_g, np.mean(runs[i][1], axis=0))
        close_rel(f_g, np.mean(runs[i][0], axis=0))
        close_rel(k_g, oracle_mod.connected_profile(runs[i][0], runs[i][1], runs[i][2], r_list, rf))
