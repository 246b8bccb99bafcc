"""GPU multilevel estimators against the oracle: two levels, field insertion
(Eq. (9)) evaluated by replay, and full-size properties at 24^4."""
import sys

import numpy as np
import pytest

from paper_1208_0166_amd import u1ml
from tests.test_oracle_multihit import multihit_corr
from tests.test_oracle_multilevel import field_identity, plain_corr

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# field profile tolerance relative to its largest entry: FP64 sums of FP64
# sines; for FP32 links the sines are FP32 (hardware sine, absolute error of
# order 1e-6 on angles up to 4 pi) before the FP64 accumulation
FIELD_REL = {u1ml.FP64: 1e-12, u1ml.FP32: 2e-5}


def close_rel(a, b, rel=1e-12):
    scale = max(np.abs(b).max(), 1e-300)
    assert np.abs(a - b).max() <= rel * scale, (np.abs(a - b).max(), scale)


@pytest.mark.parametrize("levels,n_sub,L,T,general", [
    ([4, 2], [3, 4], 4, 8, False),
    ([4, 2], [3, 4], 4, 8, True),
    ([2], [5], 4, 4, False),
    ([2], [5], 6, 4, True),
    ([6, 2], [2, 3], 4, 6, False),
    ([4, 2, 1], [2, 2, 2], 4, 8, False),
])
def test_multilevel_correlator_and_field_parity(oracle_mod, levels, n_sub, L, T, general):
    # general: the field contraction by stored transforms instead of the fused one
    r_list = [1, 2, 3]
    rf = [2, 3] if len(levels) <= 2 else []
    say(f"[gpu] multilevel parity levels={levels} n={n_sub} L={L} T={T} general={general}")
    o = oracle_mod.OracleLattice(L, T, 1.0, 5, hot=True)
    g = u1ml.init_lattice(L, T, 1.0, 5)
    if general:
        u1ml.set_debug(g, 2)
    for _ in range(2):
        o.sweep(1, 3)
        u1ml.sweep(g, 1, 3)
    c_o, f_o, _ = o.multilevel(levels, n_sub, 1, 3, r_list, rf_list=rf)
    u1ml.multilevel(g, levels, n_sub, 1, 3, r_list, rf_list=rf)
    _, c_g, f_g = u1ml.measure(g, observables=False, correlator=True, field_profile=bool(rf))
    np.testing.assert_array_equal(u1ml.get_links(g), o.get_links())
    close_rel(c_g, c_o)
    if rf:
        assert f_g.shape == f_o.shape
        close_rel(f_g, f_o)


def test_multilevel_fp32_matches_identity_at_one_update():
    # with one update per level the estimators reduce to the plain
    # definitions on the final links, for the FP32 path as well
    L, T = 6, 8
    g = u1ml.init_lattice(L, T, 1.0, 8, precision=u1ml.FP32)
    u1ml.sweep(g, 1, 3)
    u1ml.multilevel(g, [4, 2], [1, 1], 1, 3, [1, 2, 3], rf_list=[2])
    _, c, f = u1ml.measure(g, observables=False, correlator=True, field_profile=True)
    th = u1ml.get_links(g)
    ref = np.array([plain_corr(th, r) for r in (1, 2, 3)])
    np.testing.assert_allclose(c, ref, atol=1e-12)
    # the FP32 path evaluates the plaquette sines of the field in FP32
    close_rel(f[0], field_identity(th, 1.0, 2), rel=FIELD_REL[u1ml.FP32])


@pytest.mark.parametrize("prec", [u1ml.FP64, u1ml.FP32])
def test_full_size_24_identity_and_plain_observables(oracle_mod, prec):
    # 24^4 in the configuration of the benchmark: after one update per level
    # the multilevel correlator for r = 1..12 equals the plain correlator of
    # the final links, and the field at r = 2 the plain Eq. (9) definition.
    L = T = 24
    say(f"[gpu] 24^4 identity prec={prec}")
    g = u1ml.init_lattice(L, T, 1.0, 3, precision=prec, start=u1ml.COLD)
    for _ in range(3):
        u1ml.sweep(g, 1, 3)
    rl = list(range(1, 13))
    u1ml.multilevel(g, [4, 2], [1, 1], 1, 3, rl, rf_list=[2])
    obs, c, f = u1ml.measure(g, correlator=True, field_profile=True)
    th = u1ml.get_links(g)
    np.testing.assert_allclose(c, [plain_corr(th, r) for r in rl], atol=1e-12)
    close_rel(f[0], field_identity(th, 1.0, 2), rel=FIELD_REL[prec])
    o = oracle_mod.OracleLattice(L, T, 1.0, 3, hot=False)
    o.set_links(th)
    assert abs(obs["plaquette"] - o.plaquette()) < 1e-12
    p = o.polyakov()
    assert abs(obs["poly"] - complex(p[0], p[1])) < 1e-12


def test_full_size_24_sweep_bit_exact(oracle_mod):
    # one compound sweep of the 24^4 lattice from a hot start, FP64 path
    L = T = 24
    say("[gpu] 24^4 FP64 sweep vs oracle")
    o = oracle_mod.OracleLattice(L, T, 1.0, 2, hot=True)
    g = u1ml.init_lattice(L, T, 1.0, 2)
    o.sweep(1, 3)
    u1ml.sweep(g, 1, 3)
    np.testing.assert_array_equal(u1ml.get_links(g), o.get_links())


@pytest.mark.parametrize("prec", [u1ml.FP64, u1ml.FP32])
def test_multilevel_graph_replay_matches_eager(prec):
    L, T = 6, 8
    say(f"[gpu] multilevel graph vs eager prec={prec}")
    a = u1ml.init_lattice(L, T, 1.0, 12, precision=prec)
    b = u1ml.init_lattice(L, T, 1.0, 12, precision=prec, graphs=False)
    for k in range(3):
        for g in (a, b):
            u1ml.sweep(g, 1, 3)
            u1ml.multilevel(g, [4, 2], [2, 3], 1, 3, [1, 2, 3], rf_list=[2, 3])
        np.testing.assert_array_equal(u1ml.get_links(a), u1ml.get_links(b))
        _, ca, fa = u1ml.measure(a, observables=False, correlator=True, field_profile=True)
        _, cb, fb = u1ml.measure(b, observables=False, correlator=True, field_profile=True)
        np.testing.assert_array_equal(ca, cb)
        np.testing.assert_array_equal(fa, fb)
    assert u1ml.get_pass_id(a) == u1ml.get_pass_id(b) == 3 * (1 + 2 + 2 * 3)


def test_batch_multilevel_with_field_matches_oracle(oracle_mod):
    Ls, Ts = [4, 6], [8, 8]
    seeds = [41, 42]
    say("[gpu] batch multilevel with field vs oracle")
    b = u1ml.batch_create(Ls, Ts, [1.0, 0.9], seeds)
    ors = [oracle_mod.OracleLattice(L, T, be, s) for L, T, be, s in zip(Ls, Ts, [1.0, 0.9], seeds)]
    u1ml.batch_sweep(b, 1, 2)
    for o in ors:
        o.sweep(1, 2)
    u1ml.batch_multilevel(b, [4, 2], [2, 3], 1, 2, [1, 2, 3], rf_list=[2, 3])
    for i, o in enumerate(ors):
        c_o, f_o, _ = o.multilevel([4, 2], [2, 3], 1, 2, [1, 2, 3], rf_list=[2, 3])
        _, c_g, f_g = u1ml.batch_measure(b, i, correlator=True, field_profile=True)
        np.testing.assert_array_equal(u1ml.batch_get_links(b, i), o.get_links())
        close_rel(c_g, c_o)
        close_rel(f_g, f_o)


@pytest.mark.parametrize("L,rf,T,levels", [(10, [2, 3], 4, [2]), (12, [2, 3], 4, [2]), (20, [2, 3], 4, [2]),
                                           (32, [2, 3], 4, [2]), (24, list(range(1, 13)), 4, [2]),
                                           (32, [1, 2, 5, 7, 16], 4, [2]), (36, [5], 4, [2]), (40, [1, 8], 4, [2]),
                                           (48, [2, 4, 6], 4, [2]), (2, [1], 4, [2]), (6, [2, 3], 4, [2]),
                                           (8, [2, 3], 4, [2]), (16, [2, 5], 4, [2]), (18, [2, 3, 7], 4, [2]),
                                           (30, [2, 11], 4, [2]), (18, [2, 5], 8, [4, 2])])
def test_fused_field_contraction_matches_general(L, rf, T, levels):
    # the fused contraction (register FFTs of radices 2, 3, 4, 5) against the
    # general one (stored direct transforms) on the same chain, at every
    # length of the fused path (transform blocks of 1 to 12 planes, odd
    # counts and partial last groups among them); the long r lists split the
    # fused contraction into several blocks per sample; T = 8 with slabs of 2
    # under slabs of 4 gives four inner slabs, summed by the contraction
    # threads in groups of three and one
    say(f"[gpu] fused vs general field contraction L={L} T={T} levels={levels} rf={rf}")
    r_all = sorted(set(r for r in [1, 2, 3] + rf if r < L))
    res = []
    for general in (False, True):
        g = u1ml.init_lattice(L, T, 1.0, 21)
        if general:
            u1ml.set_debug(g, 2)
        u1ml.sweep(g, 1, 2)
        u1ml.multilevel(g, levels, [2] * len(levels), 1, 2, r_all, rf_list=rf)
        _, c, f = u1ml.measure(g, observables=False, correlator=True, field_profile=True)
        res.append((u1ml.get_links(g), c, f))
    np.testing.assert_array_equal(res[0][0], res[1][0])
    np.testing.assert_array_equal(res[0][1], res[1][1])
    close_rel(res[0][2], res[1][2])


@pytest.mark.parametrize("levels,n_sub,L,T,general", [
    ([4, 2], [2, 3], 4, 8, False),
    ([4, 2], [2, 3], 4, 8, True),
    ([2], [4], 6, 4, False),
    ([4, 2, 1], [2, 2, 2], 4, 8, False),
])
def test_multihit_parity(oracle_mod, levels, n_sub, L, T, general):
    # analytical multihit for r >= 2 (correlator and the averages multiplying a
    # field insertion), against the oracle's independent implementation
    r_list = [1, 2, 3]
    rf = [2, 3] if len(levels) <= 2 else []
    say(f"[gpu] multihit parity levels={levels} L={L} general={general}")
    o = oracle_mod.OracleLattice(L, T, 1.1, 31, hot=True)
    g = u1ml.init_lattice(L, T, 1.1, 31)
    u1ml.set_estimator(g, multihit=True)
    if general:
        u1ml.set_debug(g, 2)
    o.sweep(1, 3)
    u1ml.sweep(g, 1, 3)
    c_o, f_o, _ = o.multilevel(levels, n_sub, 1, 3, r_list, rf_list=rf, multihit=True)
    u1ml.multilevel(g, levels, n_sub, 1, 3, r_list, rf_list=rf)
    _, c_g, f_g = u1ml.measure(g, observables=False, correlator=True, field_profile=bool(rf))
    np.testing.assert_array_equal(u1ml.get_links(g), o.get_links())
    close_rel(c_g, c_o)
    if rf:
        close_rel(f_g, f_o)


def test_multihit_batch_and_toggle(oracle_mod):
    Ls, seeds = [4, 6], [51, 52]
    say("[gpu] multihit batch vs oracle, then off again")
    b = u1ml.batch_create(Ls, [8, 8], [1.0, 1.0], seeds)
    ors = [oracle_mod.OracleLattice(L, 8, 1.0, s) for L, s in zip(Ls, seeds)]
    for mh in (True, False):
        u1ml.batch_set_estimator(b, multihit=mh)
        u1ml.batch_multilevel(b, [4, 2], [2, 2], 1, 2, [1, 2, 3], rf_list=[2])
        for i, o in enumerate(ors):
            c_o, f_o, _ = o.multilevel([4, 2], [2, 2], 1, 2, [1, 2, 3], rf_list=[2], multihit=mh)
            _, c_g, f_g = u1ml.batch_measure(b, i, correlator=True, field_profile=True)
            np.testing.assert_array_equal(u1ml.batch_get_links(b, i), o.get_links())
            close_rel(c_g, c_o)
            close_rel(f_g, f_o)


@pytest.mark.parametrize("prec", [u1ml.FP64, u1ml.FP32])
def test_multihit_full_size_24_identity(prec):
    # 24^4, one update per level: the multihit correlator is the definition on
    # the final links (numpy); FP32 staples give ~1e-6 relative
    L = T = 24
    say(f"[gpu] 24^4 multihit identity prec={prec}")
    g = u1ml.init_lattice(L, T, 1.0, 13, precision=prec, start=u1ml.COLD)
    u1ml.set_estimator(g, multihit=True)
    for _ in range(3):
        u1ml.sweep(g, 1, 3)
    rl = [1, 2, 3, 6, 12]
    u1ml.multilevel(g, [4, 2], [1, 1], 1, 3, rl)
    _, c, _ = u1ml.measure(g, observables=False, correlator=True)
    th = u1ml.get_links(g)
    ref = np.array([plain_corr(th, 1)] + [multihit_corr(th, 1.0, r) for r in rl[1:]])
    tol = 1e-12 if prec == u1ml.FP64 else 2e-5
    assert abs(c[0] - ref[0]) < 1e-12
    assert np.abs(c[1:] - ref[1:]).max() <= tol * np.abs(ref[1:]).max()


@pytest.mark.parametrize("levels,n_sub,L,T,mh,general,prec", [
    ([4, 2], [2, 3], 4, 8, False, False, u1ml.FP64),
    ([4, 2], [2, 3], 4, 8, True, False, u1ml.FP64),
    ([4, 2], [2, 3], 4, 8, False, True, u1ml.FP64),
    ([2], [4], 6, 4, False, False, u1ml.FP64),
    ([4, 2], [2, 3], 6, 8, False, False, u1ml.FP32),
])
def test_field_squared_parity(oracle_mod, levels, n_sub, L, T, mh, general, prec):
    # squared components of Eq. (6) as the insertion, against the oracle; for
    # FP32 links the oracle starts from the same (FP32-rounded) links and only
    # the one-update identity below is exact, so here the chain must match
    r_list = [1, 2, 3]
    rf = [2, 3]
    say(f"[gpu] squared field parity levels={levels} L={L} mh={mh} general={general} prec={prec}")
    o = oracle_mod.OracleLattice(L, T, 1.2, 41, hot=True)
    g = u1ml.init_lattice(L, T, 1.2, 41, precision=prec)
    u1ml.set_estimator(g, multihit=mh, field_squared=True)
    if general:
        u1ml.set_debug(g, 2)
    if prec == u1ml.FP32:
        # the FP32 update differs from the FP64 chain; compare at one update
        # per level on the GPU's own links instead
        u1ml.multilevel(g, levels, [1] * len(levels), 1, 3, r_list, rf_list=rf)
        _, _, f_g = u1ml.measure(g, observables=False, correlator=False, field_profile=True)
        th = u1ml.get_links(g)
        for i, r in enumerate(rf):
            close_rel(f_g[i], field_identity(th, 1.2, r, squared=True), FIELD_REL[prec])
        return
    o.sweep(1, 3)
    u1ml.sweep(g, 1, 3)
    c_o, f_o, _ = o.multilevel(levels, n_sub, 1, 3, r_list, rf_list=rf, multihit=mh, field_squared=True)
    u1ml.multilevel(g, levels, n_sub, 1, 3, r_list, rf_list=rf)
    _, c_g, f_g = u1ml.measure(g, observables=False, correlator=True, field_profile=True)
    np.testing.assert_array_equal(u1ml.get_links(g), o.get_links())
    close_rel(c_g, c_o)
    close_rel(f_g, f_o)


@pytest.mark.parametrize("L,T,levels,n_sub,general", [
    (6, 8, [4, 2], [2, 2], False),
    (6, 8, [4, 2], [2, 2], True),
    (8, 4, [2], [3], False),
])
def test_field_profile_at_every_separation(oracle_mod, L, T, levels, n_sub, general):
    # E/B profiles for every r = 1 .. L - 1 in one run, against the oracle
    rf = list(range(1, L))
    say(f"[gpu] field at all r L={L} T={T} levels={levels} general={general}")
    o = oracle_mod.OracleLattice(L, T, 1.0, 71, hot=True)
    g = u1ml.init_lattice(L, T, 1.0, 71)
    if general:
        u1ml.set_debug(g, 2)
    c_o, f_o, _ = o.multilevel(levels, n_sub, 1, 2, rf, rf_list=rf)
    u1ml.multilevel(g, levels, n_sub, 1, 2, rf, rf_list=rf)
    _, c_g, f_g = u1ml.measure(g, observables=False, correlator=True, field_profile=True)
    np.testing.assert_array_equal(u1ml.get_links(g), o.get_links())
    close_rel(c_g, c_o)
    assert f_g.shape == (L - 1, 2, 6, L, L)
    for i in range(L - 1):
        close_rel(f_g[i], f_o[i])


def test_field_squared_batch_toggle_and_means(oracle_mod):
    # the flag switches between the Eq. (5) and Eq. (6) insertions in a batch;
    # the plain observables carry both lattice means
    Ls, seeds = [4, 6], [61, 62]
    say("[gpu] squared field batch toggle")
    b = u1ml.batch_create(Ls, [8, 8], [0.9, 0.9], seeds)
    ors = [oracle_mod.OracleLattice(L, 8, 0.9, s) for L, s in zip(Ls, seeds)]
    for sq in (True, False, True):
        u1ml.batch_set_estimator(b, field_squared=sq)
        u1ml.batch_multilevel(b, [4, 2], [2, 2], 1, 2, [1, 2, 3], rf_list=[3])
        for i, o in enumerate(ors):
            c_o, f_o, _ = o.multilevel([4, 2], [2, 2], 1, 2, [1, 2, 3], rf_list=[3], field_squared=sq)
            obs, c_g, f_g = u1ml.batch_measure(b, i, correlator=True, field_profile=True)
            np.testing.assert_array_equal(u1ml.batch_get_links(b, i), o.get_links())
            close_rel(c_g, c_o)
            close_rel(f_g, f_o)
            np.testing.assert_allclose(obs["field2_mean"], o.field2_means(), rtol=1e-13, atol=1e-15)
            np.testing.assert_allclose(obs["field_mean"], o.field_means(), atol=1e-14)


@pytest.mark.parametrize("prec", [u1ml.FP64, u1ml.FP32])
def test_field_squared_full_size_24_identity(prec):
    # 24^4, one update per level, squared insertion at r = 6 and 12: the
    # profile is the definition on the final links, and the squared means sum
    # to 6 beta (1 - plaquette)
    L = T = 24
    beta = 1.0
    say(f"[gpu] 24^4 squared field identity prec={prec}")
    g = u1ml.init_lattice(L, T, beta, 17, precision=prec)
    u1ml.set_estimator(g, field_squared=True)
    u1ml.sweep(g, 1, 3)
    rf = [6, 12]
    u1ml.multilevel(g, [4, 2], [1, 1], 1, 3, [1, 6, 12], rf_list=rf)
    obs, _, f = u1ml.measure(g, observables=True, correlator=False, field_profile=True)
    th = u1ml.get_links(g)
    for i, r in enumerate(rf):
        close_rel(f[i], field_identity(th, beta, r, squared=True), FIELD_REL[prec])
    # both sums are taken in FP64 from the stored links at either precision
    assert abs(sum(obs["field2_mean"]) - 6 * beta * (1 - obs["plaquette"])) < 1e-12


@pytest.mark.parametrize("levels,n_sub,L,T,mh,rf,debug", [
    ([4, 2], [2, 3], 4, 8, False, [2], 0),
    ([4, 2], [2, 3], 4, 8, True, [2, 3], 0),
    ([4, 2], [2, 3], 4, 8, True, [2, 3], 4),
    ([2], [4], 6, 4, False, [], 0),
    ([2], [4], 6, 4, False, [], 4),
    ([4, 2, 1], [2, 2, 2], 4, 8, False, [], 0),
    ([4, 2], [2, 2], 6, 8, False, [3], 2),
])
def test_symmetric_correlator_parity(oracle_mod, levels, n_sub, L, T, mh, rf, debug):
    # correlator averaged over +-x, +-y, +-z against the oracle's six
    # literal directions; debug 4 takes the per-site fold, 2 the general field
    r_list = [1, 2, 3]
    say(f"[gpu] symmetric correlator levels={levels} L={L} mh={mh} rf={rf} debug={debug}")
    o = oracle_mod.OracleLattice(L, T, 1.05, 91, hot=True)
    g = u1ml.init_lattice(L, T, 1.05, 91)
    u1ml.set_estimator(g, multihit=mh, symmetric=True)
    if debug:
        u1ml.set_debug(g, debug)
    o.sweep(1, 3)
    u1ml.sweep(g, 1, 3)
    c_o, f_o, _ = o.multilevel(levels, n_sub, 1, 3, r_list, rf_list=rf, multihit=mh, symmetric=True)
    u1ml.multilevel(g, levels, n_sub, 1, 3, r_list, rf_list=rf)
    _, c_g, f_g = u1ml.measure(g, observables=False, correlator=True, field_profile=bool(rf))
    np.testing.assert_array_equal(u1ml.get_links(g), o.get_links())
    assert np.all(c_g.imag == 0.0)
    close_rel(c_g.real, c_o.real)
    assert np.abs(c_o.imag).max() < 1e-15
    if rf:
        close_rel(f_g, f_o)


def test_symmetric_batch_and_one_update_identity(oracle_mod):
    # uneven batch (rows of different lengths in one fold launch), then the
    # one-update identity at 24^4 against numpy's six directions
    Ls, seeds = [4, 6, 8], [92, 93, 94]
    say("[gpu] symmetric batch vs oracle")
    b = u1ml.batch_create(Ls, [8, 8, 8], [1.0] * 3, seeds)
    u1ml.batch_set_estimator(b, symmetric=True)
    u1ml.batch_multilevel(b, [4, 2], [2, 2], 1, 2, [1, 2, 3])
    for i, (L, s) in enumerate(zip(Ls, seeds)):
        o = oracle_mod.OracleLattice(L, 8, 1.0, s)
        c_o, _, _ = o.multilevel([4, 2], [2, 2], 1, 2, [1, 2, 3], symmetric=True)
        _, c_g, _ = u1ml.batch_measure(b, i, correlator=True)
        np.testing.assert_array_equal(u1ml.batch_get_links(b, i), o.get_links())
        close_rel(c_g.real, c_o.real)
    from tests.test_oracle_multilevel import plain_corr_sym
    say("[gpu] symmetric one-update identity 24^4")
    g = u1ml.init_lattice(24, 24, 1.0, 95, start=u1ml.COLD)
    u1ml.set_estimator(g, symmetric=True)
    u1ml.sweep(g, 1, 3)
    rl = [1, 2, 5, 12]
    u1ml.multilevel(g, [4, 2], [1, 1], 1, 3, rl)
    _, c, _ = u1ml.measure(g, observables=False, correlator=True)
    th = u1ml.get_links(g)
    ref = np.array([plain_corr_sym(th, r) for r in rl])
    assert np.abs(c - ref.real).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("mh,sq,general,L", [
    (False, False, False, 4),
    (True, False, False, 4),
    (False, True, True, 6),
    (True, True, False, 6),
])
def test_replayed_field_run_matches_oracle(oracle_mod, mh, sq, general, L):
    # two passes over the same updates, one outer iteration of samples stored
    # at a time: links, pass ids and the accept log of the first pass equal
    # the oracle's, the correlator and field agree with its single pass
    T = 8
    r_list, rf = [1, 2, 3], [2, 3]
    say(f"[gpu] replayed field run mh={mh} sq={sq} general={general} L={L}")
    o = oracle_mod.OracleLattice(L, T, 1.0, 101, hot=True)
    g = u1ml.init_lattice(L, T, 1.0, 101)
    u1ml.set_estimator(g, multihit=mh, field_squared=sq)
    u1ml.set_debug(g, 1 | 8 | (2 if general else 0), 1 << 24)
    c_o, f_o, log_o = o.multilevel([4, 2], [3, 2], 1, 2, r_list, rf_list=rf, log_cap=1 << 24,
                                   multihit=mh, field_squared=sq)
    u1ml.multilevel(g, [4, 2], [3, 2], 1, 2, r_list, rf_list=rf)
    _, c_g, f_g = u1ml.measure(g, observables=False, correlator=True, field_profile=True)
    np.testing.assert_array_equal(u1ml.get_accept_log(g), log_o)
    np.testing.assert_array_equal(u1ml.get_links(g), o.get_links())
    assert u1ml.get_pass_id(g) == o.pass_id
    close_rel(c_g, c_o)
    close_rel(f_g, f_o)


def test_replayed_run_equals_stored_run_under_graph_replay():
    # the same chain with and without replay: identical links, pass ids and
    # correlator bits, field to rounding; the first call runs eagerly, the
    # later ones replay the captured graph
    say("[gpu] replay vs stored under graph replays")
    outs = []
    for flags in (0, 8):
        g = u1ml.init_lattice(6, 8, 1.1, 113)
        if flags:
            u1ml.set_debug(g, flags)
        runs = []
        for _ in range(3):  # first call eager, then graph replays
            u1ml.sweep(g, 1, 3)
            u1ml.multilevel(g, [4, 2], [2, 3], 1, 3, [1, 2, 3], rf_list=[2, 3])
            _, c, f = u1ml.measure(g, observables=False, correlator=True, field_profile=True)
            runs.append((u1ml.get_links(g), c, f, u1ml.get_pass_id(g)))
        outs.append(runs)
    for (l0, c0, f0, p0), (l1, c1, f1, p1) in zip(*outs):
        np.testing.assert_array_equal(l0, l1)
        np.testing.assert_array_equal(c0, c1)
        assert p0 == p1
        close_rel(f1, f0)


@pytest.mark.parametrize("L", [12, 24])
def test_fp32_fused_contraction_matches_general(L):
    # FP32 lattices keep the fused path's per-sample transforms in FP32 (the
    # transforms and sums stay FP64); the general path stores them in FP64.
    # Same chain, so the difference is the storage rounding alone.
    say(f"[gpu] FP32 fused vs general field contraction L={L}")
    res = []
    for general in (False, True):
        g = u1ml.init_lattice(L, 8, 1.0, 23, precision=u1ml.FP32)
        if general:
            u1ml.set_debug(g, 2)
        u1ml.sweep(g, 1, 2)
        u1ml.multilevel(g, [4, 2], [2, 3], 1, 2, [1, 2, 3, 4], rf_list=[2, 3, 4])
        _, c, f = u1ml.measure(g, observables=False, correlator=True, field_profile=True)
        res.append((u1ml.get_links(g), c, f))
    np.testing.assert_array_equal(res[0][0], res[1][0])
    np.testing.assert_array_equal(res[0][1], res[1][1])
    close_rel(res[0][2], res[1][2], 1e-6)


def test_field_size_and_separation_limits():
    # the most field separations a run takes (32: r = 1..32 at L = 40), fused
    # against general; 33 separations, and a field run at L = 64 (> 62), are
    # refused; at L = 62, the largest (62 is not a length of the fused path,
    # so the general contraction runs), one update per level makes the field
    # the plain Eq. (9) definition on the final links, computed here at
    # sampled offsets of both planes
    from tests.test_oracle_multilevel import field_ops, polyakov_lines

    say("[gpu] field limits: 32 separations at L=40, refusals, L=62 sampled")
    L, T = 40, 4
    rf = list(range(1, 33))
    res = []
    for general in (False, True):
        g = u1ml.init_lattice(L, T, 1.0, 31)
        if general:
            u1ml.set_debug(g, 2)
        u1ml.sweep(g, 1, 2)
        u1ml.multilevel(g, [2], [2], 1, 2, rf, rf_list=rf)
        _, c, f = u1ml.measure(g, observables=False, correlator=True, field_profile=True)
        res.append((c, f))
    np.testing.assert_array_equal(res[0][0], res[1][0])
    close_rel(res[0][1], res[1][1])
    with pytest.raises(u1ml.U1MLError) as e:
        u1ml.multilevel(g, [2], [1], 1, 1, list(range(1, 34)), rf_list=list(range(1, 34)))
    assert e.value.code == u1ml.EINVAL
    g64 = u1ml.init_lattice(64, 4, 1.0, 31)
    with pytest.raises(u1ml.U1MLError) as e:
        u1ml.multilevel(g64, [2], [1], 1, 1, [2], rf_list=[2])
    assert e.value.code == u1ml.EINVAL
    L, r = 62, 2
    g = u1ml.init_lattice(L, T, 1.0, 31)
    u1ml.sweep(g, 1, 3)
    u1ml.multilevel(g, [2], [1], 1, 3, [1, 2], rf_list=[r])
    _, c, f = u1ml.measure(g, observables=False, correlator=True, field_profile=True)
    th = u1ml.get_links(g)
    np.testing.assert_allclose(c, [plain_corr(th, k) for k in (1, 2)], atol=1e-12)
    P = polyakov_lines(th)
    w = np.conj(P) * np.roll(P, -r, axis=2)
    osum = field_ops(th, 1.0).sum(axis=1)  # [c][z][y][x]
    scale = np.abs(f[0]).max()
    for plane, m in enumerate([(r - 1) // 2, r // 2]):
        for dy, dz in [(0, 0), (1, 0), (0, 61), (30, 17), (61, 61)]:
            sh = np.roll(np.roll(np.roll(osum, -m, axis=3), -dy, axis=2), -dz, axis=1)
            want = (w[None] * sh).sum(axis=(1, 2, 3)) / (T * L ** 3)
            assert np.abs(f[0][plane, :, dy, dz] - want).max() <= 1e-12 * scale


@pytest.mark.parametrize("n_sub", [[2, 3], [10, 20]])
@pytest.mark.parametrize("prec_fold", ["rows", "rows_per_child", "general"])
def test_full_size_24_two_level_several_samples_match_oracle(oracle_mod, prec_fold, n_sub):
    # the benchmark's shape at 24^4 (levels {4, 2}, r = 1..12) with several
    # updates per level, so that every level average is over more than one
    # sample, up to the benchmark's own {10, 20} (the row fold then stages 20
    # samples of both children per row): FP64 links bit-identical to the
    # oracle and C_ML(r) to 1e-12, with the row-staged fold of the inner
    # averages (both children at once, or one at a time) and with the
    # per-site one
    L = T = 24
    r_list = list(range(1, 13))
    say(f"[gpu] 24^4 FP64 two-level {{4,2}} x {n_sub} r=1..12 vs oracle, fold={prec_fold}")
    o = oracle_mod.OracleLattice(L, T, 1.0, 31, hot=True)
    g = u1ml.init_lattice(L, T, 1.0, 31)
    if prec_fold == "general":
        u1ml.set_debug(g, 4)
    else:
        u1ml.set_tuning(g, fold_stage=2 if prec_fold == "rows_per_child" else 1)
    o.sweep(1, 3)
    u1ml.sweep(g, 1, 3)
    c_o, _, _ = o.multilevel([4, 2], n_sub, 1, 3, r_list)
    u1ml.multilevel(g, [4, 2], n_sub, 1, 3, r_list)
    obs, c_g, _ = u1ml.measure(g, correlator=True)
    np.testing.assert_array_equal(u1ml.get_links(g), o.get_links())
    np.testing.assert_allclose(c_g, c_o, rtol=1e-12, atol=0)
    assert abs(obs["plaquette"] - o.plaquette()) < 1e-13
    # the estimate is not the plain correlator of the final links (that is the
    # one-update identity); at r = 1 both are of the same order
    plain = o.plain_correlator([1])[0]
    assert abs(c_g[0] - plain) > 1e-6 * abs(plain)


@pytest.mark.parametrize("symmetric", [False, True])
def test_full_size_24_multihit_several_samples_match_oracle(oracle_mod, symmetric):
    # the benchmark's shape at 24^4 (levels {4, 2}, r = 1..12, so the row fold
    # takes six separations per thread and the multihit lines) with the
    # analytical multihit estimator, alone and with the correlator averaged
    # over +-x, +-y, +-z: FP64 links bit-identical to the oracle, C_ML(r) to
    # 1e-12 of its largest entry
    L = T = 24
    r_list = list(range(1, 13))
    say(f"[gpu] 24^4 FP64 two-level {{4,2}} x {{2,3}} multihit symmetric={symmetric} vs oracle")
    o = oracle_mod.OracleLattice(L, T, 1.0, 33, hot=True)
    g = u1ml.init_lattice(L, T, 1.0, 33)
    u1ml.set_estimator(g, multihit=True, symmetric=symmetric)
    o.sweep(1, 3)
    u1ml.sweep(g, 1, 3)
    c_o, _, _ = o.multilevel([4, 2], [2, 3], 1, 3, r_list, multihit=True, symmetric=symmetric)
    u1ml.multilevel(g, [4, 2], [2, 3], 1, 3, r_list)
    _, c_g, _ = u1ml.measure(g, observables=False, correlator=True)
    np.testing.assert_array_equal(u1ml.get_links(g), o.get_links())
    close_rel(c_g, c_o)


@pytest.mark.parametrize("multihit", [False, True])
def test_single_level_fold_modes_give_the_same_bits(oracle_mod, multihit):
    # the single-level run of the uneven batch at its largest size (24^4,
    # slabs of 2, 10 updates, r = 1..12): the row fold's parent slab is the
    # whole lattice, with 12 children of 10 samples (46 KB of rows, 92 KB
    # with the multihit lines, which only the per-child staging holds).  The
    # fold staging all children at once, one child at a time (the default
    # here) and the per-site fold give the same bits, and the oracle's
    # C_ML(r) to 1e-12 (cold start and two sweeps, so that C_ML(r) is of
    # order 1e-4 to 1e-3 at every r).
    L = T = 24
    r_list = list(range(1, 13))
    runs = []
    for mode in ("auto", "all", "per_child", "general"):
        say(f"[gpu] 24^4 FP64 single level [2] x [10] r=1..12 multihit={multihit} fold={mode}")
        g = u1ml.init_lattice(L, T, 1.0, 41, start=u1ml.COLD)
        u1ml.set_estimator(g, multihit=multihit)
        if mode == "general":
            u1ml.set_debug(g, 4)
        elif mode != "auto":
            u1ml.set_tuning(g, fold_stage=1 if mode == "all" else 2)
        for _ in range(2):
            u1ml.sweep(g, 1, 3)
        u1ml.multilevel(g, [2], [10], 1, 3, r_list)
        _, c, _ = u1ml.measure(g, observables=False, correlator=True)
        runs.append((u1ml.get_links(g), c))
    for th, c in runs[1:]:
        np.testing.assert_array_equal(th, runs[0][0])
        np.testing.assert_array_equal(c, runs[0][1])
    o = oracle_mod.OracleLattice(L, T, 1.0, 41, hot=False)
    for _ in range(2):
        o.sweep(1, 3)
    c_o, _, _ = o.multilevel([2], [10], 1, 3, r_list, multihit=multihit)
    np.testing.assert_array_equal(runs[0][0], o.get_links())
    np.testing.assert_allclose(runs[0][1], c_o, rtol=1e-12, atol=0)


@pytest.mark.parametrize("multihit", [False, True])
def test_single_level_fold_with_long_rows(oracle_mod, multihit):
    # 24^3 x 8, slabs of 2, 40 updates per slab, r = 1..12: one child's rows
    # take 15 KB (30 KB with the multihit lines) and all four children more
    # than the 48 KB a block stages, so the fold goes child by child; the
    # plain run prefetches the next child's rows with 256 threads for 48
    # items, the multihit run (two buffers would take 60 KB) stages each
    # child in turn.  Same bits as the per-site fold, C_ML(r) to 1e-12 of
    # the oracle's.
    L, T = 24, 8
    r_list = list(range(1, 13))
    runs = []
    for mode in ("auto", "general"):
        say(f"[gpu] 24^3x8 FP64 single level [2] x [40] r=1..12 multihit={multihit} fold={mode}")
        g = u1ml.init_lattice(L, T, 1.0, 43, start=u1ml.COLD)
        u1ml.set_estimator(g, multihit=multihit)
        if mode == "general":
            u1ml.set_debug(g, 4)
        for _ in range(2):
            u1ml.sweep(g, 1, 3)
        u1ml.multilevel(g, [2], [40], 1, 3, r_list)
        _, c, _ = u1ml.measure(g, observables=False, correlator=True)
        runs.append((u1ml.get_links(g), c))
    np.testing.assert_array_equal(runs[1][0], runs[0][0])
    np.testing.assert_array_equal(runs[1][1], runs[0][1])
    o = oracle_mod.OracleLattice(L, T, 1.0, 43, hot=False)
    for _ in range(2):
        o.sweep(1, 3)
    c_o, _, _ = o.multilevel([2], [40], 1, 3, r_list, multihit=multihit)
    np.testing.assert_array_equal(runs[0][0], o.get_links())
    np.testing.assert_allclose(runs[0][1], c_o, rtol=1e-12, atol=0)


def test_batch_fold_mixes_staging_paths(oracle_mod):
    # one fold launch over a 4^3 x 8 and a 24^3 x 8 lattice with the multihit
    # lines, slabs of 2 and 40 updates: the 24^3 rows of a child (30 KB) are
    # staged child by child, while the 4^3 blocks hold theirs twice over and
    # prefetch the next child; both lattices against the oracle (links
    # bit-identical, C_ML(r) to 1e-12)
    Ls, seeds = [4, 24], [44, 45]
    r_list = [1, 2, 3]
    say("[gpu] batch 4^3x8 + 24^3x8 FP64 single level [2] x [40] multihit vs oracle")
    b = u1ml.batch_create(Ls, [8, 8], [1.0, 1.0], seeds, start=u1ml.COLD)
    u1ml.batch_set_estimator(b, multihit=True)
    for _ in range(2):
        u1ml.batch_sweep(b, 1, 3)
    u1ml.batch_multilevel(b, [2], [40], 1, 3, r_list)
    for i, (L, s) in enumerate(zip(Ls, seeds)):
        o = oracle_mod.OracleLattice(L, 8, 1.0, s, hot=False)
        for _ in range(2):
            o.sweep(1, 3)
        c_o, _, _ = o.multilevel([2], [40], 1, 3, r_list, multihit=True)
        _, c_g, _ = u1ml.batch_measure(b, i, correlator=True)
        np.testing.assert_array_equal(u1ml.batch_get_links(b, i), o.get_links())
        np.testing.assert_allclose(c_g, c_o, rtol=1e-12, atol=0)


def test_full_size_48_two_level_several_samples_match_oracle(oracle_mod):
    # the large configuration's lattice, 48^4 FP64 (one lattice, the
    # single-lattice class passes), a two-level run {4,2} x {2,2} with
    # r = 1..24 (four groups of six separations per row): the three fold
    # modes give the same bits, the links are the oracle's and C_ML(r) is to
    # 1e-12
    L = T = 48
    r_list = list(range(1, 25))
    runs = []
    for mode in ("all", "per_child", "general"):
        say(f"[gpu] 48^4 FP64 two-level {{4,2}} x {{2,2}} r=1..24 fold={mode}")
        g = u1ml.init_lattice(L, T, 1.0, 73)
        if mode == "general":
            u1ml.set_debug(g, 4)
        else:
            u1ml.set_tuning(g, fold_stage=1 if mode == "all" else 2)
        u1ml.sweep(g, 1, 3)
        u1ml.multilevel(g, [4, 2], [2, 2], 1, 3, r_list)
        _, c, _ = u1ml.measure(g, observables=False, correlator=True)
        runs.append((u1ml.get_links(g), c))
        del g
    for th, c in runs[1:]:
        np.testing.assert_array_equal(th, runs[0][0])
        np.testing.assert_array_equal(c, runs[0][1])
    say("  oracle 48^4")
    o = oracle_mod.OracleLattice(L, T, 1.0, 73, hot=True)
    o.sweep(1, 3)
    c_o, _, _ = o.multilevel([4, 2], [2, 2], 1, 3, r_list)
    np.testing.assert_array_equal(runs[0][0], o.get_links())
    np.testing.assert_allclose(runs[0][1], c_o, rtol=1e-12, atol=0)


@pytest.mark.parametrize("L,T,levels,n_sub,rf", [
    (12, 12, [6, 2], [2, 2], [3, 6]),
    (16, 8, [4, 2], [2, 3], [2, 4]),
])
def test_field_with_several_samples_at_larger_sizes(oracle_mod, L, T, levels, n_sub, rf):
    # the fused contraction at sizes with several transform blocks per plane
    # set and lengths 12 (radices 4, 3) and 16 (4, 4), three children per top
    # slab or two top slabs, several updates per level: the correlator
    # (r = 1..L/2) and the E/B profiles against the oracle
    r_list = list(range(1, L // 2 + 1))
    say(f"[gpu] field with several samples L={L} T={T} levels={levels} n_sub={n_sub} rf={rf}")
    o = oracle_mod.OracleLattice(L, T, 1.0, 77, hot=True)
    g = u1ml.init_lattice(L, T, 1.0, 77)
    o.sweep(1, 3)
    u1ml.sweep(g, 1, 3)
    c_o, f_o, _ = o.multilevel(levels, n_sub, 1, 3, r_list, rf_list=rf)
    u1ml.multilevel(g, levels, n_sub, 1, 3, r_list, rf_list=rf)
    _, c_g, f_g = u1ml.measure(g, observables=False, correlator=True, field_profile=True)
    np.testing.assert_array_equal(u1ml.get_links(g), o.get_links())
    np.testing.assert_allclose(c_g, c_o, rtol=1e-12, atol=0)
    close_rel(f_g, f_o)


@pytest.mark.parametrize("multihit", [False, True])
def test_fold_stagings_with_the_symmetric_correlator(oracle_mod, multihit):
    # rows along y and z (strided by L and L^2) staged all at once and one
    # child slab at a time: same bits, and the oracle's six literal
    # directions to 1e-12 of the largest entry (12^4, slabs of 2, 10 updates)
    L = T = 12
    r_list = [1, 2, 3, 5]
    runs = []
    for stage in (1, 2):
        say(f"[gpu] symmetric correlator 12^4 [2] x [10] multihit={multihit} fold_stage={stage}")
        g = u1ml.init_lattice(L, T, 1.0, 79, start=u1ml.COLD)
        u1ml.set_estimator(g, multihit=multihit, symmetric=True)
        u1ml.set_tuning(g, fold_stage=stage)
        for _ in range(2):
            u1ml.sweep(g, 1, 3)
        u1ml.multilevel(g, [2], [10], 1, 3, r_list)
        _, c, _ = u1ml.measure(g, observables=False, correlator=True)
        runs.append((u1ml.get_links(g), c))
    np.testing.assert_array_equal(runs[1][0], runs[0][0])
    np.testing.assert_array_equal(runs[1][1], runs[0][1])
    o = oracle_mod.OracleLattice(L, T, 1.0, 79, hot=False)
    for _ in range(2):
        o.sweep(1, 3)
    c_o, _, _ = o.multilevel([2], [10], 1, 3, r_list, multihit=multihit, symmetric=True)
    np.testing.assert_array_equal(runs[0][0], o.get_links())
    close_rel(runs[0][1].real, c_o.real)
