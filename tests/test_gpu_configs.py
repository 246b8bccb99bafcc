"""The full-size workloads: 64 batched instances of uneven size and coupling
(sweeps + one-level multilevel in captured cycles), and the 48^4 lattice with
the two-level multilevel and the field profiles."""
import math
import sys

import numpy as np
import pytest

from paper_1208_0166_amd import u1ml
from tests.test_oracle_multilevel import field_ops, plain_corr, polyakov_lines

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def uneven_instances(n=64, seed=7):
    rng = np.random.default_rng(seed)
    Ls = [int(v) for v in rng.choice([8, 12, 16, 20, 24], n)]
    betas = [float(v) for v in rng.choice([0.9, 1.0, 1.1], n)]
    return Ls, betas, [1000 + i for i in range(n)]


def test_64_uneven_instances_fp32_cycles():
    Ls, betas, seeds = uneven_instances()
    say(f"[gpu] 64 instances, L counts {dict(zip(*np.unique(Ls, return_counts=True)))}")
    b = u1ml.batch_create(Ls, Ls, betas, seeds, start=u1ml.COLD, precision=u1ml.FP32)
    for _ in range(20):
        u1ml.batch_sweep(b, 1, 3)
    # one update per level: the multilevel correlator is the plain one of the final links
    u1ml.batch_cycle(b, 2, 1, 3, 2, 1, use_graph=True)
    for i in range(64):
        th = u1ml.batch_get_links(b, i)
        _, c, _ = u1ml.batch_measure(b, i)
        ref = [plain_corr(th, r) for r in range(1, Ls[i] // 2 + 1)]
        np.testing.assert_allclose(c, ref, rtol=0, atol=1e-12)
    # the configured cycle (th 2, 10 updates), captured and replayed
    for _ in range(3):
        u1ml.batch_cycle(b, 2, 1, 3, 2, 10, use_graph=True)
    for i in range(64):
        obs, c, _ = u1ml.batch_measure(b, i)
        assert np.all(np.isfinite(c)) and np.all(np.abs(c) <= 1.0)
        assert 0.3 < obs["plaquette"] < 0.8


def test_64_uneven_instances_fp64_match_oracle(oracle_mod):
    # the FP64 twin of the uneven batch: the same 64 sizes and couplings in one
    # batch, hot start, one sweep, then two measurement cycles (one sweep plus
    # the single-level multilevel with slabs of 2 and 10 updates, r = 1..L/2),
    # the second replayed from the captured graph.  Every lattice is followed
    # by the oracle through the same sequence: links bit-identical and C_ML(r)
    # to 1e-12.
    Ls, betas, seeds = uneven_instances()
    say("[gpu] 64 instances FP64 vs oracle, every lattice")
    b = u1ml.batch_create(Ls, Ls, betas, seeds, start=u1ml.HOT, precision=u1ml.FP64)
    u1ml.batch_sweep(b, 1, 3)
    u1ml.batch_cycle(b, 1, 1, 3, 2, 10, use_graph=True)
    u1ml.batch_cycle(b, 1, 1, 3, 2, 10, use_graph=True)
    assert sorted(set(Ls)) == [8, 12, 16, 20, 24] and len({(L, be) for L, be in zip(Ls, betas)}) == 15
    for i, (L, be) in enumerate(zip(Ls, betas)):
        say(f"  lattice {i}: L={L} beta={be}")
        o = oracle_mod.OracleLattice(L, L, be, seeds[i], hot=True)
        o.sweep(1, 3)
        for _ in range(2):
            o.sweep(1, 3)
            c_o, _, _ = o.multilevel([2], [10], 1, 3, list(range(1, L // 2 + 1)))
        obs, c_g, _ = u1ml.batch_measure(b, i)
        np.testing.assert_array_equal(u1ml.batch_get_links(b, i), o.get_links())
        np.testing.assert_allclose(c_g, c_o, rtol=1e-12, atol=1e-15)
        assert abs(obs["plaquette"] - o.plaquette()) < 1e-13


def field_points(th, beta, r, points):
    """Plain Eq. (9) definition at one update per level for the listed
    (plane, dy, dz): (1/V) sum_{x0,t} P*(x0) P(x0 + r) O_c(x0 + m + dy + dz, t)."""
    T, L = th.shape[0], th.shape[1]
    P = polyakov_lines(th)
    w = np.conj(P) * np.roll(P, -r, axis=2)
    Osum = field_ops(th, beta).sum(axis=1)  # [c][z][y][x]
    out = []
    for plane, dy, dz in points:
        m = (r - 1) // 2 if plane == 0 else r // 2
        sh = np.roll(np.roll(np.roll(Osum, -m, axis=3), -dy, axis=2), -dz, axis=1)
        out.append((w[None] * sh).sum(axis=(1, 2, 3)) / (T * L ** 3))
    return np.array(out)  # [point][c]


def test_large_48_identity_fp32():
    L = T = 48
    say("[gpu] 48^4 FP32 two-level identity with field")
    g = u1ml.init_lattice(L, T, 1.0, 5, precision=u1ml.FP32, start=u1ml.COLD)
    for _ in range(3):
        u1ml.sweep(g, 1, 3)
    rl = list(range(1, 25))
    u1ml.multilevel(g, [4, 2], [1, 1], 1, 3, rl, rf_list=[2, 4, 6])
    obs, c, f = u1ml.measure(g, correlator=True, field_profile=True)
    th = u1ml.get_links(g)
    np.testing.assert_allclose(c, [plain_corr(th, r) for r in rl], rtol=0, atol=1e-12)
    rng = np.random.default_rng(11)
    points = [(int(p), int(a), int(b)) for p, a, b in zip(rng.integers(0, 2, 12), rng.integers(0, L, 12),
                                                       rng.integers(0, L, 12))]
    points += [(0, 0, 0), (1, 0, 0)]
    scale = np.abs(f).max()
    for k, r in enumerate([2, 4, 6]):
        ref = field_points(th, 1.0, r, points)
        got = np.array([f[k, p, :, dy, dz] for p, dy, dz in points])
        assert np.abs(got - ref).max() <= 2e-5 * scale, (r, np.abs(got - ref).max(), scale)
    assert math.isfinite(obs["plaquette"])


def test_bench_batch_shape_identity_fp32():
    # the benchmark's launch configuration: a batch of 16 24^4 FP32 lattices
    # (one of its three batches) with its tuned shapes (class pass 256
    # threads, XCD-contiguous; transforms of 4 planes per block; contraction
    # 128 threads) through the two-level run
    # with the field at r = 2, 4, 6, one update per level: every lattice's
    # C_ML(r), r = 1..12, equals the plain correlator of its final links and
    # its field the plain Eq. (9) definition at sampled offsets
    L = T = 24
    n = 16
    say(f"[gpu] batch of {n} x 24^4 FP32 with the bench's shapes, one-update identity")
    b = u1ml.batch_create([L] * n, [T] * n, [1.0] * n, [61 + i for i in range(n)], precision=u1ml.FP32,
                          start=u1ml.COLD)
    u1ml.set_tuning(b, pass_block=256, pass_xcd_map=1, sample_block=256, fold_threads=64, field_w_planes=4,
                    field_o_planes=4, field_zcon_threads=128)
    for _ in range(3):
        u1ml.batch_sweep(b, 1, 3)
    rl = list(range(1, 13))
    u1ml.batch_multilevel(b, [4, 2], [1, 1], 1, 3, rl, rf_list=[2, 4, 6])
    rng = np.random.default_rng(12)
    points = [(int(p), int(a), int(c)) for p, a, c in zip(rng.integers(0, 2, 8), rng.integers(0, L, 8),
                                                       rng.integers(0, L, 8))]
    points += [(0, 0, 0), (1, 0, 0)]
    for i in range(n):
        _, c, f = u1ml.batch_measure(b, i, correlator=True, field_profile=True)
        th = u1ml.batch_get_links(b, i)
        np.testing.assert_allclose(c, [plain_corr(th, r) for r in rl], rtol=0, atol=1e-12)
        scale = np.abs(f).max()
        for k, r in enumerate([2, 4, 6]):
            ref = field_points(th, 1.0, r, points)
            got = np.array([f[k, p, :, dy, dz] for p, dy, dz in points])
            assert np.abs(got - ref).max() <= 2e-5 * scale, (i, r, np.abs(got - ref).max(), scale)
    b.close()


def test_64_uneven_instances_fp32_agree_with_fp64_statistically():
    # the batched FP32 form against its FP64 twin: both batches of the 64 sizes
    # and couplings from a cold start, 200 sweeps, then 20 captured cycles (2
    # sweeps + single-level multilevel, slabs of 2, 10 updates, r = 1..L/2).
    # Lattice i of one batch and lattice i of the other are independent chains
    # of the same law, so their difference d_i of the cycle averages (plaquette,
    # Re C(1)) has mean zero.  Per (L, beta) group a t-test on the d_i (their
    # spread gives the error), and Fisher's combination of the group p-values
    # over all groups must not reject at 1e-3.
    from scipy import stats
    Ls, betas, seeds = uneven_instances()
    say("[gpu] 64 instances FP32 vs FP64, 20 cycles each")
    avg = {}
    for prec in (u1ml.FP32, u1ml.FP64):
        b = u1ml.batch_create(Ls, Ls, betas, seeds, start=u1ml.COLD, precision=prec)
        for _ in range(200):
            u1ml.batch_sweep(b, 1, 3)
        acc = np.zeros((64, 2))
        for _ in range(20):
            u1ml.batch_cycle(b, 2, 1, 3, 2, 10, use_graph=True)
            for i in range(64):
                obs, c, _ = u1ml.batch_measure(b, i)
                acc[i] += [obs["plaquette"], c[0].real]
        avg[prec] = acc / 20
        b.close()
    d = avg[u1ml.FP32] - avg[u1ml.FP64]
    groups = {}
    for i, key in enumerate(zip(Ls, betas)):
        groups.setdefault(key, []).append(i)
    for j, name in enumerate(("plaquette", "C(1)")):
        pvals = []
        for key, idx in sorted(groups.items()):
            if len(idx) < 2:
                continue
            x = d[idx, j]
            t = x.mean() / (x.std(ddof=1) / np.sqrt(len(x)))
            pvals.append(2 * stats.t.sf(abs(t), len(x) - 1))
        chi2 = -2 * np.sum(np.log(pvals))
        p = stats.chi2.sf(chi2, 2 * len(pvals))
        say(f"  {name}: {len(pvals)} groups, Fisher chi2 {chi2:.1f} on {2 * len(pvals)} dof, p = {p:.3f}; "
            f"mean |relative deviation| {np.mean(np.abs(d[:, j] / avg[u1ml.FP64][:, j])):.2e}")
        assert p > 1e-3, (name, p)
