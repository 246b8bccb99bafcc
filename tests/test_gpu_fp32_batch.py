"""FP32 update path (statistical agreement with FP64) and batched lattices
(bit-exact against the oracle, graph replay against eager launches)."""
import math
import sys

import numpy as np
import pytest

from paper_1208_0166_amd import u1ml

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def binned_mean_err(x, nb=10):
    x = np.asarray(x)
    n = len(x) // nb
    m = x[: n * nb].reshape(nb, n).mean(axis=1)
    return m.mean(), m.std(ddof=1) / math.sqrt(nb)


def test_fp32_agrees_with_fp64_statistically():
    # 8^4 at beta = 1: plaquette and |P| from FP32 and FP64 chains within 3 sigma
    L = T = 8
    res = {}
    for prec in (u1ml.FP64, u1ml.FP32):
        say(f"[gpu] chain prec={prec}")
        g = u1ml.init_lattice(L, T, 1.0, 100 + prec, precision=prec)
        for _ in range(100):
            u1ml.sweep(g, 1, 3)
        pl = []
        for _ in range(400):
            u1ml.sweep(g, 1, 3)
            obs, _, _ = u1ml.measure(g)
            pl.append(obs["plaquette"])
        res[prec] = binned_mean_err(pl)
    (m64, e64), (m32, e32) = res[u1ml.FP64], res[u1ml.FP32]
    dev = abs(m64 - m32) / math.hypot(e64, e32)
    say(f"plaquette fp64 {m64:.6f}({e64:.6f}) fp32 {m32:.6f}({e32:.6f}) dev {dev:.2f} sigma")
    assert dev < 3.0
    assert 0.5 < m64 < 0.7


def test_batch_matches_oracle_bit_exact(oracle_mod):
    Ls = [4, 6, 8, 4]
    betas = [0.9, 1.0, 1.1, 1.0]
    seeds = [1000, 1001, 1002, 1003]
    say("[gpu] batch sweeps vs oracle")
    b = u1ml.batch_create(Ls, Ls, betas, seeds, precision=u1ml.FP64)
    ors = [oracle_mod.OracleLattice(L, L, be, s, hot=True) for L, be, s in zip(Ls, betas, seeds)]
    for _ in range(3):
        u1ml.batch_sweep(b, 1, 3)
        for o in ors:
            o.sweep(1, 3)
    for i, o in enumerate(ors):
        np.testing.assert_array_equal(u1ml.batch_get_links(b, i), o.get_links())
    # one measurement cycle: 2 sweeps + one-level multilevel (th 2, 4 updates), r = 1..L/2
    u1ml.batch_cycle(b, 2, 1, 3, 2, 4, use_graph=False)
    for i, o in enumerate(ors):
        for _ in range(2):
            o.sweep(1, 3)
        c_o, _, _ = o.multilevel([2], [4], 1, 3, list(range(1, Ls[i] // 2 + 1)))
        obs, c_g, _ = u1ml.batch_measure(b, i)
        np.testing.assert_array_equal(u1ml.batch_get_links(b, i), o.get_links())
        np.testing.assert_allclose(c_g, c_o, rtol=1e-12, atol=1e-15)
        assert abs(obs["plaquette"] - o.plaquette()) < 1e-13


@pytest.mark.parametrize("prec", [u1ml.FP64, u1ml.FP32])
def test_batch_graph_replay_matches_eager(prec):
    Ls = [8, 12, 8, 16]
    betas = [0.9, 1.0, 1.1, 1.0]
    seeds = [7, 8, 9, 10]
    say(f"[gpu] graph vs eager prec={prec}")
    a = u1ml.batch_create(Ls, Ls, betas, seeds, precision=prec)
    e = u1ml.batch_create(Ls, Ls, betas, seeds, precision=prec, graphs=False)
    for k in range(4):
        u1ml.batch_cycle(a, 2, 1, 3, 2, 3, use_graph=True)
        u1ml.batch_cycle(e, 2, 1, 3, 2, 3, use_graph=False)
        for i in range(len(Ls)):
            np.testing.assert_array_equal(u1ml.batch_get_links(a, i), u1ml.batch_get_links(e, i))
            _, ca, _ = u1ml.batch_measure(a, i)
            _, ce, _ = u1ml.batch_measure(e, i)
            np.testing.assert_array_equal(ca, ce)


def test_autotune_keeps_links_and_results():
    g = u1ml.init_lattice(8, 8, 1.0, 4)
    th = u1ml.get_links(g)
    best = u1ml.autotune(g)
    assert best in (64, 128, 256, 512, 1024)
    np.testing.assert_array_equal(u1ml.get_links(g), th)
    assert u1ml.get_pass_id(g) == 0


def test_fp32_metropolis_draws_philox4x32():
    # beta = 0 accepts every proposal, so theta' = eps (2 u1 - 1) from a cold
    # start exposes u1 of every link: it must be the Philox4x32-10 word 0 of
    # counter (n, 2<<16 | hit<<8 | mu, pass_id, 0) under key (seed lo, seed hi)
    from tests.philox_ref import philox4x32_10
    L, T, eps, seed = 4, 6, 0.5, (7 << 32) | 3
    g = u1ml.init_lattice(L, T, 0.0, seed, precision=u1ml.FP32, start=u1ml.COLD, eps=eps)
    u1ml.set_pass_id(g, 5)
    u1ml.sweep(g, 1, 0)
    th = u1ml.get_links(g).reshape(-1, 4)
    n = np.arange(L ** 3 * T, dtype=np.uint64)
    for mu in range(4):
        w = philox4x32_10(n, (2 << 16) | mu, 5, 0, seed & 0xFFFFFFFF, seed >> 32)
        u1 = (w[0] >> np.uint64(8)).astype(np.float32) * np.float32(2.0 ** -24)
        expect = np.float32(eps) * (np.float32(2) * u1 - np.float32(1))
        np.testing.assert_array_equal(th[:, mu].astype(np.float32), expect)
