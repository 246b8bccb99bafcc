"""The largest lattice the library accepts: L = T = 84, where V L = 4.18e9 lies
just below the 2^32 bound of the kernels' 32-bit site arithmetic (86^4 and
86^3 x 84 are refused, tests/test_abi_cpu.py).  From a hot start, one FP64
compound sweep gives the oracle's links bit for bit (Sec. 2.1); the FP32 path
starts from the same angles to FP32 rounding and, after its own sweep, has the
FP64 chain's plaquette to within the fluctuation of a 5e7-site average; and a
single-level multilevel run with one update per slab reproduces the plain
correlator of its final configuration (the slab updates are disjoint,
Sec. 2.2), through the row fold staging one child slab at a time (42 slabs
of 84 sites exceed what one block stages at once)."""
import sys

import numpy as np
import pytest

from paper_1208_0166_amd import u1ml

pytestmark = pytest.mark.gpu

L = T = 84


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_largest_lattice_fp64_sweep_bit_exact(oracle_mod):
    say(f"[gpu] {L}^4 FP64 hot start seed 77 and one compound sweep")
    o = oracle_mod.OracleLattice(L, T, 1.0, 77, hot=True)
    g = u1ml.init_lattice(L, T, 1.0, 77, precision=u1ml.FP64)
    np.testing.assert_array_equal(u1ml.get_links(g), o.get_links())
    u1ml.sweep(g, 1, 3)
    o.sweep(1, 3)
    np.testing.assert_array_equal(u1ml.get_links(g), o.get_links())
    obs, _, _ = u1ml.measure(g)
    assert abs(obs["plaquette"] - o.plaquette()) < 1e-12
    r = [1, 2, 42, 83]
    ref = o.plain_correlator(r)
    np.testing.assert_allclose(u1ml.plain_correlator(g, r), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    say("  one-update single-level multilevel, r = 1, 2, 42, 83")
    u1ml.multilevel(g, [2], [1], 1, 3, r)
    _, c, _ = u1ml.measure(g, correlator=True)
    plain = u1ml.plain_correlator(g, r)
    np.testing.assert_allclose(c, plain, rtol=0, atol=1e-12 * np.abs(plain).max())
    g.close()


def test_largest_lattice_fp32_path(oracle_mod):
    say(f"[gpu] {L}^4 FP32 and FP64 hot start seed 78, one compound sweep each")
    o = oracle_mod.OracleLattice(L, T, 1.0, 78, hot=True)
    g32 = u1ml.init_lattice(L, T, 1.0, 78, precision=u1ml.FP32)
    assert np.abs(u1ml.get_links(g32) - o.get_links()).max() < 4e-7
    del o
    g64 = u1ml.init_lattice(L, T, 1.0, 78, precision=u1ml.FP64)
    u1ml.sweep(g32, 1, 3)
    u1ml.sweep(g64, 1, 3)
    p32 = u1ml.measure(g32)[0]["plaquette"]
    p64 = u1ml.measure(g64)[0]["plaquette"]
    say(f"  plaquette FP32 {p32:.6f} FP64 {p64:.6f}")
    # two chains of one distribution (their own random numbers): the
    # plaquette over 3e8 plaquettes fluctuates by ~1e-4 after one sweep
    assert 0.05 < p64 < 0.6 and abs(p32 - p64) < 1e-3
    g32.close()
    g64.close()
