"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function the header declares, and rejects bad arguments before touching
the device."""
import ctypes as C
import os

import pytest

from paper_1208_0166_amd import u1ml

pytestmark = pytest.mark.skipif(not os.path.exists(u1ml.LIB_PATH), reason="libu1ml.so not built")


def test_every_declared_function_is_exported():
    lib = u1ml.load_library()
    names = u1ml.header_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []


def test_link_bytes_and_defaults():
    assert u1ml.link_bytes(24, 24, u1ml.FP64) == 4 * 24 ** 4 * 8
    assert u1ml.link_bytes(24, 24, u1ml.FP32) == 4 * 24 ** 4 * 4
    assert u1ml.link_bytes(3, 4, u1ml.FP64) == 0
    assert u1ml.link_bytes(4, 4, 7) == 0
    o = u1ml.default_options()
    assert (o.start, o.precision, o.eps, o.block) == (u1ml.HOT, u1ml.FP64, 1.0, 0)


def test_strerror_codes():
    lib = u1ml.load_library()
    for code in (0, -1, -2, -3, -4, -5, -99):
        assert lib.u1ml_strerror(code)


@pytest.mark.parametrize("L,T,beta,prec,eps,block", [
    (3, 4, 1.0, 0, 1.0, 0),      # odd L
    (4, 2 * 200, 1.0, 0, 1.0, 0),  # T too large
    (0, 4, 1.0, 0, 1.0, 0),
    (4, 4, -1.0, 0, 1.0, 0),     # negative beta
    (4, 4, float("nan"), 0, 1.0, 0),
    (4, 4, 1.0, 5, 1.0, 0),      # precision
    (4, 4, 1.0, 0, -1.0, 0),     # eps
    (4, 4, 1.0, 0, 6.3, 0),      # eps above 2 pi
    (4, 4, 1.0, 1, 1e20, 0),     # huge eps (the proposal's fold into [-pi, pi) would not end)
    (4, 4, 1.0, 0, float("inf"), 0),
    (4, 4, 1.0, 0, float("nan"), 0),
    (4, 4, 1.0, 0, 1.0, 100),    # block not a multiple of 64
    (86, 86, 1.0, 1, 1.0, 0),    # V L = 4.7e9: beyond the kernels' 32-bit site arithmetic
    (86, 84, 1.0, 0, 1.0, 0),    # V L = 4.6e9
])
def test_init_rejects_bad_arguments(L, T, beta, prec, eps, block):
    lib = u1ml.load_library()
    o = u1ml.default_options()
    o.precision, o.eps, o.block = prec, eps, block
    h = C.c_void_p()
    assert lib.u1ml_init_lattice(L, T, beta, 1, C.byref(o), C.byref(h)) == u1ml.EINVAL
    assert not h.value
    assert lib.u1ml_last_error()


def test_null_handles_rejected():
    lib = u1ml.load_library()
    assert lib.u1ml_sweep(None, 1, 3) == u1ml.EINVAL
    assert lib.u1ml_measure(None, None, None, None) == u1ml.EINVAL
    assert lib.u1ml_ensemble_reset(None) == u1ml.EINVAL
    assert lib.u1ml_ensemble_add(None) == u1ml.EINVAL
    assert lib.u1ml_ensemble_info(None, None, None, None) == u1ml.EINVAL
    assert lib.u1ml_ensemble_read(None, None, None, None) == u1ml.EINVAL
    assert lib.u1ml_batch_ensemble_add(None) == u1ml.EINVAL
    assert lib.u1ml_batch_ensemble_read(None, 0, None, None, None) == u1ml.EINVAL
    assert lib.u1ml_init_lattice(4, 4, 1.0, 1, None, None) == u1ml.EINVAL
    assert lib.u1ml_batch_save(None, b"x") == u1ml.EINVAL
    assert lib.u1ml_batch_load(None, b"x") == u1ml.EINVAL
    pid = C.c_uint64()
    assert lib.u1ml_batch_get_pass_id(None, 0, C.byref(pid)) == u1ml.EINVAL
    assert lib.u1ml_batch_set_pass_id(None, 0, 1) == u1ml.EINVAL
    # an empty batch is refused before any device call
    one_i, one_d, one_u = (C.c_int * 1)(8), (C.c_double * 1)(1.0), (C.c_uint64 * 1)(1)
    bp = C.c_void_p()
    assert lib.u1ml_batch_create(0, one_i, one_i, one_d, one_u, None, C.byref(bp)) == u1ml.EINVAL
    assert not bp.value
    lib.u1ml_destroy(None)
    lib.u1ml_batch_destroy(None)


def test_workspace_bytes_is_a_pure_size_function():
    wb = u1ml.workspace_bytes
    assert wb(3, 8, [4, 2], [2, 3], 3) == 0            # odd L
    assert wb(4, 8, [3], [2], 3) == 0                  # slab does not divide T
    assert wb(4, 8, [4, 2, 1], [1, 1, 1], 3, n_rf=2) == 0  # field with three levels
    base = wb(4, 8, [4, 2], [2, 3], 3)
    assert base > 0
    # multihit doubles the stored lines; the symmetric correlator triples the
    # accumulators; the field adds the stored sums and at least the scratch
    L3, kept = 4 ** 3, 3
    assert wb(4, 8, [4, 2], [2, 3], 3, multihit=True) == base + kept * 4 * L3 * 16
    acc = (2 * L3 * 3 + L3 * 3) * 16
    assert wb(4, 8, [4, 2], [2, 3], 3, symmetric=True) == base + 2 * acc
    assert wb(4, 8, [4, 2], [2, 3], 3, n_rf=2) > base + (512 << 20)
    assert wb(4, 8, [4, 2], [2, 3], 3, n_rf=2, field_squared=True) == wb(4, 8, [4, 2], [2, 3], 3, n_rf=2)
    # FP32 lattices store the field sums in FP32: 4 of the 8 bytes of each of the
    # samples x 6 components x 4 slabs x L^3 sums
    f64 = wb(4, 8, [4, 2], [2, 3], 3, n_rf=2)
    assert f64 - wb(4, 8, [4, 2], [2, 3], 3, n_rf=2, precision=u1ml.FP32) == 6 * 6 * 4 * L3 * 4  # 2 x 3 samples kept
    assert wb(4, 8, [4, 2], [2, 3], 3, precision=7) == 0


@pytest.mark.parametrize("n_metro,n_or", [(256, 3), (1000, 0), (-1, 3), (1, -1)])
def test_hit_count_out_of_range_rejected(n_metro, n_or):
    # the hit index is one byte of the random-number counter: more than 255
    # hits per pass would repeat random numbers, so every entry point refuses
    # them (checked before the handle, so no GPU is needed here)
    lib = u1ml.load_library()
    one = (C.c_int * 1)(2)
    calls = [
        lambda: lib.u1ml_sweep(None, n_metro, n_or),
        lambda: lib.u1ml_batch_sweep(None, n_metro, n_or),
        lambda: lib.u1ml_multilevel(None, 1, one, one, n_metro, n_or, 1, one, 0, None),
        lambda: lib.u1ml_batch_multilevel(None, 1, one, one, n_metro, n_or, 1, one, 0, None),
        lambda: lib.u1ml_batch_cycle(None, 1, n_metro, n_or, 2, 2, 0),
    ]
    for call in calls:
        assert call() == u1ml.EINVAL
        assert b"n_metro" in lib.u1ml_last_error()


def test_stream_bandwidth_arguments_checked():
    # the bandwidth probe refuses bad arguments before touching the device
    lib = u1ml.load_library()
    out = C.c_double()
    for kind, n, reps in ((2, 1 << 24, 1), (-1, 1 << 24, 1), (0, 1 << 10, 1), (0, (1 << 24) + 8, 1), (1, 1 << 24, 0)):
        assert lib.u1ml_stream_bandwidth(kind, n, reps, C.byref(out)) == u1ml.EINVAL
    assert lib.u1ml_stream_bandwidth(0, 1 << 24, 1, None) == u1ml.EINVAL
