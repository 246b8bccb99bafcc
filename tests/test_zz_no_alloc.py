"""The allocation-free multilevel entry point (u1ml_multilevel_noalloc),
called through the C ABI, against u1ml_multilevel + u1ml_measure on twin
lattices: identical links and bit-identical correlators, on two calls in a
row (the second smaller), for both precisions, at the 24^4 benchmark shape,
and the refusal of runs larger than the static array.  Device memory in use
must not grow across the calls."""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

from paper_1208_0166_amd import u1ml

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ints(v):
    a = (C.c_int * len(v))(*v)
    return a


def call_noalloc(lat, levels, n_sub, r_list, out):
    lib = u1ml.load_library()
    return lib.u1ml_multilevel_noalloc(lat.handle, len(levels), ints(levels), ints(n_sub), 1, 3, len(r_list),
                                       ints(r_list), C.c_void_p(out.data_ptr()))


def twin(L, prec, seed):
    a = u1ml.init_lattice(L, L, 1.0, seed, precision=prec)
    b = u1ml.init_lattice(L, L, 1.0, seed, precision=prec)
    for g in (a, b):
        u1ml.sweep(g, 1, 3)
    return a, b


@pytest.mark.parametrize("prec", [u1ml.FP64, u1ml.FP32])
def test_noalloc_matches_multilevel_two_calls(prec):
    calls = [  # second call smaller: smaller lattice, one level, fewer separations
        (12, [4, 2], [3, 4], [1, 2, 3, 4, 5, 6]),
        (8, [2], [3], [1, 2, 3]),
    ]
    for k, (L, levels, n_sub, r_list) in enumerate(calls):
        say(f"[gpu] noalloc call {k}: L={L} prec={prec} levels={levels} n_sub={n_sub} r={r_list}")
        a, b = twin(L, prec, 40 + k)
        u1ml.multilevel(a, levels, n_sub, 1, 3, r_list)
        _, c_ref, _ = u1ml.measure(a, observables=False, correlator=True)
        out = torch.full((2 * len(r_list),), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        used0, free0 = torch.cuda.memory_allocated(), torch.cuda.mem_get_info()[0]
        rc = call_noalloc(b, levels, n_sub, r_list, out)
        assert rc == 0, u1ml.load_library().u1ml_last_error()
        # no device memory taken by torch or by the library during the call
        assert torch.cuda.memory_allocated() == used0
        assert torch.cuda.mem_get_info()[0] >= free0
        got = out.cpu().numpy()
        np.testing.assert_array_equal(got[0::2] + 1j * got[1::2], c_ref)
        np.testing.assert_array_equal(u1ml.get_links(b), u1ml.get_links(a))
        assert u1ml.get_pass_id(b) == u1ml.get_pass_id(a)
        # the handle's own workspace stays untouched: nothing was allocated for it
        assert u1ml.device_bytes(b) == 0


def test_noalloc_at_the_benchmark_shape_and_repeated():
    # 24^4, levels {4, 2} x {10, 20}, r = 1..12 (72 MB of workspace), then a
    # second run on the same lattice: the static array keeps the first run's
    # contents, which the second must not see
    L = 24
    r_list = list(range(1, 13))
    a, b = twin(L, u1ml.FP32, 77)
    out = torch.empty(2 * len(r_list), dtype=torch.float64, device="cuda")
    for k in range(2):
        say(f"[gpu] noalloc 24^4 run {k}")
        u1ml.multilevel(a, [4, 2], [10, 20], 1, 3, r_list)
        _, c_ref, _ = u1ml.measure(a, observables=False, correlator=True)
        assert call_noalloc(b, [4, 2], [10, 20], r_list, out) == 0
        got = out.cpu().numpy()
        np.testing.assert_array_equal(got[0::2] + 1j * got[1::2], c_ref)
    np.testing.assert_array_equal(u1ml.get_links(b), u1ml.get_links(a))
    # the Python binding gives the same
    c = u1ml.multilevel_noalloc(b, [2], [2], 1, 3, [1, 2], out=torch.empty(4, dtype=torch.float64, device="cuda"))
    u1ml.multilevel(a, [2], [2], 1, 3, [1, 2])
    _, c_ref, _ = u1ml.measure(a, observables=False, correlator=True)
    np.testing.assert_array_equal(c.cpu().numpy()[0::2] + 1j * c.cpu().numpy()[1::2], c_ref)


@pytest.mark.parametrize("flags", [dict(multihit=True), dict(symmetric=True), dict(multihit=True, symmetric=True)])
def test_noalloc_with_estimator_options(flags):
    # the lattice's estimator flags apply to the allocation-free run as well:
    # multihit lines (twice the stored lines) and the correlator over +-x, +-y, +-z
    say(f"[gpu] noalloc with {flags}")
    a, b = twin(8, u1ml.FP64, 61)
    for g in (a, b):
        u1ml.set_estimator(g, **flags)
    r_list = [1, 2, 3]
    u1ml.multilevel(a, [4, 2], [2, 3], 1, 3, r_list)
    _, c_ref, _ = u1ml.measure(a, observables=False, correlator=True)
    out = torch.empty(2 * len(r_list), dtype=torch.float64, device="cuda")
    assert call_noalloc(b, [4, 2], [2, 3], r_list, out) == 0
    got = out.cpu().numpy()
    np.testing.assert_array_equal(got[0::2] + 1j * got[1::2], c_ref)
    np.testing.assert_array_equal(u1ml.get_links(b), u1ml.get_links(a))


def test_noalloc_refuses_runs_beyond_the_static_array():
    lib = u1ml.load_library()
    g = u1ml.init_lattice(24, 24, 1.0, 3, precision=u1ml.FP32)
    th = u1ml.get_links(g)
    out = torch.empty(24, dtype=torch.float64, device="cuda")
    # 200 inner samples of 12 slabs of 24^3 time lines: 530 MB
    rc = call_noalloc(g, [2], [200], list(range(1, 13)), out)
    assert rc == u1ml.EINVAL
    assert b"static device array" in lib.u1ml_last_error()
    # nothing ran: links unchanged
    np.testing.assert_array_equal(u1ml.get_links(g), th)
    assert u1ml.get_pass_id(g) == 0
    # argument errors
    assert lib.u1ml_multilevel_noalloc(g.handle, 1, ints([2]), ints([2]), 1, 3, 1, ints([1]), None) == u1ml.EINVAL
    assert lib.u1ml_multilevel_noalloc(g.handle, 1, ints([5]), ints([2]), 1, 3, 1, ints([1]),
                                       C.c_void_p(out.data_ptr())) == u1ml.EINVAL
