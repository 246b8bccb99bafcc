"""Distinct handles are independent: driven from host threads of their own,
on streams of their own, they give the results of the same runs made one
after the other (the library's host-device copies stay in each handle's
stream order, so one handle's graph capture does not disturb another)."""
import sys
import threading

import numpy as np
import pytest

from paper_1208_0166_amd import u1ml

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _make(torch, seed0):
    st = torch.cuda.Stream()
    b = u1ml.batch_create([6, 4], [8, 8], [1.0, 0.9], [seed0, seed0 + 1], start=u1ml.HOT, precision=u1ml.FP64,
                          stream=st.cuda_stream)
    return b, st


def _run(b):
    for _ in range(3):
        u1ml.batch_sweep(b, 1, 3)
    # the first run sets up, runs eagerly and captures; the later ones replay
    for _ in range(3):
        u1ml.batch_multilevel(b, [4, 2], [2, 3], 1, 3, [1, 2, 3], rf_list=[2])
    u1ml.batch_synchronize(b)


def _results(b):
    out = []
    for i in range(2):
        _, c, f = u1ml.batch_measure(b, i, correlator=True, field_profile=True)
        out.append((u1ml.batch_get_links(b, i), c, f))
    return out


def test_handles_on_threads_match_sequential_runs():
    import torch

    torch.cuda.set_device(0)
    say("[gpu] two batch handles on two host threads, first multilevel runs (capture) concurrent")
    ref = []
    for seed in (11, 21):
        b, st = _make(torch, seed)
        _run(b)
        ref.append(_results(b))
    handles = [_make(torch, 11), _make(torch, 21)]
    errors = []

    def worker(b):
        try:
            _run(b)
        except Exception as e:  # reported by the main thread
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(b,)) for b, _ in handles]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for (b, _), want in zip(handles, ref):
        for (links, c, f), (links_r, c_r, f_r) in zip(_results(b), want):
            np.testing.assert_array_equal(links, links_r)
            np.testing.assert_array_equal(c, c_r)
            np.testing.assert_array_equal(f, f_r)
