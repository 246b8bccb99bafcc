"""Launch shapes and the batch autotuner: results are bit-identical for every
shape of every kernel family (class-pass block size and XCD order, per-sample
kernel block, row-fold staging and threads, field transform planes per block
and contraction threads), and the autotuner leaves the chain where it was."""
import sys

import numpy as np
import pytest

from paper_1208_0166_amd import u1ml

pytestmark = pytest.mark.gpu

LS = [12, 24, 12]
BETAS = [1.0, 1.0, 0.9]
SEEDS = [50, 51, 52]
LEVELS, NSUB = [4, 2], [2, 3]
R_LIST = [1, 2, 3, 4, 5, 6]
RF = [2, 4]

SHAPES = [
    dict(pass_block=64, pass_xcd_map=0, sample_block=1024, fold_threads=64, field_w_planes=1, field_o_planes=1,
         field_zcon_threads=64, fold_stage=2),
    dict(pass_block=1024, pass_xcd_map=1, sample_block=64, fold_threads=256, field_w_planes=64, field_o_planes=64,
         field_zcon_threads=256, fold_stage=1),
    dict(pass_block=128, pass_xcd_map=0, sample_block=512, fold_threads=192, field_w_planes=2, field_o_planes=3,
         field_zcon_threads=192, fold_stage=2),
]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(b):
    for _ in range(2):
        u1ml.batch_sweep(b, 1, 3)
    u1ml.batch_multilevel(b, LEVELS, NSUB, 1, 3, R_LIST, rf_list=RF)
    out = []
    for i in range(len(LS)):
        obs, c, f = u1ml.batch_measure(b, i, correlator=True, field_profile=True)
        out.append((u1ml.batch_get_links(b, i), c, f, obs["plaquette"]))
    return out


def same(a, b):
    for (la, ca, fa, pa), (lb, cb, fb, pb) in zip(a, b):
        np.testing.assert_array_equal(la, lb)
        np.testing.assert_array_equal(ca, cb)
        np.testing.assert_array_equal(fa, fb)
        assert pa == pb


@pytest.mark.parametrize("prec", [u1ml.FP32, u1ml.FP64])
def test_every_launch_shape_gives_the_same_bits(prec):
    say(f"[gpu] default shapes prec={prec}")
    ref_b = u1ml.batch_create(LS, LS, BETAS, SEEDS, precision=prec)
    ref = run(ref_b)
    for k, shape in enumerate(SHAPES):
        say(f"[gpu] shape {k}: {shape}")
        b = u1ml.batch_create(LS, LS, BETAS, SEEDS, precision=prec)
        u1ml.set_tuning(b, **shape)
        got = u1ml.get_tuning(b)
        assert got["pass_block"] == shape["pass_block"] and got["pass_xcd_map"] == shape["pass_xcd_map"]
        same(run(b), ref)


def test_autotune_keeps_the_chain_and_its_choice_gives_the_same_bits():
    say("[gpu] batch autotune")
    ref_b = u1ml.batch_create(LS, LS, BETAS, SEEDS, precision=u1ml.FP32)
    ref = run(ref_b)
    b = u1ml.batch_create(LS, LS, BETAS, SEEDS, precision=u1ml.FP32)
    th0 = [u1ml.batch_get_links(b, i) for i in range(len(LS))]
    best = u1ml.batch_autotune(b, LEVELS, [1, 2], R_LIST, RF)
    say(f"  chosen {best}")
    assert best["pass_block"] in (64, 128, 256, 512, 1024) and best["pass_xcd_map"] in (0, 1)
    assert best["sample_block"] in (64, 128, 256, 512, 1024) and best["fold_threads"] in (64, 128, 192, 256)
    assert best["field_w_planes"] >= 1 and best["field_o_planes"] >= 1
    assert best["field_zcon_threads"] in (64, 128, 192, 256) and best["fold_stage"] == 0
    assert u1ml.get_tuning(b) == best
    for i in range(len(LS)):
        np.testing.assert_array_equal(u1ml.batch_get_links(b, i), th0[i])
    # the tuning runs' results are discarded
    with pytest.raises(u1ml.U1MLError):
        u1ml.batch_measure(b, 0, correlator=True)
    same(run(b), ref)


def test_tuning_values_are_checked():
    b = u1ml.batch_create([8, 8], [8, 8], [1.0, 1.0], [1, 2])
    for bad in (dict(pass_block=100), dict(pass_xcd_map=2), dict(sample_block=2048), dict(fold_threads=512),
                dict(field_w_planes=-1), dict(field_zcon_threads=96), dict(fold_stage=3), dict(fold_stage=-1)):
        with pytest.raises(u1ml.U1MLError):
            u1ml.set_tuning(b, **bad)
    # class passes only (no multilevel shape)
    best = u1ml.batch_autotune(b)
    assert best["pass_block"] in (64, 128, 256, 512, 1024)


def test_stream_bandwidth_probe():
    # the streaming references of the bench: a read of more than the Infinity
    # Cache, a cache-sized read and a copy give positive rates below the
    # nameplate 8 TB/s (with headroom for the cache)
    rd = u1ml.stream_bandwidth("read", 1 << 30, 3)
    rc = u1ml.stream_bandwidth("read", 64 << 20, 10)
    cp = u1ml.stream_bandwidth("copy", 1 << 30, 3)
    say(f"  read {rd:.0f}, cache-sized read {rc:.0f}, copy {cp:.0f} GB/s")
    assert 1000 < rd < 8500 and 1000 < cp < 8500 and 1000 < rc < 20000
