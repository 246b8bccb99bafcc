"""Host logic of bench.py (no GPU): refusals, the update and sample counts
against a brute-force count of frozen links, and the counter summary it
reads for the roofline traffic."""
import os
import subprocess
import sys

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bad_replica_split_is_refused():
    for args in (["--replicas", "0"], ["--replicas", "2", "--streams", "3"]):
        r = _run(*args)
        assert r.returncode == 2, args
        assert "--replicas" in r.stderr


def _free_links(L, T, th):
    # brute force: the spatial links at times t = 0 mod th are frozen
    mask = np.ones((T, L, L, L, 4), dtype=bool)
    mask[::th, ..., 1:] = False
    return int(mask.sum())


def test_update_and_sample_counts():
    L, T = bench.L, bench.T
    V = L ** 3 * T
    sweeps, ml = bench.chain_updates_per_step()
    # a compound sweep is 1 Metropolis + 3 overrelaxation passes over every link
    assert sweeps == bench.N_BETWEEN * 4 * 4 * V
    n0, n1 = bench.N_SUB
    th0, th1 = bench.LEVELS
    assert ml == 4 * (n0 * _free_links(L, T, th0) + n0 * n1 * _free_links(L, T, th1))
    # a sample is one innermost-slab update with its measurement, per slab
    assert bench.samples_per_step() == n0 * n1 * (T // th1)


def test_counter_summary_matches_the_class_pass_sources():
    # the roofline's HBM traffic is read from profiles/traffic.json only while
    # the class-pass sources hash to the value recorded there: keep them in step
    # (the benchmark's batch, and the batch larger than the Infinity Cache)
    for R in (bench.DEFAULT_REPLICAS, bench.SPILL_REPLICAS):
        t = bench.traffic_from_profiles("class_pass_batch_kernel<Fast32, mu, kind>", R, 4)
        assert t is not None, R
        algo = R * bench.L ** 3 * bench.T // 2 * bench.WORDS_PER_UPDATE * 4
        assert 1.0 <= t / algo < 1.1


def test_samples_at_the_update_roofline():
    # the samples/s the bench reports at peak: a step's samples over the time
    # of its updates at 36 B per update and 8 TB/s; the multilevel alone (no
    # sweeps) gives 7.5e5 samples/s, the full step (100 sweeps per
    # configuration) 4.3e5
    peak = bench.HBM_PEAK_GBS * 1e9 / (bench.WORDS_PER_UPDATE * 4)
    sweeps, ml = bench.chain_updates_per_step()
    assert bench.chain_updates_per_step(0) == (0, ml)
    assert abs(bench.samples_per_step() * peak / ml - 7.547e5) < 1e2
    assert abs(bench.samples_per_step() * peak / (sweeps + ml) - 4.310e5) < 1e2
