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


def _pass_links_bruteforce(L, T, mu, parity, th):
    """(links read, links written) by one class pass on an L^3 x T lattice,
    by enumeration: every plaquette of the lattice as its four links, the
    updated links (direction mu at the sites of one parity, the spatial ones
    on frozen slices t = 0 mod th excepted), and every link of a plaquette
    containing an updated link read.  Direction 0 is time."""
    shape = (T, L, L, L)
    V = T * L ** 3
    t, z, y, x = np.indices(shape)
    coords = [t, z, y, x]
    ext = [T, L, L, L]

    def link_id(c, d):
        return ((((c[0] % T) * L + c[1] % L) * L + c[2] % L) * L + c[3] % L) * 4 + d

    def shift(c, d):
        c = list(c)
        c[d] = c[d] + 1
        return c

    plaqs = []
    for a in range(4):
        for b in range(a + 1, 4):
            plaqs.append(np.stack([link_id(coords, a), link_id(shift(coords, a), b),
                                   link_id(shift(coords, b), a), link_id(coords, b)], axis=-1).reshape(-1, 4))
    plaqs = np.concatenate(plaqs)
    assert plaqs.shape == (6 * V, 4) and ext[0] == T
    upd = (t + z + y + x) % 2 == parity
    if mu != 0 and th:
        upd &= t % th != 0
    updated = np.zeros(4 * V, dtype=bool)
    updated[link_id(coords, mu)[upd]] = True
    touching = updated[plaqs].any(axis=1)
    read = np.zeros(4 * V, dtype=bool)
    read[plaqs[touching].ravel()] = True
    return int(read.sum()), int(updated.sum())


def test_stencil_words_match_a_brute_force_count():
    # every class pass of a plain sweep and inside slabs of 1, 2 and 4 (frozen
    # spatial links at t = 0 mod th), both parities, every direction
    L, T = 4, 8
    V = T * L ** 3
    for th in (0, 1, 2, 4):
        for mu in range(4):
            for p in (0, 1):
                r, w = _pass_links_bruteforce(L, T, mu, p, th)
                er, ew = bench.pass_words(mu != 0, th)
                assert (r, w) == (er * V, ew * V), (th, mu, p, r, w)
    # per update: 9 words without slabs, 12 with slabs of 2, 10 with slabs of 4
    for th, per_update in ((0, 9), (2, 12), (4, 10)):
        r, w = bench.pass_words(True, th)
        assert (r + w) / w == per_update


def test_stencil_step_words():
    # the benchmark's step on one 24^4 chain: 100 sweeps (4 hits of 36 words
    # per site), 10 level-0 sweeps in slabs of 4 (31.5 words per site and
    # hit) and 200 level-1 sweeps in slabs of 2 (27 words)
    V = bench.L ** 3 * bench.T
    assert bench.hit_words(0) == 36 and bench.hit_words(2) == 27 and bench.hit_words(4) == 31.5
    assert bench.chain_stencil_words() == (100 * 4 * 36 + 10 * 4 * 31.5 + 200 * 4 * 27) * V
    assert bench.chain_stencil_words(0) == (10 * 4 * 31.5 + 200 * 4 * 27) * V
    ro = bench.stencil_roofline(48 * bench.chain_stencil_words(), 4, 440.0)
    assert abs(ro["ms_at_peak"] - 296.687) < 1e-2 and abs(ro["frac"] - 296.687 / 440.0) < 1e-4
    # the measurement alone: 48 x 2400 samples in 182.0 ms at peak
    ro = bench.stencil_roofline(48 * bench.chain_stencil_words(0), 4, 305.0, 48 * bench.samples_per_step())
    assert bench.samples_per_step() == 2400
    assert abs(ro["samples_per_s_at_peak"] - 115200 / 0.18202558) < 1.0
