"""Benchmark: multilevel compact U(1) on 24^4 lattices at beta = 1 on one MI355X.

One step advances R independent 24^4 chains (R = 48 by default, in 3 batches
of 16 on 3 streams whose launches overlap) by one pass of the whole method
each:
  * 100 compound sweeps (1 Metropolis hit + 3 overrelaxation passes per link)
    between measured configurations (Sec. 2.1);
  * one two-level multilevel measurement (Sec. 2.2): slabs of 4 (10 updates)
    holding slabs of 2 (20 updates), Polyakov correlators for r = 1..12 along
    x, and the E/B field profiles (Eq. (5), Eq. (9)) over the 24^2 planes at
    the mid-point of charges at r = 2, 4, 6;
  * the plain observables and the read-back of all results.
The lattices are synthetic (cold start + 200 thermalisation sweeps, seeds 3..);
the launch shapes of every kernel family are picked by the batch autotuner
first.

Printed: one JSON line with link updates/s of the Markov chains (the replay of
the update sequence that the field insertion needs is not counted as
updates), multilevel samples/s (one sample = one innermost-slab update
followed by its two-link measurement for all L^3 sources and all r), the
roofline of the dominant kernel (the class pass, on the benchmark's batch,
which fits the 256 MB Infinity Cache) and of the same kernel on a batch that
does not fit it, a plain device copy for the achievable bandwidth, the
FP32-vs-FP64 deviation of each observable, the 64-lattice uneven batch, one
48^4 lattice in FP32 and FP64, single-chain legs, and the CPU oracle timed on
this host with one thread and with all.  --counters makes the short run used
for the hardware-counter passes instead.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

L = T = 24
BETA = 1.0
LEVELS = [4, 2]
N_SUB = [10, 20]
R_LIST = list(range(1, 13))
RF_LIST = [2, 4, 6]
N_BETWEEN = 100
N_THERM = 200
HBM_PEAK_GBS = 8000.0
INFINITY_CACHE_BYTES = 256 << 20
WORDS_PER_UPDATE = 9  # 8 link reads + 1 write per update in a class pass
DEFAULT_REPLICAS = 48
DEFAULT_STREAMS = 3
CPU_N_SUB = [2, 5]  # reduced multilevel sample for the oracle
CPU_N_SUB_1T = [1, 2]  # the same on one thread
SPILL_REPLICAS = 64  # 64 x 24^4 FP32 = 340 MB of links: more than the 256 MB Infinity Cache
# multilevel shape the autotuner times: 20 kept samples per lattice, so that
# the field contraction runs grids of the size of the benchmark's chunks
TUNE_N_SUB = [2, 10]
COPY_ELEMS = 1 << 27  # calibration copy: 512 MiB read, 512 MiB written


def chain_updates_per_step(n_between=N_BETWEEN):
    V = L ** 3 * T
    sweeps = n_between * 4 * (4 * V)            # 4 passes (1 Metropolis + 3 OR) over 4V links
    free1 = 4 * V - (T // LEVELS[0]) * 3 * L ** 3
    free2 = 4 * V - (T // LEVELS[1]) * 3 * L ** 3
    ml = N_SUB[0] * 4 * free1 + N_SUB[0] * N_SUB[1] * 4 * free2
    return sweeps, ml


def samples_per_step():
    return N_SUB[0] * N_SUB[1] * (T // LEVELS[-1])


def pass_words(spatial, th):
    """(reads, writes) of one class pass in link words per lattice site: the
    distinct links it needs.  A pass updates the direction-mu links at the
    sites of one parity and reads every link of the plaquettes that contain
    them (Sec. 2.1).  With no frozen slices (th = 0), or for time links, that
    is the whole lattice (4 words per site) for half the sites' updates.
    Inside slabs of th time slices (Sec. 2.2) a spatial pass updates the
    slices t != 0 mod th (a fraction f of them) and reads all four links there
    plus, on the frozen slices, the opposite-parity mu links (the time
    plaquettes' far sides) and the time links leaving them: 4 f + 1.5 (1 - f)."""
    if not spatial or th == 0:
        return 4.0, 0.5
    if th == 1:
        return 0.0, 0.0  # every spatial link frozen: the pass updates and reads nothing
    f = (th - 1) / th
    return 4.0 * f + 1.5 * (1.0 - f), f / 2.0


def hit_words(th):
    """Link words of one hit (one Metropolis or one OR pass over every class:
    2 parities x (1 time + 3 spatial directions)) per lattice site."""
    return 2 * sum(pass_words(False, th)) + 6 * sum(pass_words(True, th))


def stencil_words(V, n_sweeps, levels, n_sub):
    """Link words the class passes of n_sweeps compound sweeps and one
    multilevel run (levels, n_sub) move on one lattice of V sites, each pass
    counted by its stencil (pass_words); 4 hits (1 Metropolis + 3 OR) per
    compound sweep."""
    words = n_sweeps * 4 * hit_words(0)
    reps = 1
    for th, n in zip(levels, n_sub):
        reps *= n
        words += reps * 4 * hit_words(th)
    return words * V


def chain_stencil_words(n_between=N_BETWEEN):
    return stencil_words(L ** 3 * T, n_between, LEVELS, N_SUB)


def stencil_roofline(words, bytes_per_word, ms, samples=None):
    """The link traffic of a step counted by its stencils, against the HBM
    peak: bytes, the step time at peak, the fraction of it achieved and, with
    the step's samples, the samples/s at peak."""
    b = words * bytes_per_word
    ms_peak = b / (HBM_PEAK_GBS * 1e9) * 1e3
    out = {"bytes_per_step": b, "ms_at_peak": ms_peak, "frac": ms_peak / ms}
    if samples is not None:
        out["samples_per_s_at_peak"] = samples / (ms_peak * 1e-3)
    return out


def sweep_sources_sha():
    h = hashlib.sha256()
    for f in ("sweep_impl.h", "device_common.h", "sweep_f32.hip", "sweep_f64.hip"):
        with open(os.path.join(ROOT, "paper_1208_0166_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_key, replicas, bytes_per_word):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources and this batch shape; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(p) as f:
            d = json.load(f)
        e = d.get(kernel_key)
        if e and e.get("sources_sha") == sweep_sources_sha() and e.get("bytes_per_word") == bytes_per_word:
            r = e.get("by_replicas", {}).get(str(replicas))
            if r:
                return r["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_leg(oracle, seconds, n_sub):
    o = oracle.OracleLattice(L, T, BETA, 3, hot=False)
    o.sweep(1, 3)  # warm-up
    n, t0 = 0, time.perf_counter()
    while True:
        o.sweep(1, 3)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds and n >= 2:
            break
    ups = n * 16 * L ** 3 * T / el
    t0 = time.perf_counter()
    o.multilevel(LEVELS, n_sub, 1, 3, R_LIST)  # no field: the oracle's field accumulators exceed memory at 24^4
    el_ml = time.perf_counter() - t0
    samp = n_sub[0] * n_sub[1] * (T // LEVELS[-1])
    return ups, samp / el_ml, n, el, samp, el_ml


def cpu_baseline(seconds: float):
    """The FP64 oracle on this host, on all its cores and on one: compound
    sweeps of the 24^4 lattice for about `seconds` each, and one reduced
    multilevel run for samples/s."""
    import oracle
    n_all = oracle.max_threads()
    ups, sps, n, el, samp, el_ml = _oracle_leg(oracle, seconds, CPU_N_SUB)
    oracle.set_threads(1)
    try:
        ups1, sps1, n1, el1, samp1, el_ml1 = _oracle_leg(oracle, seconds, CPU_N_SUB_1T)
    finally:
        oracle.set_threads(n_all)
    return {"value": ups, "unit": "link updates/s", "cores": n_all, "kind": "oracle",
            "samples_per_s": sps, "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{n} compound sweeps (1 Metropolis + 3 OR) of 24^4 FP64 in {el:.1f} s; "
                      f"multilevel levels {LEVELS} with n_sub {CPU_N_SUB}, r = 1..12, no field ({samp} samples) "
                      f"in {el_ml:.1f} s",
            "single_thread": {"value": ups1, "unit": "link updates/s", "cores": 1, "samples_per_s": sps1,
                              "sample": f"{n1} compound sweeps in {el1:.1f} s; multilevel n_sub {CPU_N_SUB_1T} "
                                        f"({samp1} samples) in {el_ml1:.1f} s"}}


def run_chain(u1ml, torch, prec, R, rf, steps, warmup, n_streams=1, multihit=False, squared=False, symmetric=False,
              tune=True, n_between=N_BETWEEN, pipeline=True):
    """Build R independent 24^4 chains split into n_streams groups (one batch,
    or one lattice, per group, each on a stream of its own), thermalise, and
    time `steps` steps; the groups' launches overlap on the GPU.  With
    pipeline, a step queues every group's sweeps before it reads the previous
    step's results of each group and queues that group's multilevel run, so
    that no stream idles at the step boundary; every step's results are read
    inside the timed region, and the plain observables are then those of the
    links after the next step's sweeps.  Returns a dict of timings and the
    last results of group 0."""
    sizes = [R // n_streams + (1 if g < R % n_streams else 0) for g in range(n_streams)]
    sizes = [n for n in sizes if n > 0]
    groups = []
    first = 0
    for n in sizes:
        st = torch.cuda.Stream()
        seeds = [3 + first + i for i in range(n)]
        if n == 1:
            lat = u1ml.init_lattice(L, T, BETA, seeds[0], start=u1ml.COLD, precision=prec, stream=st.cuda_stream)
            sw = (lambda lt: lambda: u1ml.sweep(lt, 1, 3))(lat)
        else:
            lat = u1ml.batch_create([L] * n, [T] * n, [BETA] * n, seeds, start=u1ml.COLD, precision=prec,
                                    stream=st.cuda_stream)
            sw = (lambda lt: lambda: u1ml.batch_sweep(lt, 1, 3))(lat)
        if multihit or squared or symmetric:
            (u1ml.set_estimator if n == 1 else u1ml.batch_set_estimator)(lat, multihit=multihit,
                                                                          field_squared=squared, symmetric=symmetric)
        groups.append({"lat": lat, "sw": sw, "st": st, "n": n})
        first += n
    tuning = None
    if isinstance(tune, dict):
        tuning = dict(tune)
        for gr in groups:
            if gr["n"] > 1:
                u1ml.set_tuning(gr["lat"], **tuning)
    elif tune and groups[0]["n"] > 1:
        # launch shapes picked on the first batch, applied to the others (same shape)
        tuning = u1ml.batch_autotune(groups[0]["lat"], LEVELS, TUNE_N_SUB, R_LIST, rf)
        for gr in groups[1:]:
            if gr["n"] > 1:
                u1ml.set_tuning(gr["lat"], **tuning)
    for _ in range(N_THERM):
        for gr in groups:
            gr["sw"]()
    torch.cuda.synchronize()

    def queue_sweeps(gr, ev=None):
        if ev:
            ev[0].record(gr["st"])
        for _ in range(n_between):
            gr["sw"]()
        if ev:
            ev[1].record(gr["st"])

    def queue_ml(gr, ev=None):
        if gr["n"] == 1:
            u1ml.multilevel(gr["lat"], LEVELS, N_SUB, 1, 3, R_LIST, rf_list=rf)
        else:
            u1ml.batch_multilevel(gr["lat"], LEVELS, N_SUB, 1, 3, R_LIST, rf_list=rf)
        if ev:
            ev[2].record(gr["st"])

    def launch(gr, ev=None):
        queue_sweeps(gr, ev)
        queue_ml(gr, ev)

    def results(gr):
        if gr["n"] == 1:
            return [u1ml.measure(gr["lat"], correlator=True, field_profile=bool(rf))]
        return [u1ml.batch_measure(gr["lat"], i, correlator=True, field_profile=bool(rf)) for i in range(gr["n"])]

    def step(evs=None):
        for g, gr in enumerate(groups):  # all groups queued before any result is read
            launch(gr, evs[g] if evs else None)
        res = [results(gr) for gr in groups]
        return res[0][0]

    def pipelined_step(read_prev, evs=None):
        # every group's sweeps first; then per group: the previous step's
        # results (waits for that group's stream), and this step's multilevel
        for g, gr in enumerate(groups):
            queue_sweeps(gr, evs[g] if evs else None)
        first = None
        for g, gr in enumerate(groups):
            if read_prev:
                r = results(gr)
                first = first or r[0]
            queue_ml(gr, evs[g] if evs else None)
        return first

    def drain():
        return [results(gr) for gr in groups][0][0]

    for w in range(warmup):
        if pipeline:
            pipelined_step(w > 0)
        else:
            step()
    if pipeline and warmup:
        drain()
    torch.cuda.synchronize()
    evs = [[[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in groups] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        if pipeline:
            pipelined_step(k > 0, evs[k])
        else:
            obs, corr, field = step(evs[k])
    if pipeline:
        obs, corr, field = drain()  # the last step's results
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_sweeps = sum(e[0][0].elapsed_time(e[0][1]) for e in evs) / steps  # group 0
    ms_ml = sum(e[0][1].elapsed_time(e[0][2]) for e in evs) / steps
    up_sw, up_ml = chain_updates_per_step(n_between)
    n0 = groups[0]["n"]
    return {"groups": groups, "el": el, "ms_step": 1e3 * el / steps, "ms_sweeps": ms_sweeps, "ms_ml": ms_ml,
            "updates_per_s": R * (up_sw + up_ml) * steps / el,
            "samples_per_s": R * samples_per_step() * steps / el,
            "group0_sweep_updates_per_s": n0 * up_sw / (ms_sweeps * 1e-3) if ms_sweeps > 0 else None,
            "group0_ml_updates_per_s": n0 * up_ml / (ms_ml * 1e-3),
            "group0_ml_samples_per_s": n0 * samples_per_step() / (ms_ml * 1e-3),
            "obs": obs, "corr": corr, "tuning": tuning}


def roofline_leg(u1ml, torch, prec, R, steps, n_sweeps=N_BETWEEN, tune=True):
    """The dominant kernel alone: n_sweeps compound sweeps of one R-lattice
    batch on one stream (class-pass shapes from the autotuner), timed with HIP
    events on that stream around each step's sweeps."""
    st = torch.cuda.Stream()
    tuning = None
    if R == 1:
        lat = u1ml.init_lattice(L, T, BETA, 3, start=u1ml.COLD, precision=prec, stream=st.cuda_stream)
        sw = lambda: u1ml.sweep(lat, 1, 3)  # noqa: E731
    else:
        lat = u1ml.batch_create([L] * R, [T] * R, [BETA] * R, [3 + i for i in range(R)], start=u1ml.COLD,
                                precision=prec, stream=st.cuda_stream)
        sw = lambda: u1ml.batch_sweep(lat, 1, 3)  # noqa: E731
        if isinstance(tune, dict):
            u1ml.set_tuning(lat, **tune)
            tuning = u1ml.get_tuning(lat)
        elif tune:
            tuning = u1ml.batch_autotune(lat)
    for _ in range(20):
        sw()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record(st)
        for _ in range(n_sweeps):
            sw()
        b.record(st)
    torch.cuda.synchronize()
    ms = sum(a.elapsed_time(b) for a, b in ev) / steps
    if R > 1:
        iso = u1ml.batch_profile_sweeps(lat, 5, 1, 3)
    else:
        iso = u1ml.profile_sweeps(lat, 5, 1, 3)
    del lat
    return ms, iso, tuning


def roofline_entry(u1ml, prec, R, ms, n_sweeps, steps, iso, tuning, traffic):
    """Class-pass roofline from the average duration of the timed sweeps:
    algorithmic bytes (9 link words per update) per launch over the average
    launch time, against the 8 TB/s HBM peak."""
    passes_per_step = n_sweeps * 4 * 8
    avg_us = 1e3 * ms / passes_per_step
    bw = 4 if prec == u1ml.FP32 else 8
    updates_per_launch = R * L ** 3 * T // 2
    bytes_per_launch = updates_per_launch * WORDS_PER_UPDATE * bw
    achieved = bytes_per_launch / (avg_us * 1e-6) / 1e9
    pname = "Fast32" if prec == u1ml.FP32 else "Det64"
    kname = f"class_pass_batch_kernel<{pname}, mu, kind>" if R > 1 else f"class_pass_kernel<{pname}, mu, kind>"
    batch_bytes = R * 4 * L ** 3 * T * bw
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kname, "avg_us": avg_us,
            "launches_timed": passes_per_step * steps, "replicas": R, "batch_bytes": batch_bytes,
            "cache_resident": batch_bytes <= INFINITY_CACHE_BYTES,
            "isolated_event_us": {"metropolis": iso[0], "or": iso[1]},
            "algorithmic_bytes_per_launch": bytes_per_launch, "tuning": tuning}


def main_tuning(tune, out):
    """The launch shapes the main run used (its autotuner's choice), for legs of the same shape."""
    if isinstance(tune, dict):
        return tune
    if tune and out.get("tuning"):
        return out["tuning"]
    return tune


def stream_bandwidth(u1ml, n_bytes=2 << 30, cached_bytes=192 << 20, reps=5):
    """Reference streaming rates of this GPU from the library's plain
    grid-stride kernels of 16-byte accesses, timed with HIP events: a read of
    n_bytes (HBM), a read of cached_bytes repeated (small enough to stay in the
    256 MB Infinity Cache), and a copy of n_bytes (read + write counted)."""
    return {"read_GB_per_s": u1ml.stream_bandwidth("read", n_bytes, reps),
            "read_cache_resident_GB_per_s": u1ml.stream_bandwidth("read", cached_bytes, 4 * reps),
            "copy_GB_per_s": u1ml.stream_bandwidth("copy", n_bytes, reps),
            "bytes": {"read": n_bytes, "read_cache_resident": cached_bytes, "copy": 2 * n_bytes}}


def precision_leg():
    """FP32 sweeps / FP64 accumulation against the FP64 path on the benchmark's
    workload (24^4, beta = 1, multilevel {4,2} x {10,20}): 8 chains per
    precision, 3 configurations 50 sweeps apart after 200 thermalisation
    sweeps; relative deviation and its size in combined jackknife errors, for
    the plaquette, |P|, C_ML(r = 1..4) and the E_x insertion at r = 2."""
    from paper_1208_0166_amd import precision
    rows = precision.compare(L=L, beta=BETA, n_chains=8, n_therm=N_THERM, n_configs=3, n_between=50,
                             levels=tuple(LEVELS), n_sub=tuple(N_SUB), r_list=(1, 2, 3, 4), seed0=2000, rf=2)
    return {"chains_per_precision": 8, "configurations_per_chain": 3,
            "observables": {r["name"]: {"rel_dev": r["rel_dev"], "sigmas": r["sigmas"], "rel_err": r["rel_err"],
                                        "fp32": r["fp32"], "fp64": r["fp64"]} for r in rows}}


def counters_run(args):
    """Short run for hardware-counter passes: a plain elementwise copy of a known
    size (the calibration of FETCH_SIZE / WRITE_SIZE); the library's streaming
    read of a 1 GiB buffer (HBM) and then of a 64 MiB one (served by the
    Infinity Cache once warm), the references of the L2-miss read latency
    (1 + 3 and 1 + 10 dispatches of `stream_read_kernel`, in that order);
    then a few compound sweeps of the benchmark batch."""
    import torch
    from paper_1208_0166_amd import u1ml
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    n = COPY_ELEMS
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst
    u1ml.stream_bandwidth("read", 1 << 30, 3)
    u1ml.stream_bandwidth("read", 64 << 20, 10)
    if args.counters_uneven:
        # the 64 uneven lattices: two sweeps and one measurement cycle (one
        # sweep, the single-level run with slabs of 2 and 10 updates,
        # r = 1..L/2), launched one kernel at a time
        import numpy as np

        rng = np.random.default_rng(7)
        Ls = [int(v) for v in rng.choice([8, 12, 16, 20, 24], UNEVEN_N)]
        betas = [float(v) for v in rng.choice([0.9, 1.0, 1.1], UNEVEN_N)]
        b = u1ml.batch_create(Ls, Ls, betas, [1000 + i for i in range(UNEVEN_N)], start=u1ml.COLD,
                              precision=u1ml.FP32, stream=stream.cuda_stream)
        for _ in range(2):
            u1ml.batch_sweep(b, 1, 3)
        u1ml.batch_cycle(b, 1, 1, 3, UNEVEN_TH, UNEVEN_NSUB, use_graph=False)
        u1ml.batch_synchronize(b)
        print(json.dumps({"counters_run": True, "copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n,
                          "uneven": UNEVEN_N}), flush=True)
        return
    R = args.replicas
    prec = u1ml.FP32 if args.precision == "fp32" else u1ml.FP64
    lat = u1ml.batch_create([L] * R, [T] * R, [BETA] * R, [3 + i for i in range(R)], start=u1ml.COLD,
                            precision=prec, stream=stream.cuda_stream)
    for _ in range(4):
        u1ml.batch_sweep(lat, 1, 3)
    if args.counters_multilevel:
        # the class passes inside slabs of 4 and of 2 (one update per level),
        # told apart from the plain passes by their grid sizes: R V / 2
        # threads plain, R V 3 / 8 in slabs of 4, R V / 4 in slabs of 2
        u1ml.batch_multilevel(lat, LEVELS, [1, 1], 1, 3, [1])
    torch.cuda.synchronize()
    print(json.dumps({"counters_run": True, "copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n,
                      "replicas": R, "sweeps": 4, "multilevel": bool(args.counters_multilevel)}), flush=True)


LARGE_L = 48
LARGE_LEVELS = [4, 2]
LARGE_N_SUB = [20, 10]
LARGE_THERM = 500


def large_leg(u1ml, torch, n_therm=LARGE_THERM):
    """One 48^4 beta=1 chain per precision (same seed, cold start): n_therm
    sweeps, then N_BETWEEN timed sweeps and one timed two-level multilevel
    {4,2} x {20,10}, r = 1..24, E/B profiles at r = 2, 4, 6.  Returns the
    sweep and multilevel throughput of the FP32 and FP64 paths, the
    deviation of the two timed chains' plaquettes (two chains of the same
    distribution: the FP32 path draws its own random numbers, so the
    difference is statistical), and the FP32 / FP64 comparison over 16
    independent chains per precision."""
    r_list = list(range(1, LARGE_L // 2 + 1))
    res = {}
    for name, prec in (("fp32", u1ml.FP32), ("fp64", u1ml.FP64)):
        st = torch.cuda.Stream()
        g = u1ml.init_lattice(LARGE_L, LARGE_L, BETA, 3, start=u1ml.COLD, precision=prec, stream=st.cuda_stream)
        for _ in range(n_therm):
            u1ml.sweep(g, 1, 3)
        u1ml.multilevel(g, LARGE_LEVELS, LARGE_N_SUB, 1, 3, r_list, rf_list=RF_LIST)  # set-up, capture
        u1ml.synchronize(g)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(st)
        for _ in range(N_BETWEEN):
            u1ml.sweep(g, 1, 3)
        ev[1].record(st)
        u1ml.multilevel(g, LARGE_LEVELS, LARGE_N_SUB, 1, 3, r_list, rf_list=RF_LIST)
        ev[2].record(st)
        obs, corr, _ = u1ml.measure(g, correlator=True, field_profile=True)
        ms_sw, ms_ml = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
        V = LARGE_L ** 4
        up_ml = 0
        prod = 1
        for l, th in enumerate(LARGE_LEVELS):
            prod *= LARGE_N_SUB[l]
            up_ml += prod * (4 * V - 3 * V // th)  # links not frozen at level l
        up_ml *= 1 + 3  # Metropolis + 3 OR
        res[name] = {"sweep_updates_per_s": N_BETWEEN * 16 * V / (ms_sw * 1e-3), "ms_100_sweeps": ms_sw,
                     "multilevel_ms": ms_ml, "multilevel_updates_per_s": up_ml / (ms_ml * 1e-3),
                     "plaquette": obs["plaquette"], "poly_abs": obs["poly_abs"],
                     "C": [[c.real, c.imag] for c in corr[:6]]}
        del g
    d_plaq = abs(res["fp32"]["plaquette"] - res["fp64"]["plaquette"]) / abs(res["fp64"]["plaquette"])
    # the controlled comparison at this size: independent chains per precision
    from paper_1208_0166_amd import precision
    rows = precision.compare(L=LARGE_L, beta=BETA, n_chains=16, n_therm=100, n_configs=2, n_between=40,
                             levels=tuple(LARGE_LEVELS), n_sub=tuple(LARGE_N_SUB), r_list=(1, 2), seed0=4000)
    split = {"chains_per_precision": 16, "configurations_per_chain": 2,
             "protocol": "cold start, 100 sweeps, then 2 x (40 sweeps + multilevel {4,2} x {20,10}, r = 1, 2)",
             "observables": {r["name"]: {"rel_dev": r["rel_dev"], "sigmas": r["sigmas"], "rel_err": r["rel_err"],
                                         "fp32": r["fp32"], "fp64": r["fp64"]} for r in rows}}
    return {"workload": f"one 48^4 beta=1 chain per precision: {n_therm} sweeps, then {N_BETWEEN} timed sweeps "
                        f"and one two-level multilevel {{4,2}} x {{20,10}}, r=1..24, E/B mid-plane profiles at "
                        "r=2,4,6",
            "fp32": res["fp32"], "fp64": res["fp64"],
            "fp32_over_fp64_sweeps": res["fp32"]["sweep_updates_per_s"] / res["fp64"]["sweep_updates_per_s"],
            "fp32_over_fp64_multilevel": res["fp32"]["multilevel_updates_per_s"] /
                                         res["fp64"]["multilevel_updates_per_s"],
            "plaquette_rel_deviation": d_plaq,
            "precision_split": split,
            "note": "plaquette_rel_deviation compares the one timed chain per precision (one draw of a "
                    "statistical difference); precision_split is the controlled comparison over 16 independent "
                    "chains per precision (jackknife errors)"}


def large_run(args):
    import torch
    from paper_1208_0166_amd import u1ml

    torch.cuda.set_device(0)
    leg = large_leg(u1ml, torch)
    out = {"metric": "link updates/s (Metropolis+OR), 48^4 beta=1, FP32 and FP64 paths",
           "value": leg["fp32"]["sweep_updates_per_s"], "unit": "link updates/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic (cold start, seed 3)",
           "config": {"workload": leg["workload"]}}
    out.update({k: v for k, v in leg.items() if k != "workload"})
    print(json.dumps(out), flush=True)


UNEVEN_N = 64
UNEVEN_SWEEPS = 10
UNEVEN_TH, UNEVEN_NSUB = 2, 10


def uneven_leg(u1ml, torch, n_cycles, warmup=1, tune=True):
    """64 independent lattices of sizes drawn from {8,12,16,20,24}^4 and beta
    from {0.9, 1.0, 1.1} (numpy default_rng(7)), FP32 links, one batch on one
    stream (launch shapes from the autotuner, timed on the cycle's multilevel
    shape with r = 1..4): after N_THERM sweeps,
    n_cycles cycles of UNEVEN_SWEEPS compound sweeps plus a single-level
    multilevel (slab thickness 2, 10 updates) with correlators at r = 1..L/2,
    each cycle one captured HIP graph; then every lattice's results are read
    back."""
    import numpy as np

    rng = np.random.default_rng(7)
    Ls = [int(v) for v in rng.choice([8, 12, 16, 20, 24], UNEVEN_N)]
    betas = [float(v) for v in rng.choice([0.9, 1.0, 1.1], UNEVEN_N)]
    st = torch.cuda.Stream()
    b = u1ml.batch_create(Ls, Ls, betas, [1000 + i for i in range(UNEVEN_N)], start=u1ml.COLD,
                          precision=u1ml.FP32, stream=st.cuda_stream)
    tuning = None
    if isinstance(tune, dict):
        u1ml.set_tuning(b, **tune)
        tuning = u1ml.get_tuning(b)
    elif tune:
        # the cycle's multilevel shape, with the separations every lattice has
        tuning = u1ml.batch_autotune(b, [UNEVEN_TH], [UNEVEN_NSUB], list(range(1, min(Ls) // 2 + 1)))
    for _ in range(N_THERM):
        u1ml.batch_sweep(b, 1, 3)

    def cycle():
        u1ml.batch_cycle(b, UNEVEN_SWEEPS, 1, 3, UNEVEN_TH, UNEVEN_NSUB, use_graph=True)

    for _ in range(max(warmup, 1)):
        cycle()
    u1ml.batch_synchronize(b)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    t0 = time.perf_counter()
    ev[0].record(st)
    for _ in range(n_cycles):
        cycle()
    ev[1].record(st)
    res = [u1ml.batch_measure(b, i, correlator=True) for i in range(UNEVEN_N)]
    el = time.perf_counter() - t0
    ms_cycles = ev[0].elapsed_time(ev[1])
    V = [L_ ** 4 for L_ in Ls]
    up = sum(UNEVEN_SWEEPS * 16 * v + UNEVEN_NSUB * 4 * (4 * v - 3 * v // UNEVEN_TH) for v in V)
    samples = sum(UNEVEN_NSUB * (L_ // UNEVEN_TH) for L_ in Ls)
    counts = {int(k): int(c) for k, c in zip(*np.unique(Ls, return_counts=True))}
    del b
    return {"workload": f"64 independent lattices L^4, L counts {counts}, beta in {{0.9, 1.0, 1.1}}, one "
                        f"batch; per cycle {UNEVEN_SWEEPS} sweeps + single-level multilevel (th 2, 10 "
                        "updates), r = 1..L/2, one captured graph per cycle",
            "updates_per_s": up * n_cycles / el, "samples_per_s": samples * n_cycles / el,
            "cycles": n_cycles, "ms_per_cycle": 1e3 * el / n_cycles, "gpu_ms_per_cycle": ms_cycles / n_cycles,
            "updates_per_s_gpu": up * n_cycles / (ms_cycles * 1e-3),
            "step_roofline_frac": up * n_cycles / el / (HBM_PEAK_GBS * 1e9 / (WORDS_PER_UPDATE * 4)),
            "stencil_exact": stencil_roofline(sum(stencil_words(v, UNEVEN_SWEEPS, [UNEVEN_TH], [UNEVEN_NSUB])
                                                  for v in V), 4, 1e3 * el / n_cycles),
            "plaquette_min_max": [min(r[0]["plaquette"] for r in res), max(r[0]["plaquette"] for r in res)],
            "tuning": tuning}


def uneven_run(args):
    import torch
    from paper_1208_0166_amd import u1ml

    torch.cuda.set_device(0)
    leg = uneven_leg(u1ml, torch, 10 * args.steps, args.warmup)
    out = {"metric": "link updates/s (Metropolis+OR) and multilevel correlator samples/s, 64 uneven instances",
           "value": leg["updates_per_s"], "unit": "link updates/s", "n_gpus": 1, "steps": leg["cycles"],
           "warmup": max(args.warmup, 1), "ms_per_step": leg["ms_per_cycle"], "higher_is_better": True,
           "dtype": "f32", "data": "synthetic (cold start, 200 thermalisation sweeps, sizes and beta from default_rng(7))",
           "config": {"workload": leg["workload"]}}
    out.update({k: v for k, v in leg.items() if k != "workload"})
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--no-field", action="store_true", help="skip the field-profile insertion")
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the single-chain FP32 and FP64 comparison legs")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the cache-spilling roofline, copy, precision, uneven and 48^4 legs")
    ap.add_argument("--no-tune", action="store_true", help="default launch shapes instead of the autotuner's")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="read every step's results before the next step is queued (the streams drain per step)")
    ap.add_argument("--tuning", default=None,
                    help="JSON object of launch shapes (u1ml_tuning fields) applied to every batch instead of "
                         "running the autotuner (reproducible profiles)")
    ap.add_argument("--replicas", type=int, default=DEFAULT_REPLICAS,
                    help="independent 24^4 chains advanced by the same launches (one batch)")
    ap.add_argument("--streams", type=int, default=DEFAULT_STREAMS,
                    help="the replicas are split into this many batches, each on a stream of its own")
    ap.add_argument("--multihit", action="store_true",
                    help="multihit means for the correlator lines at r >= 2 (the paper's potential)")
    ap.add_argument("--squared", action="store_true", help="insert the squared field components of Eq. (6)")
    ap.add_argument("--symmetric", action="store_true",
                    help="correlator averaged over separations along +-x, +-y, +-z")
    ap.add_argument("--counters", action="store_true", help="short run for hardware-counter passes")
    ap.add_argument("--counters-multilevel", action="store_true",
                    help="with --counters: one multilevel run {4,2} x {1,1} after the sweeps")
    ap.add_argument("--counters-uneven", action="store_true",
                    help="with --counters: the 64 uneven lattices (two sweeps and one measurement cycle) instead")
    ap.add_argument("--large", action="store_true",
                    help="instead of the 24^4 workload: one 48^4 chain per precision (FP32 vs FP64)")
    ap.add_argument("--uneven", action="store_true",
                    help="instead of the 24^4 workload: 64 lattices of uneven size and beta in captured cycles")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); there is no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    if args.replicas < 1 or not 1 <= args.streams <= args.replicas:
        print("need --replicas >= 1 and 1 <= --streams <= --replicas", file=sys.stderr)
        sys.exit(2)
    if args.counters:
        counters_run(args)
        return
    if args.large:
        large_run(args)
        return
    if args.uneven:
        uneven_run(args)
        return

    import torch
    from paper_1208_0166_amd import u1ml

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    # every lattice or batch gets a stream of its own (passed explicitly); torch's
    # own work goes to a dedicated stream as well
    torch.cuda.set_stream(torch.cuda.Stream())
    prec = u1ml.FP32 if args.precision == "fp32" else u1ml.FP64
    rf = [] if args.no_field else RF_LIST
    R = args.replicas
    tune = json.loads(args.tuning) if args.tuning else not args.no_tune

    progress("main run")
    main_run = run_chain(u1ml, torch, prec, R, rf, args.steps, args.warmup, args.streams, args.multihit,
                         args.squared, args.symmetric, tune=tune, pipeline=not args.no_pipeline)

    # dominant kernel: the class pass (Metropolis or OR, 9 words per update),
    # timed alone on one stream: N_BETWEEN compound sweeps of 4 x 8 class passes
    # plus one pass-id bump per step, so (sweep time) / (class passes) bounds
    # the average dispatch time from above.  Per-launch event timings are
    # recorded beside it.
    progress("roofline leg")
    bw = 4 if prec == u1ml.FP32 else 8
    ms_rf, iso, rf_tuning = roofline_leg(u1ml, torch, prec, R, args.steps, tune=tune)
    pname = "Fast32" if prec == u1ml.FP32 else "Det64"
    kname = f"class_pass_batch_kernel<{pname}, mu, kind>" if R > 1 else f"class_pass_kernel<{pname}, mu, kind>"
    roofline = roofline_entry(u1ml, prec, R, ms_rf, N_BETWEEN, args.steps, iso, rf_tuning,
                              traffic_from_profiles(kname, R, bw))
    roofline["note"] = ("the benchmark's batch fits the 256 MB Infinity Cache, which serves part of every class "
                        "pass; roofline_spilled is the same kernel on a batch larger than the cache")

    obs, corr = main_run["obs"], main_run["corr"]
    out = {
        "metric": "link updates/s (Metropolis+OR) and multilevel correlator samples/s, 24^4 beta=1",
        "value": main_run["updates_per_s"],
        "unit": "link updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == u1ml.FP32 else "f64",
        "data": "synthetic (cold start, 200 thermalisation sweeps, seeds 3..)",
        "config": {"workload": f"{R} independent 24^4 beta=1 chains on {args.streams} stream(s), each step "
                               "per chain: 100 sweeps (1 Metropolis + 3 OR) + two-level multilevel {4,2} x {10,20}, "
                               "r=1..12, E/B mid-plane profiles at r=2,4,6",
                   "lattice": [L, L, L, T], "beta": BETA, "levels": LEVELS, "n_sub": N_SUB,
                   "r": [1, 12], "field_r": rf, "accumulate": "f64", "replicas": R, "streams": args.streams,
                   "multihit": args.multihit, "field_squared": args.squared, "symmetric": args.symmetric,
                   "pipelined_steps": not args.no_pipeline},
        "samples_per_s": main_run["samples_per_s"],
        "samples_per_step": samples_per_step() * R,
        # complete two-level multilevel estimates (one per chain per step)
        "multilevel_estimates_per_s": R * args.steps / (main_run["ms_step"] * 1e-3 * args.steps),
        "chain_updates_per_step": R * sum(chain_updates_per_step()),
        "streams": args.streams,
        "tuning": main_run["tuning"],
        "group0_phase_ms": {"sweeps": main_run["ms_sweeps"], "multilevel": main_run["ms_ml"]},
        "group0_sweep_updates_per_s": main_run["group0_sweep_updates_per_s"],
        "group0_multilevel_chain_updates_per_s": main_run["group0_ml_updates_per_s"],
        "group0_multilevel_phase_samples_per_s": main_run["group0_ml_samples_per_s"],
        "plaquette": obs["plaquette"],
        "poly_abs": obs["poly_abs"],
        "C_r1": [corr[0].real, corr[0].imag],
        "roofline": roofline,
        # the whole step against the same bound: every link update at 9 words
        # per update and the HBM peak (the field contraction, folds and
        # time-line sums are work on top of the updates, not counted as updates)
        # samples come with the updates of their step, so the samples/s at
        # the same bound is the step's samples over the time of its updates
        # at peak, and their fraction equals the updates' fraction
        "step_roofline": {"updates_per_s_at_peak": HBM_PEAK_GBS * 1e9 / (WORDS_PER_UPDATE * bw),
                          "frac": main_run["updates_per_s"] / (HBM_PEAK_GBS * 1e9 / (WORDS_PER_UPDATE * bw)),
                          "samples_per_s_at_peak": samples_per_step() * HBM_PEAK_GBS * 1e9 /
                                                   (WORDS_PER_UPDATE * bw * sum(chain_updates_per_step())),
                          # the passes inside slabs read their frozen neighbour
                          # slices too: 12 words per update with slabs of 2,
                          # 10 with slabs of 4 (pass_words); every pass counted
                          # by its stencil
                          "stencil_exact": stencil_roofline(R * chain_stencil_words(), bw, main_run["ms_step"],
                                                            R * samples_per_step())},
    }
    del main_run
    if not args.no_extra:
        # the multilevel measurement alone (no sweeps between configurations):
        # the samples/s of the two-level run itself
        progress("multilevel-only leg")
        ml_run = run_chain(u1ml, torch, prec, R, rf, args.steps, 1, args.streams, args.multihit, args.squared,
                           args.symmetric, tune=main_tuning(tune, out), n_between=0, pipeline=not args.no_pipeline)
        out["multilevel_only"] = {
            "workload": f"{R} chains, each step one two-level multilevel {{4,2}} x {{10,20}} per chain, r=1..12, "
                        f"field at r={rf}, no sweeps between",
            "samples_per_s": ml_run["samples_per_s"], "updates_per_s": ml_run["updates_per_s"],
            "ms_per_step": ml_run["ms_step"],
            "step_roofline_frac": ml_run["updates_per_s"] / (HBM_PEAK_GBS * 1e9 / (WORDS_PER_UPDATE * bw)),
            "samples_per_s_at_peak": samples_per_step() * HBM_PEAK_GBS * 1e9 /
                                     (WORDS_PER_UPDATE * bw * chain_updates_per_step(0)[1]),
            "stencil_exact": stencil_roofline(R * chain_stencil_words(0), bw, ml_run["ms_step"], R * samples_per_step())}
        del ml_run
        progress("cache-spilling roofline leg")
        ms_sp, iso_sp, tun_sp = roofline_leg(u1ml, torch, prec, SPILL_REPLICAS, 3, tune=tune)
        out["roofline_spilled"] = roofline_entry(u1ml, prec, SPILL_REPLICAS, ms_sp, N_BETWEEN, 3, iso_sp, tun_sp,
                                                 traffic_from_profiles(kname, SPILL_REPLICAS, bw))
        progress("streaming references")
        out["device_stream"] = stream_bandwidth(u1ml)
        cp = out["device_stream"]
        out["roofline"]["frac_of_cache_resident_read"] = out["roofline"]["achieved"] / cp["read_cache_resident_GB_per_s"]
        out["roofline_spilled"]["frac_of_hbm_read"] = out["roofline_spilled"]["achieved"] / cp["read_GB_per_s"]
        progress("precision split")
        out["precision_split"] = precision_leg()
        progress("uneven batch")
        out["uneven_64"] = uneven_leg(u1ml, torch, 10, tune=tune)
        progress("48^4 lattice")
        out["large_48"] = large_leg(u1ml, torch, n_therm=200)
    if not args.no_compare:
        # one chain (no batching), FP32 path and plain FP64 path
        progress("single-chain legs")
        legs = {}
        for name, pr in (("single_chain_fp32", u1ml.FP32), ("single_chain_fp64", u1ml.FP64)):
            r = run_chain(u1ml, torch, pr, 1, rf, 1, 1, tune=False)
            legs[name] = {"updates_per_s": r["updates_per_s"], "samples_per_s": r["samples_per_s"],
                          "ms_per_step": r["ms_step"], "phase_ms": {"sweeps": r["ms_sweeps"], "multilevel": r["ms_ml"]}}
            del r
        legs["speedup_vs_single_chain_fp64"] = out["value"] / legs["single_chain_fp64"]["updates_per_s"]
        out["compare"] = legs
    if not args.no_cpu:
        progress("CPU oracle")
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
