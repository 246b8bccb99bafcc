"""Benchmark: multilevel compact U(1) on a 24^4 lattice at beta = 1 on one MI355X.

One step is one pass of the whole method over the 24^4 lattice:
  * 100 compound sweeps (1 Metropolis hit + 3 overrelaxation passes per link)
    between measured configurations (Sec. 2.1);
  * one two-level multilevel measurement (Sec. 2.2): slabs of 4 (10 updates)
    holding slabs of 2 (20 updates), Polyakov correlators for r = 1..12 along
    x, and the E/B field profiles (Eq. (5), Eq. (9)) over the 24^2 planes at
    the mid-point of charges at r = 2, 4, 6;
  * the plain observables and the read-back of all results.
The lattice is synthetic (cold start + 200 thermalisation sweeps, seed 3).

Printed: one JSON line with link updates/s of the Markov chain (the replay of
the update sequence that the field insertion needs is not counted as
updates), multilevel samples/s (one sample = one innermost-slab update
followed by its two-link measurement for all L^3 sources and all r), the
roofline of the dominant kernel and the CPU oracle timed on this host.
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
WORDS_PER_UPDATE = 9  # 8 link reads + 1 write per update in a class pass


def chain_updates_per_step():
    V = L ** 3 * T
    sweeps = N_BETWEEN * 4 * (4 * V)            # 4 passes (1 Metropolis + 3 OR) over 4V links
    free1 = 4 * V - (T // LEVELS[0]) * 3 * L ** 3
    free2 = 4 * V - (T // LEVELS[1]) * 3 * L ** 3
    ml = N_SUB[0] * 4 * free1 + N_SUB[0] * N_SUB[1] * 4 * free2
    return sweeps, ml


def samples_per_step():
    return N_SUB[0] * N_SUB[1] * (T // LEVELS[-1])


def sweep_sources_sha():
    h = hashlib.sha256()
    for f in ("sweep_impl.h", "device_common.h", "sweep_f32.hip", "sweep_f64.hip"):
        with open(os.path.join(ROOT, "paper_1208_0166_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_key):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(p) as f:
            d = json.load(f)
        e = d.get(kernel_key)
        if e and e.get("sources_sha") == sweep_sources_sha():
            return e["bytes_per_launch"]
    except (OSError, ValueError):
        pass
    return None


def cpu_baseline(seconds: float):
    """The FP64 oracle on this host: compound sweeps of the 24^4 lattice for
    about `seconds`, and one reduced multilevel run for samples/s."""
    import oracle
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
    o.multilevel(LEVELS, [1, 2], 1, 3, R_LIST)
    el_ml = time.perf_counter() - t0
    samp = 1 * 2 * (T // LEVELS[-1])
    return {"value": ups, "unit": "link updates/s", "cores": oracle.max_threads(), "kind": "oracle",
            "samples_per_s": samp / el_ml,
            "sample": f"{n} compound sweeps (1 Metropolis + 3 OR) of 24^4 FP64 in {el:.1f} s; "
                      f"multilevel levels {LEVELS} with n_sub [1, 2], r = 1..12 ({samp} samples) in {el_ml:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--no-field", action="store_true", help="skip the field-profile insertion")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--fp64-compare", action="store_true", help="also time one step of the FP64 path")
    ap.add_argument("--replicas", type=int, default=1,
                    help="independent 24^4 chains advanced by the same launches (one batch)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1208_0166_amd import u1ml

    torch.cuda.set_device(0)
    # a dedicated stream: the library queues its kernels on torch's current
    # stream, and the events below are recorded on the same one
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    prec = u1ml.FP32 if args.precision == "fp32" else u1ml.FP64
    rf = [] if args.no_field else RF_LIST

    R = args.replicas

    def make(pr):
        if R == 1:
            lat = u1ml.init_lattice(L, T, BETA, 3, start=u1ml.COLD, precision=pr)
            sw = lambda: u1ml.sweep(lat, 1, 3)  # noqa: E731
        else:
            lat = u1ml.batch_create([L] * R, [T] * R, [BETA] * R, [3 + i for i in range(R)], start=u1ml.COLD,
                                    precision=pr, stream=stream.cuda_stream)
            sw = lambda: u1ml.batch_sweep(lat, 1, 3)  # noqa: E731
        for _ in range(N_THERM):
            sw()
        torch.cuda.synchronize()
        return lat, sw

    lat, sw = make(prec)

    def step(lt, swf, ev=None):
        if ev:
            ev[0].record(stream)
        for _ in range(N_BETWEEN):
            swf()
        if ev:
            ev[1].record(stream)
        if R == 1:
            u1ml.multilevel(lt, LEVELS, N_SUB, 1, 3, R_LIST, rf_list=rf)
        else:
            u1ml.batch_multilevel(lt, LEVELS, N_SUB, 1, 3, R_LIST, rf_list=rf)
        if ev:
            ev[2].record(stream)
        if R == 1:
            return u1ml.measure(lt, correlator=True, field_profile=bool(rf))
        res = [u1ml.batch_measure(lt, i, correlator=True, field_profile=bool(rf)) for i in range(R)]
        return res[0]

    for _ in range(args.warmup):
        step(lat, sw)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        obs, corr, field = step(lat, sw, evs[k])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_sweeps = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps
    ms_ml = sum(e[1].elapsed_time(e[2]) for e in evs) / args.steps

    up_sw, up_ml = chain_updates_per_step()
    up_sw, up_ml = up_sw * R, up_ml * R
    ms_step = 1e3 * el / args.steps
    value = (up_sw + up_ml) * args.steps / el
    samples = samples_per_step() * R

    # dominant kernel: the FP32/FP64 overrelaxation class pass on the full lattice
    prof_lat = lat if R == 1 else u1ml.init_lattice(L, T, BETA, 3, start=u1ml.COLD, precision=prec)
    us_metro, us_or = u1ml.profile_sweeps(prof_lat, 20, 1, 3)
    bw = 4 if prec == u1ml.FP32 else 8
    updates_per_launch = L ** 3 * T // 2
    bytes_per_launch = updates_per_launch * WORDS_PER_UPDATE * bw
    achieved = bytes_per_launch / (us_or * 1e-6) / 1e9
    kname = f"class_pass_kernel<{'Fast32' if prec == u1ml.FP32 else 'Det64'}, OR>"
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_profiles(kname),
                "kernel": kname, "avg_us": us_or, "metropolis_avg_us": us_metro,
                "algorithmic_bytes_per_launch": bytes_per_launch}

    out = {
        "metric": "link updates/s (Metropolis+OR) and multilevel correlator samples/s, 24^4 beta=1",
        "value": value,
        "unit": "link updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == u1ml.FP32 else "f64",
        "data": "synthetic (cold start, 200 thermalisation sweeps, seed 3)",
        "config": {"workload": "24^4 beta=1: 100 sweeps(1 Metropolis + 3 OR) + two-level multilevel "
                               "{4,2} x {10,20}, r=1..12, E/B mid-plane profiles at r=2,4,6",
                   "lattice": [L, L, L, T], "beta": BETA, "levels": LEVELS, "n_sub": N_SUB,
                   "r": [1, 12], "field_r": rf, "accumulate": "f64", "replicas": R},
        "samples_per_s": samples / (ms_ml * 1e-3),
        "samples_per_step": samples,
        "chain_updates_per_step": up_sw + up_ml,
        "phase_ms": {"sweeps": ms_sweeps, "multilevel": ms_ml, "measure_and_readback": ms_step - ms_sweeps - ms_ml},
        "sweep_updates_per_s": up_sw / (ms_sweeps * 1e-3),
        "multilevel_chain_updates_per_s": up_ml / (ms_ml * 1e-3),
        "plaquette": obs["plaquette"],
        "poly_abs": obs["poly_abs"],
        "C_r1": [corr[0].real, corr[0].imag],
        "roofline": roofline,
    }
    if args.fp64_compare and prec == u1ml.FP32:
        lat64, sw64 = make(u1ml.FP64)
        step(lat64, sw64)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        step(lat64, sw64)
        torch.cuda.synchronize()
        el64 = time.perf_counter() - t1
        out["fp64_path"] = {"ms_per_step": 1e3 * el64, "link_updates_per_s": (up_sw + up_ml) / el64,
                            "fp32_speedup": el64 / (el / args.steps)}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
