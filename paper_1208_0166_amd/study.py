"""Reduced-statistics physics runs of the paper's measurements (Sec. 3) on
the GPU, analysed on the host.

    python -m paper_1208_0166_amd.study potential [--replicas 16] [--n1 10] [--n2 100] ...
    python -m paper_1208_0166_amd.study width [--replicas 8] [--n1 10] [--n2 100] ...

The defaults are reduced statistics (10 x 100 iterations per configuration,
500 thermalisation sweeps); the paper's are --n1 100 --n2 1000.

``potential``: independent chains at 24^4, beta = 1 (cold start, thermalised),
one two-level multilevel run per configuration (slabs 4 and 2, analytical
multihit for r >= 2), V(r) of Eq. (4) with jackknife errors over the
configurations, and the fit of Eq. (1) with the Luscher coefficient fixed to
pi/12 and free (the paper fits without its first two points).

``width``: the same chains with the E_x insertion at r = 2, 4, 6; the
connected profile of Eq. (7) in the mediator plane, the ansatz of Eq. (10)
and the squared width of Eq. (2), with jackknife errors.

Both print one progress line per configuration and a JSON summary, and write
the summary to --out if given.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import analysis as an
from . import u1ml


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _chains(args):
    prec = u1ml.FP32 if args.prec == "fp32" else u1ml.FP64
    R = args.replicas
    b = u1ml.batch_create([args.L] * R, [args.L] * R, [args.beta] * R, [args.seed + i for i in range(R)],
                          start=u1ml.HOT if args.start == "hot" else u1ml.COLD, precision=prec)
    t0 = time.time()
    for _ in range(args.therm):
        u1ml.batch_sweep(b, 1, 3)
    u1ml.batch_synchronize(b)
    obs = [u1ml.batch_measure(b, i, correlator=False)[0]["plaquette"] for i in range(R)]
    _say(f"[study] {R} chains of {args.L}^4 beta={args.beta} {args.prec}, {args.start} start: {args.therm} "
         f"thermalisation sweeps in {time.time() - t0:.1f} s, plaquette {np.mean(obs):.5f} +- {np.std(obs):.5f}")
    return b


def potential_study(args):
    b = _chains(args)
    u1ml.batch_set_estimator(b, multihit=not args.no_multihit)
    r_list = list(range(1, args.L // 2 + 1))
    corrs = []
    t0 = time.time()
    for cfg in range(args.configs):
        if cfg:
            for _ in range(args.between):
                u1ml.batch_sweep(b, 1, 3)
        u1ml.batch_multilevel(b, [4, 2], [args.n1, args.n2], 1, 3, r_list)
        for i in range(args.replicas):
            _, c, _ = u1ml.batch_measure(b, i, correlator=True)
            corrs.append(c.real)
        _say(f"[study] configuration round {cfg + 1}/{args.configs}: {len(corrs)} configurations, "
             f"{time.time() - t0:.1f} s")
    corrs = np.array(corrs)
    n_t = args.L
    V, dV, _ = an.jackknife(corrs, lambda m: an.potential(m, n_t))
    # fit range: from r = 3 (the paper drops the first two points) while the
    # correlator is determined to better than 20 %
    _, dC, _ = an.jackknife(corrs)
    Cm = corrs.mean(axis=0)
    ok = [k for k, r in enumerate(r_list) if r >= args.rmin and Cm[k] > 0 and dC[k] < 0.2 * Cm[k]]
    rmax = r_list[ok[-1]] if ok else None
    sel = [k for k in ok if r_list[k] <= rmax]
    r_fit = np.array([r_list[k] for k in sel], dtype=float)
    fits = {}
    for name, c in (("luscher_fixed", an.luscher_coefficient(4)), ("luscher_free", None)):
        if len(r_fit) > (2 if c is not None else 3):
            f = an.fit_potential(r_fit, V[sel], dV[sel], c=c)
            fits[name] = {k: float(v) for k, v in f.items()}
            # jackknife error of sigma (correlated points): refit every
            # leave-one-out sample with the same weights
            _, err, _ = an.jackknife(corrs, lambda m: np.array(
                [an.fit_potential(r_fit, an.potential(m, n_t)[sel], dV[sel], c=c)["sigma"]]))
            fits[name]["d_sigma_jackknife"] = float(err[0])
    return {
        "study": "potential", "L": args.L, "beta": args.beta, "precision": args.prec, "start": args.start,
        "therm": args.therm, "between": args.between,
        "configurations": int(corrs.shape[0]), "n1": args.n1, "n2": args.n2, "multihit": not args.no_multihit,
        "r": r_list, "C": Cm.tolist(), "dC": dC.tolist(), "V": V.tolist(), "dV": dV.tolist(),
        "fit_r": r_fit.tolist(), "fits": fits, "seconds": time.time() - t0,
    }


def width_study(args):
    b = _chains(args)
    rf = [2, 4, 6]
    r_list = list(range(1, max(rf) + 1))
    u1ml.batch_set_estimator(b, multihit=not args.no_multihit)
    profiles = {r: [] for r in rf}
    corrs, omeans = [], []
    t0 = time.time()
    for cfg in range(args.configs):
        if cfg:
            for _ in range(args.between):
                u1ml.batch_sweep(b, 1, 3)
        u1ml.batch_multilevel(b, [4, 2], [args.n1, args.n2], 1, 3, r_list, rf_list=rf)
        for i in range(args.replicas):
            obs, c, f = u1ml.batch_measure(b, i, correlator=True, field_profile=True)
            for j, r in enumerate(rf):
                profiles[r].append(f[j])
            corrs.append(c)
            omeans.append(obs["field_mean"])
        _say(f"[study] configuration round {cfg + 1}/{args.configs}: {len(corrs)} configurations, "
             f"{time.time() - t0:.1f} s")
    corrs = np.array(corrs)
    out = {"study": "width", "L": args.L, "beta": args.beta, "precision": args.prec,
           "configurations": int(corrs.shape[0]), "n1": args.n1, "n2": args.n2, "multihit": not args.no_multihit,
           "rows": []}
    for r in rf:
        k = r_list.index(r)
        row = {"r": r}
        # mean connected E_x profile over the mediator plane (planes averaged)
        conn = an.connected_part(np.mean(profiles[r], axis=0), corrs[:, k].mean(), np.mean(omeans, axis=0))
        row["profile_Ex"] = np.mean(conn[:, 0], axis=0).tolist()
        for dims in (2, 1):
            try:
                w2, err, p = an.flux_tube_width(profiles[r], corrs[:, k], omeans, comp=0, dims=dims)
                row.update({f"w2_{dims}d": w2, f"dw2_{dims}d": err, "ansatz": [float(x) for x in p]})
            except (RuntimeError, ValueError) as e:  # fit did not converge at this statistics
                row[f"error_{dims}d"] = str(e)
        out["rows"].append(row)
    out["seconds"] = time.time() - t0
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("study", choices=["potential", "width"])
    ap.add_argument("--replicas", type=int, default=None)
    ap.add_argument("--configs", type=int, default=1, help="multilevel configurations per chain")
    ap.add_argument("--n1", type=int, default=None)
    ap.add_argument("--n2", type=int, default=None)
    ap.add_argument("--L", type=int, default=24)
    ap.add_argument("--beta", type=float, default=1.0)
    ap.add_argument("--therm", type=int, default=500)
    ap.add_argument("--start", choices=["cold", "hot"], default="cold")
    ap.add_argument("--between", type=int, default=100)
    ap.add_argument("--seed", type=int, default=3000)
    ap.add_argument("--rmin", type=int, default=3)
    ap.add_argument("--prec", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--no-multihit", action="store_true")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    # reduced statistics by default (a physics smoke run of a few seconds);
    # the paper's production statistics are 100 level-1 x 1000 level-2
    # iterations per configuration (--n1 100 --n2 1000)
    defaults = {"potential": (16, 10, 100), "width": (8, 10, 100)}[args.study]
    args.replicas = args.replicas or defaults[0]
    args.n1 = args.n1 or defaults[1]
    args.n2 = args.n2 or defaults[2]
    res = potential_study(args) if args.study == "potential" else width_study(args)
    line = json.dumps(res)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(line + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
