"""Locality of the overlap operator (section 2.2, Eq. 12 and Fig. 1): the mean absolute entry
of the blocks D_ov(x, . ; y, .) from smpq_dov_locality, averaged over the sites at one
distance from y (Euclidean and taxi-driver, minimum image on the torus), and the decay rate
gamma from a least-squares fit of log(shell mean) against the distance for distances >= 3.

    python -m paper_1901_02211_amd.locality --workload flux8 [--site 0] [--fp64] [--json out.json]
"""
import argparse
import json

import numpy as np

from . import binding as smpq

KAPPA, TOL, POLES, RELIABLE = 0.21, 1e-12, 14, 50


def site_distances(dims, site):
    """(Euclidean, taxi-driver) minimum-image distances of every site from `site`; sites are
    numbered x + nx (y + ny (z + nz t))."""
    V = int(np.prod(dims))
    idx = np.arange(V)
    coords = []
    for n in dims:
        coords.append(idx % n)
        idx = idx // n
    c = np.stack(coords, axis=1)
    d = np.abs(c - c[site])
    d = np.minimum(d, np.asarray(dims) - d)
    return np.sqrt((d * d).sum(axis=1)), d.sum(axis=1).astype(float)


def shells(values, dist):
    """Distinct distances (ascending), the mean of `values` over each shell and its size."""
    key = np.round(dist, 9)
    u, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
    sums = np.bincount(inv, weights=values)
    return u, sums / cnt, cnt


def fit_decay(d, mean, dmin=3.0):
    """Least-squares slope and intercept of log(mean) against d over d >= dmin: mean ~
    exp(intercept + slope d), so gamma = -slope."""
    sel = (d >= dmin) & (mean > 0)
    if sel.sum() < 2:
        return float("nan"), float("nan")
    slope, icpt = np.polyfit(d[sel], np.log(mean[sel]), 1)
    return float(slope), float(icpt)


def profile(ctx, dims, site=0, dmin=3.0):
    m, st = smpq.smpq_dov_locality(ctx, site)
    eu, tx = site_distances(dims, site)
    out = dict(site=site, iterations=st["total_iters"], seconds=st["t_solve_s"])
    for name, dist in (("euclid", eu), ("taxi", tx)):
        d, mean, cnt = shells(m, dist)
        slope, icpt = fit_decay(d, mean, dmin)
        out[name] = dict(distance=d.tolist(), mean=mean.tolist(), count=cnt.tolist(), gamma=-slope, log_c=icpt)
    return out


def main():
    import smpq_inputs as si

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="flux8")
    ap.add_argument("--site", type=int, default=0)
    ap.add_argument("--fp64", action="store_true")
    ap.add_argument("--json", default=None)
    args = ap.parse_args()
    w = si.WORKLOADS[args.workload]
    dims = w["dims"]
    c = smpq.smpq_create(dims, 0)
    smpq.smpq_load_gauge(c, si.workload(args.workload))
    smpq.smpq_set_zolotarev(c, POLES, *smpq.smpq_estimate_bounds(c, 300))
    prec = smpq.SMPQ_FP64 if args.fp64 else smpq.SMPQ_MIXED_FP32
    smpq.smpq_set_solver(c, prec, TOL, 10000, RELIABLE if prec == smpq.SMPQ_MIXED_FP32 else 0)
    res = profile(c, dims, args.site)
    print(f"### locality of D_ov: {args.workload} {dims}, source site {args.site}, "
          f"{'FP64' if args.fp64 else 'mixed FP32'}\n")
    for name in ("euclid", "taxi"):
        r = res[name]
        print(f"{name}: gamma = {r['gamma']:.3f} (fit of log mean over distance >= 3)")
        print("| distance | sites | mean abs entry |\n|---|---|---|")
        for d, m, n in zip(r["distance"], r["mean"], r["count"]):
            print(f"| {d:.3f} | {n} | {m:.3e} |")
        print()
    if args.json:
        with open(args.json, "w") as f:
            json.dump(dict(workload=args.workload, **res), f, indent=1)


if __name__ == "__main__":
    main()
