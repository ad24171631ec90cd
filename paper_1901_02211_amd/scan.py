"""Probing-scheme scan (section 3, Tables 1-3 and Fig. 8): for one gauge field, the exact
density q(x) from the point-source trace (Eq. 5) and, for every SMP scheme (gap r, mode), the
estimate q^P(x) of Eq. 16 with its number of sources, its r_min (Eq. 18) and its errors
|Q^P - Q| and max / rms |q^P(x) - q(x)|.  With --quantity trinv the same for the trace density
of D_W^-1 (the application proposed in the Conclusion).  Every solve runs through the library.

    python -m paper_1901_02211_amd.scan --workload flux8 [--no-gauge | --gauge-seed S]
        [--gaps 2 4 8] [--fp64] [--quantity qx|trinv] [--json out.json]
"""
import argparse
import json
import sys
import time

import numpy as np

from . import binding as smpq

KAPPA, TOL, POLES, RELIABLE = 0.21, 1e-12, 14, 50


def _density(c, quantity):
    """(real density, imaginary part, iterations) of the current scheme."""
    if quantity == "trinv":
        t, st = smpq.smpq_compute_trinv(c)
        return t.real, t.imag, st["total_iters"]
    q, qi, _, st = smpq.smpq_compute_qx(c)
    return q, qi, st["total_iters"]


def scan(U, dims, gaps=(2, 4, 8), modes=(0, 1, 2), precision=smpq.SMPQ_MIXED_FP32, tol=TOL, quantity="qx"):
    """Returns {"Q_exact", "n_point_sources", "interval", "rows": [...]}; one row per valid
    (r, mode), r the same in all four directions, ordered by number of sources.  quantity
    "qx": the charge density (Q = sum q); "trinv": tr_sc D_W^-1(x, x) (Q = Tr D_W^-1)."""
    c = smpq.smpq_create(dims, 0)
    smpq.smpq_load_gauge(c, U)
    lo = hi = None
    if quantity == "qx":
        lo, hi = smpq.smpq_estimate_bounds(c, 300)
        smpq.smpq_set_zolotarev(c, POLES, lo, hi)
    smpq.smpq_set_solver(c, precision, tol, 10000, RELIABLE if precision == smpq.SMPQ_MIXED_FP32 else 0)
    smpq.smpq_autotune(c, 48)
    t0 = time.perf_counter()
    _, n_pt = smpq.smpq_set_point_scheme(c)
    print(f"scan: exact density from {n_pt} point sources", file=sys.stderr, flush=True)
    q_ex, _, _ = _density(c, quantity)
    Q_ex = float(q_ex.sum())
    t_ex = time.perf_counter() - t0
    rows = []
    for r in gaps:
        for mode in modes:
            try:
                ncls, nsrc = smpq.smpq_set_scheme(c, (r,) * 4, mode)
            except smpq.SmpqError:
                continue            # r does not divide the lattice, or the mode's condition fails
            rmin, nearest = smpq.smpq_get_scheme_rmin(c)
            print(f"scan: r = {r}, mode {mode}, {nsrc} sources", file=sys.stderr, flush=True)
            t0 = time.perf_counter()
            q, qi, iters = _density(c, quantity)
            Q = float(q.sum())
            dq = q - q_ex
            rows.append(dict(r=r, mode=mode, r_min=rmin, nearest=nearest, n_classes=ncls, n_sources=nsrc,
                             sources_over_point=nsrc / n_pt, Q=Q, abs_dQ=abs(Q - Q_ex),
                             max_abs_dq=float(np.abs(dq).max()), rms_dq=float(np.sqrt(np.mean(dq ** 2))),
                             max_abs_imag_q=float(np.abs(qi).max()), seconds=time.perf_counter() - t0,
                             iterations=iters))
    rows.sort(key=lambda row: row["n_sources"])
    return dict(quantity=quantity, Q_exact=Q_ex, n_point_sources=n_pt, seconds_exact=t_ex, interval=(lo, hi),
                rows=rows)


def markdown(res, title):
    name = "Q" if res["quantity"] == "qx" else "Tr D_W^-1"
    interval = "" if res["interval"][0] is None else \
        f"; Zolotarev interval [{res['interval'][0]:.4f}, {res['interval'][1]:.4f}]"
    out = [f"### {title}", "",
           f"Exact {name} = {res['Q_exact']:.6f} from {res['n_point_sources']} point sources "
           f"({res['seconds_exact']:.1f} s){interval}.",
           "", "| r | mode | r_min | nearest | N_src | N_src/N_pt | estimate | abs(error) | max abs(dq) | rms dq | s |",
           "|---|---|---|---|---|---|---|---|---|---|---|"]
    for w in res["rows"]:
        out.append(f"| {w['r']} | {w['mode']} | {w['r_min']:.3f} | {w['nearest']} | {w['n_sources']} | "
                   f"{w['sources_over_point']:.4f} | {w['Q']:.5f} | {w['abs_dQ']:.2e} | {w['max_abs_dq']:.2e} | "
                   f"{w['rms_dq']:.2e} | {w['seconds']:.1f} |")
    return "\n".join(out)


def main():
    import smpq_inputs as si

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="flux8")
    ap.add_argument("--no-gauge", action="store_true", help="leave out the workload's random gauge transform")
    ap.add_argument("--gauge-seed", type=int, default=None, help="apply a Haar gauge transform with this seed")
    ap.add_argument("--gaps", type=int, nargs="+", default=[2, 4, 8])
    ap.add_argument("--fp64", action="store_true")
    ap.add_argument("--quantity", default="qx", choices=["qx", "trinv"])
    ap.add_argument("--json", default=None)
    args = ap.parse_args()
    w = si.WORKLOADS[args.workload]
    U = si.workload(args.workload, gauge=not args.no_gauge, gauge_seed=args.gauge_seed)
    res = scan(U, w["dims"], args.gaps, precision=smpq.SMPQ_FP64 if args.fp64 else smpq.SMPQ_MIXED_FP32,
               quantity=args.quantity)
    gauge = "no gauge transform" if args.no_gauge or (args.gauge_seed is None and "gauge_seed" not in w) else \
        f"Haar gauge transform seed {args.gauge_seed if args.gauge_seed is not None else w['gauge_seed']}"
    what = "q(x)" if args.quantity == "qx" else "tr D_W^-1(x,x)"
    print(markdown(res, f"{what}: {args.workload} {w['dims']}, {gauge}, {'FP64' if args.fp64 else 'mixed FP32'}"),
          flush=True)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(dict(workload=args.workload, gauge=gauge, **res), f, indent=1)


if __name__ == "__main__":
    main()
