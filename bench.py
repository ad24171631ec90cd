"""Benchmark: seconds per q(x) map on one MI355X, mixed precision vs plain FP64.

Default workload: 16^3 x 32 periodic lattice, near-identity SU(3) links (eps = 0.2, seed 4),
kappa = 0.21, 14-pole Zolotarev sign function on Lanczos bounds, SMP normal mode with
r = 4 (256 classes x 12 = 3072 sources), per-shift CG tolerance 1e-12.  One step is one
whole q(x) map: Lanczos bounds + Zolotarev + every multi-shift CG solve + contraction +
copy-out of q(x) and Q, with the gauge field already resident in HBM.  The map runs in
FP32 with FP64 reliable updates every 50 iterations and FP64 accumulation.

--workload selects another lattice of the same family (24^3x48 flux, 16^4, 24^4, 32^3x64);
maps that take minutes are timed on a sample of classes and the value is extrapolated by
classes/sample (labelled "extrapolated").  --workload uneven times 16^4 + 24^4 + 32^3x64
together, the same fraction of classes of each, concurrently (one stream per lattice) and
one after another; --workload ensemble does the same for eight whole 8^4 maps.

Defaults: 3 steps (maps), no warmup; value = their mean (median_s and step_s beside it).
Printed: one JSON line.  value = seconds per map (lower is better).  Beside it:
  roofline      the dominant kernel of the step (HIP events on the library's stream),
                algorithmic bytes per launch / mean launch duration vs 8 TB/s
  dslash        the Wilson stencil in situ and standalone (rotating buffers > 1 GB)
  fp64          the plain FP64 GPU path on a sample of classes, scaled to a map
  accuracy      mixed vs FP64 GPU on the sample; |Q - round(Q)| of the map
  cpu_baseline  the FP64 numpy oracle on a bounded sample (single thread), scaled
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KAPPA, TOL, POLES, RELIABLE = 0.21, 1e-12, 14, 50
# workload -> gap r, default sample of classes (0 = whole map), FP64 comparison classes, description
BENCH = {
    "noise16x32": (4, 0, 16, "16^3x32 near-identity SU(3) eps=0.2 seed 4, SMP normal mode r=4"),
    "flux24x48": (6, 24, 6, "24^3x48 U(1) flux (1,1) x near-identity eps=0.15 seed 5, SMP normal mode r=6"),
    "noise16": (4, 0, 16, "16^4 near-identity SU(3) eps=0.1 seed 6, SMP normal mode r=4"),
    "noise24": (6, 48, 12, "24^4 near-identity SU(3) eps=0.2 seed 7, SMP normal mode r=6"),
    "noise32x64": (8, 16, 4, "32^3x64 near-identity SU(3) eps=0.3 seed 8, SMP normal mode r=8"),
    "rough8": (4, 0, 16, "8^4 near-identity eps=0.3 seed 60 with a Haar-random 3^4 block, SMP normal mode r=4"),
}
UNEVEN = ("noise16", "noise24", "noise32x64")
# storage of the shifted search directions in the mixed path -> precision, label
DIR_STORAGE = {"fp32": ("SMPQ_MIXED_FP32", ""),
               "fp16": ("SMPQ_MIXED_FP16DIR", "; shifted search directions stored in FP16 (scaled)"),
               "bf16": ("SMPQ_MIXED_BF16DIR", "; shifted search directions stored in BF16")}


def kernel_source_hash():
    """Hash of the device code (kernels.hip and wilson_site.h without comments and blank
    lines), so that profiles/traffic.json is used only for the kernels it was measured on."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "wilson_site.h"):
        with open(os.path.join(ROOT, "paper_1901_02211_amd", "csrc", f)) as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """Counter-measured HBM bytes / algorithmic bytes of a kernel, from the committed summary,
    if it was measured on the current kernel source and this workload."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    if data.get("workload") != workload:
        return None
    entry = data.get(kernel)
    if not entry or entry.get("kernel_hash") != kernel_source_hash():
        return None
    return entry


def cpu_baseline(workload, dims, r_gap, total_iters, n_sources, iters_sample):
    """Time the oracle's multi-shift CG on one source of the workload for a bounded number of
    iterations in a single-threaded subprocess; scale by the map's measured iteration count."""
    code = f"""
import os, sys, time
sys.path.insert(0, {ROOT!r})
import numpy as np
import smpq_inputs as si
from oracle.lattice import Lattice
from oracle.dirac import apply_h2
from oracle.mscg import multishift_cg, NotConverged
from oracle.lanczos import bounds
from oracle.zolotarev import zolotarev
from oracle.probing import colouring
U = si.workload({workload!r}); lat = Lattice({tuple(dims)!r})
col, _ = colouring(lat, ({r_gap},) * 4, 0)
b = np.zeros((lat.volume, 4, 3), dtype=np.complex128); b[col == 0, 0, 0] = 1.0
c0, c, q, _ = zolotarev({POLES}, 0.14, 2.73)
s = q.min()
from oracle.dirac import apply_dw
t0 = time.perf_counter()
apply_dw(U, lat, {KAPPA}, b)
t_dw = time.perf_counter() - t0
t0 = time.perf_counter()
try:
    multishift_cg(lambda v: apply_h2(U, lat, {KAPPA}, v) + s * v, b, q - s, {TOL}, {iters_sample})
except NotConverged:
    pass
print(t_dw, time.perf_counter() - t0)
"""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    if out.returncode != 0:
        raise RuntimeError(out.stderr)
    t_dw, t = (float(x) for x in out.stdout.strip().splitlines()[-1].split())
    per_iter = t / iters_sample
    V = int(np.prod(dims))
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": per_iter * total_iters, "unit": "s/map", "cores": 1, "kind": "oracle",
            "host_cpu": cpu_model, "host_nproc": os.cpu_count(),
            "oracle_dw_ns_per_site": 1e9 * t_dw / V,
            "oracle_dw_GBs": V * (72 + 48) * 8 / t_dw / 1e9,
            "sample": f"{iters_sample} multi-shift CG iterations of one r={r_gap} source on the {workload} field "
                      f"({t:.1f} s), scaled by the map's {total_iters} iterations over {n_sources} sources",
            "seconds_per_iteration": per_iter}


def uneven(args, smpq, si):
    """16^4 + 24^4 + 32^3x64 together: the same fraction of the classes of each lattice, solved
    concurrently (smpq_compute_qx_multi) and one after another; both scaled to whole maps."""
    frac = 1.0 / 256 if args.classes < 0 else 1.0 / max(1, args.classes)
    ctxs, plan = [], []
    for name in UNEVEN:
        r = BENCH[name][0]
        print(f"bench: building {name}", file=sys.stderr, flush=True)
        c = smpq.smpq_create(si.WORKLOADS[name]["dims"], 0)
        smpq.smpq_load_gauge(c, si.workload(name))
        ncls, _ = smpq.smpq_set_scheme(c, (r,) * 4, 0)
        smpq.smpq_set_solver(c, smpq.SMPQ_MIXED_FP32, TOL, 10000, RELIABLE)
        smpq.smpq_set_zolotarev(c, POLES, *smpq.smpq_estimate_bounds(c, 300))
        smpq.smpq_autotune(c, 48)
        k = max(1, round(ncls * frac))
        ctxs.append(c)
        plan.append((name, ncls, list(range(k))))
    for c, (_, _, cl) in zip(ctxs, plan):   # untimed: workspaces, graphs, first launches
        smpq.smpq_compute_qx_classes(c, cl[:1])
    t0 = time.perf_counter()
    seq = [smpq.smpq_compute_qx_classes(c, cl) for c, (_, _, cl) in zip(ctxs, plan)]
    t_seq = time.perf_counter() - t0
    print(f"bench: one after another {t_seq:.2f} s", file=sys.stderr, flush=True)
    smpq.smpq_compute_qx_multi(ctxs, [cl[:1] for _, _, cl in plan])
    t0 = time.perf_counter()
    par = smpq.smpq_compute_qx_multi(ctxs, [cl for _, _, cl in plan])
    t_par = time.perf_counter() - t0
    print(f"bench: concurrent {t_par:.2f} s", file=sys.stderr, flush=True)
    same = all(np.array_equal(a[0], b[0]) for a, b in zip(seq, par))
    scale = sum(n for _, n, _ in plan) / sum(len(cl) for _, _, cl in plan)
    line = {
        "metric": "sec per set of q(x) maps (16^4 + 24^4 + 32^3x64), concurrent",
        "value": round(t_par * scale, 3), "unit": "s/set", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(1000 * t_par * scale, 1), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "16^4 r=4 + 24^4 r=6 + 32^3x64 r=8, near-identity SU(3), mixed precision",
                   "lattices": {n: {"classes_timed": len(cl), "classes_per_map": nc,
                                    "sources_timed": 12 * len(cl),
                                    "iterations": st[2]["total_iters"], "batches": st[2]["n_batches"]}
                                for (n, nc, cl), st in zip(plan, par)},
                   "extrapolated": True, "fraction_of_each_map": frac},
        "sequential_s_per_set": round(t_seq * scale, 3),
        "concurrent_over_sequential": round(t_par / t_seq, 4),
        "results_identical": same,
    }
    print(json.dumps(line), flush=True)


def ensemble(args, smpq, si):
    """Eight 8^4 near-identity fields (eps 0.3, seeds 10-17), SMP r = 2 (192 sources each), whole
    maps: concurrently through smpq_compute_qx_multi and one after another.  Small lattices
    leave the GPU idle between short launches and host round trips; several contexts fill it."""
    dims, n = (8, 8, 8, 8), 8
    ctxs = []
    for k in range(n):
        c = smpq.smpq_create(dims, 0)
        smpq.smpq_load_gauge(c, si.near_identity_su3(dims, 0.3, 10 + k))
        smpq.smpq_set_scheme(c, (2,) * 4, 0)
        smpq.smpq_set_solver(c, smpq.SMPQ_MIXED_FP32, TOL, 10000, RELIABLE)
        smpq.smpq_set_zolotarev(c, POLES, *smpq.smpq_estimate_bounds(c, 300))
        ctxs.append(c)
    smpq.smpq_compute_qx_multi(ctxs)                 # untimed: workspaces, graphs
    for c in ctxs:
        smpq.smpq_compute_qx(c)
    t0 = time.perf_counter()
    seq = [smpq.smpq_compute_qx(c) for c in ctxs]
    t_seq = time.perf_counter() - t0
    t0 = time.perf_counter()
    par = smpq.smpq_compute_qx_multi(ctxs)
    t_par = time.perf_counter() - t0
    same = all(np.array_equal(a[0], b[0]) for a, b in zip(seq, par))
    line = {
        "metric": "sec per ensemble of eight 8^4 q(x) maps (r=2), concurrent",
        "value": round(t_par, 4), "unit": "s/ensemble", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(1000 * t_par, 2), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "8 x 8^4 near-identity SU(3) eps=0.3 seeds 10-17, SMP normal mode r=2, mixed precision",
                   "sources_per_map": seq[0][3]["n_sources"], "extrapolated": False},
        "sequential_s": round(t_seq, 4), "concurrent_over_sequential": round(t_par / t_seq, 4),
        "Q": [round(float(x[2]), 6) for x in seq], "results_identical": same,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="noise16x32", choices=sorted(BENCH) + ["uneven", "ensemble"])
    ap.add_argument("--fp64-classes", type=int, default=-1, help="classes in the FP64 comparison sample")
    ap.add_argument("--full-fp64", action="store_true", help="run the FP64 comparison as a whole map")
    ap.add_argument("--classes", type=int, default=-1,
                    help="time only the first N classes and extrapolate (0 = whole map)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=0)
    ap.add_argument("--deflate", type=int, default=0, help="deflate this many low modes of H_W^2 in each step")
    ap.add_argument("--deflate-steps", type=int, default=80)
    ap.add_argument("--dir-storage", default="fp32", choices=sorted(DIR_STORAGE),
                    help="storage of the shifted systems' search directions in the mixed path")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the probing sources would shard over GPUs with no communication in the solver loop)",
              file=sys.stderr)
        sys.exit(2)

    import paper_1901_02211_amd as smpq
    import smpq_inputs as si

    if args.workload == "uneven":
        return uneven(args, smpq, si)
    if args.workload == "ensemble":
        return ensemble(args, smpq, si)
    WORKLOAD = args.workload
    DIMS = si.WORKLOADS[WORKLOAD]["dims"]
    R_GAP, sample, fp64_default, desc = BENCH[WORKLOAD]
    if args.classes < 0:
        args.classes = sample
    if args.fp64_classes < 0:
        args.fp64_classes = fp64_default
    if args.cpu_iters <= 0:
        args.cpu_iters = max(2, round(8 * 131072 / int(np.prod(DIMS))))
    print(f"bench: building {WORKLOAD} {DIMS}", file=sys.stderr, flush=True)
    U = si.workload(WORKLOAD)
    ctx = smpq.smpq_create(DIMS, 0)
    smpq.smpq_load_gauge(ctx, U)                    # resident in HBM before any timed region
    ncls, nsrc = smpq.smpq_set_scheme(ctx, (R_GAP,) * 4, 0)
    prec_mixed = getattr(smpq, DIR_STORAGE[args.dir_storage][0])
    smpq.smpq_set_solver(ctx, prec_mixed, TOL, 10000, RELIABLE)
    classes = list(range(ncls if args.classes == 0 else min(args.classes, ncls)))
    scale = ncls / len(classes)             # extrapolation factor of a sampled map

    defl_info = {}

    def one_map():
        """One step: Lanczos bounds (or the deflated modes), Zolotarev coefficients and the whole
        q(x) map."""
        t0 = time.perf_counter()
        if args.deflate > 0:    # the lowest modes exactly; the interval above them
            theta, tmax, resid = smpq.smpq_deflate(ctx, args.deflate, args.deflate_steps)
            defl_info.update(theta=theta.tolist(), theta_max=tmax, max_resid=resid)
            lo, hi = 0.9 * np.sqrt(theta[-1]), 1.02 * np.sqrt(tmax)
        else:
            lo, hi = smpq.smpq_estimate_bounds(ctx, 300)
        smpq.smpq_set_zolotarev(ctx, POLES, lo, hi)
        t1 = time.perf_counter()
        if args.classes:
            q, qi, st = smpq.smpq_compute_qx_classes(ctx, classes)
            Q = float(q.sum())
        else:
            q, qi, Q, st = smpq.smpq_compute_qx(ctx)
        t2 = time.perf_counter()
        st["t_bounds_s"] = t1 - t0
        return t2 - t0, q, Q, st

    # untimed set-up: workspace allocation and first launches of every kernel
    smpq.smpq_set_zolotarev(ctx, POLES, 0.14, 2.73)
    tuning = smpq.smpq_autotune(ctx, 0)            # at the map's batch size
    print(f"bench: stencil variants {tuning}", file=sys.stderr, flush=True)
    smpq.smpq_prepare(ctx)
    smpq.smpq_compute_qx_classes(ctx, [0])
    smpq.smpq_set_timing(ctx, True)
    for w in range(args.warmup):
        print(f"bench: warmup step {w}", file=sys.stderr, flush=True)
        one_map()
    times, last = [], None
    for k in range(args.steps):
        dt, q, Q, st = one_map()
        times.append(dt)
        last = (q, Q, st)
        print(f"bench: step {k}: {dt:.2f} s, Q = {Q:.6f}, iters {st['total_iters']}, "
              f"batches {st['n_batches']}", file=sys.stderr, flush=True)
    q_mixed, Q, st = last
    ms_per_step = 1000.0 * float(np.mean(times)) * scale

    # kernels: dominant by in-situ time
    kern = {
        "dslash": dict(ms=st["dslash_ms"], bytes=st["dslash_bytes"], launches=st["dslash_launches"]),
        "shift_update": dict(ms=st["update_ms"], bytes=st["update_bytes"], launches=st["update_launches"]),
    }
    dom = max(kern, key=lambda k: kern[k]["ms"])
    kd = kern[dom]
    mean_ms = kd["ms"] / kd["launches"]
    bytes_launch = kd["bytes"] / kd["launches"]
    achieved = bytes_launch / (mean_ms * 1e-3) / 1e9
    tr = measured_traffic(dom, WORKLOAD)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": round(tr["traffic_over_algorithmic"] * bytes_launch) if tr else None,
                "traffic_over_algorithmic": tr["traffic_over_algorithmic"] if tr else None,
                "launch_ms": round(mean_ms, 4), "launches": kd["launches"],
                "algorithmic_bytes_per_launch": bytes_launch}
    map_GBs = (st["dslash_bytes"] + st["update_bytes"]) / (st["t_solve_s"]) / 1e9

    ds_insitu = st["dslash_bytes"] / (st["dslash_ms"] * 1e-3) / 1e9
    trd = measured_traffic("dslash", WORKLOAD)
    print("bench: standalone stencil", file=sys.stderr, flush=True)
    copy_ms = smpq.smpq_bench_copy(ctx, 1 << 31, 20)
    copy_GBs = 2.0 * (1 << 31) / (copy_ms * 1e-3) / 1e9
    ms32, by32 = smpq.smpq_bench_dslash(ctx, smpq.SMPQ_MIXED_FP32, 24, 4, 50)
    ms64, by64 = smpq.smpq_bench_dslash(ctx, smpq.SMPQ_FP64, 24, 4, 50)
    dslash = {"insitu_GBs": round(ds_insitu, 1), "insitu_frac": round(ds_insitu / HBM_PEAK_GBS, 4),
              "launches": st["dslash_launches"], "algorithmic_bytes": st["dslash_bytes"],
              "traffic_over_algorithmic": trd["traffic_over_algorithmic"] if trd else None,
              "standalone_fp32_n24_GBs": round(by32 / ms32 / 1e6, 1),
              "standalone_fp64_n24_GBs": round(by64 / ms64 / 1e6, 1),
              "standalone_note": "24 right-hand sides, 4 rotating input/output/link sets (> 1 GB)"}

    # plain FP64 GPU path on a sample of classes (or the whole map)
    print("bench: FP64 comparison", file=sys.stderr, flush=True)
    fcls = list(range(ncls)) if args.full_fp64 else list(range(min(args.fp64_classes, len(classes))))
    smpq.smpq_set_solver(ctx, smpq.SMPQ_FP64, TOL, 10000, 0)
    smpq.smpq_set_timing(ctx, False)
    t0 = time.perf_counter()
    q64, qi64, st64 = smpq.smpq_compute_qx_classes(ctx, fcls)
    t64 = time.perf_counter() - t0
    colour = smpq.smpq_get_coloring(ctx)
    mask = np.isin(colour, fcls)
    fp64 = {"seconds": round(t64, 3), "classes": len(fcls),
            "s_per_map": round(t64 * ncls / len(fcls), 3),
            "scaled": not args.full_fp64, "total_iters": st64["total_iters"]}
    accuracy = {"max_abs_dq_mixed_vs_fp64": float(np.abs(q_mixed[mask] - q64[mask]).max()),
                "dQ_mixed_vs_fp64_on_sample": float(q_mixed[mask].sum() - q64[mask].sum()),
                "Q": Q if scale == 1.0 else None,
                "abs_Q_minus_round": abs(Q - round(Q)) if scale == 1.0 else None,
                "max_abs_imag_q": st["max_abs_imag_q"], "sum_imag_q": st["sum_imag_q"],
                "lam_min": st["lam_min"], "lam_max": st["lam_max"], "zolo_delta": st["zolo_delta"],
                "max_true_resid_base_fp64": st["max_true_resid"],
                "deflation": dict(modes=args.deflate, **defl_info) if args.deflate else None}
    if args.full_fp64:
        accuracy["Q_fp64"] = float(q64.sum())
        accuracy["abs_Q_minus_round_fp64"] = abs(float(q64.sum()) - round(float(q64.sum())))

    cpu = None
    if not args.no_cpu:
        print("bench: CPU oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(WORKLOAD, DIMS, R_GAP, round(st["total_iters"] * scale), round(st["n_sources"] * scale),
                           args.cpu_iters)

    line = {
        "metric": "sec per q(x) map + D_W HBM GB/s; mixed/batched vs plain FP64 at 16^3x32"
                  if WORKLOAD == "noise16x32" else f"sec per q(x) map, {WORKLOAD}",
        "value": round(ms_per_step / 1000.0, 3), "unit": "s/map",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 1),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc,
                   "lattice": list(DIMS), "n_sources": st["n_sources"], "n_batches": st["n_batches"],
                   "kappa": KAPPA, "zolotarev_poles": POLES, "cg_tol": TOL, "reliable_interval": RELIABLE,
                   "precision": "FP32 stencil and CG body, FP64 scalars/reliable updates/accumulation"
                                + DIR_STORAGE[args.dir_storage][1],
                   "classes": len(classes), "classes_per_map": ncls,
                   "extrapolated": scale != 1.0,
                   "stencil_variants": {"f32_kind": ["site", "plane", "xy-tile", "plane, xy links in LDS"][tuning["f32_kind"]],
                                        "f32_rhs_per_thread": tuning["f32_nr"],
                                        "plane_band": tuning["plane_band"],
                                        "f64_rhs_per_block": 1 << tuning["f64_lgr"]}},
        "speedup_vs_fp64": round(fp64["s_per_map"] / (ms_per_step / 1000.0), 3),
        "roofline": roofline, "dslash": dslash, "fp64": fp64, "accuracy": accuracy,
        "bandwidth_context": {"device_copy_GBs": round(copy_GBs, 1),
                              "device_copy_note": "hipMemcpyAsync device to device, 2 GiB, read + write bytes",
                              "map_stencil_and_update_GBs": round(map_GBs, 1),
                              "map_note": "stencil + shift-update algorithmic bytes over the whole solve time"},
        "step_s": [round(t * scale, 3) for t in times],
        "median_s": round(float(np.median(times)) * scale, 3),
        "breakdown_s": {"bounds": round(st["t_bounds_s"], 3), "solve": round(st["t_solve_s"], 3),
                        "contract": round(st["t_contract_s"], 3)},
        "iterations": {"total": st["total_iters"], "max": st["max_iters"], "reliable_updates": st["n_reliable_updates"],
                       "mean_active_shifts": round(st["shift_updates"] / max(1, st["total_iters"]), 2)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
