"""Benchmark: seconds per q(x) map on one MI355X, mixed precision vs plain FP64.

Default workload: 16^3 x 32 periodic lattice, near-identity SU(3) links (eps = 0.2, seed 4),
kappa = 0.21, 14-pole Zolotarev sign function on Lanczos bounds, SMP normal mode with
r = 4 (256 classes x 12 = 3072 sources), per-shift CG tolerance 1e-12.  One step is one
whole q(x) map: Lanczos bounds + Zolotarev + every multi-shift CG solve + contraction +
copy-out of q(x) and Q, with the gauge field already resident in HBM.  The map runs in
FP32 with FP64 reliable updates every 50 iterations and FP64 accumulation.

Wall-clock budget (--budget-s, default 470 s for the whole process): --steps and --warmup are
upper bounds.  At most one untimed warmup map runs (the set-up already primes workspaces and
graphs); timed maps stop once the next would not leave room for the legs after them (the FP64
map, the CPU leg, the standalone figures).  `steps` reports the maps actually timed,
`steps_requested` the request.

--workload selects another lattice of the same family (24^3x48 flux, 16^4, 24^4, 32^3x64);
maps that take minutes are timed on a sample of classes and the value is extrapolated by
classes/sample (labelled "extrapolated").  --workload uneven times 16^4 + 24^4 + 32^3x64
together, the same fraction of classes of each, concurrently (one stream per lattice) and
one after another; --workload ensemble does the same for eight whole 8^4 maps.

Printed: one JSON line.  value = mean seconds per map of the timed maps (lower is better).
Beside it:
  roofline      the dominant kernel of the step (HIP events on the library's stream),
                algorithmic bytes per launch / mean launch duration vs 8 TB/s
  dslash        the Wilson stencil in situ and standalone (rotating buffers > 1 GB)
  fp64          the plain FP64 GPU path: the whole map when the map is whole (else a sample
                of classes, scaled)
  accuracy      mixed vs FP64 GPU (max |dq|, dQ) and |Q - round(Q)| of both maps
  cpu_baseline  the FP64 numpy oracle, one process per host core: a bounded sample of the
                workload scaled to a map, and one whole 4^4 map timed as it runs (with the
                GPU's time for the same map and the GPU-vs-oracle difference)
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

T_START = time.perf_counter()
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


# names of the FP32 stencil variants, by the tuning's kind number
F32_KINDS = ("site", "plane", "xy-tile", "plane, xy links in LDS", "xy-tile, links read per right-hand side")


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


def host_cores():
    """Host cores the CPU leg may use: the process's CPU affinity, at most 16 (the host share
    of one GPU on the MI355X boxes)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            return next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        return ""


# The CPU leg runs in a child interpreter that never touches the GPU and forks its workers
# there: one process per host core, one BLAS thread each.  It prints one JSON line per part.
CPU_LEG = r"""
import json, os, sys, time
sys.path.insert(0, ROOT)
import multiprocessing as mp
import numpy as np
import smpq_inputs as si
from oracle.lattice import Lattice
from oracle.dirac import apply_dw, apply_h2
from oracle.mscg import multishift_cg, NotConverged
from oracle.probing import colouring
from oracle.zolotarev import zolotarev
from oracle.charge import qx_probing

P, WORKLOAD, DIMS, RGAP, ITERS, POLES, KAPPA, TOL, SMALL = json.loads(sys.argv[1])
DIMS = tuple(DIMS)

def big_source(k):
    # ITERS multi-shift CG iterations of the source (class k, spin-colour 0) of the workload
    b = np.zeros((LAT.volume, 4, 3), dtype=np.complex128)
    b[COL == k, 0, 0] = 1.0
    t0 = time.perf_counter()
    try:
        multishift_cg(lambda v: apply_h2(U, LAT, KAPPA, v) + S0 * v, b, QS - S0, TOL, ITERS)
    except NotConverged:
        pass
    return time.perf_counter() - t0

def small_class(k):
    return qx_probing(U4, LAT4, KAPPA, Z4, COL4, [k], TOL, 5000)

if __name__ == "__main__":
    ctx = mp.get_context("fork")
    # part 1: a bounded sample of the big workload, one source per core at once
    U = si.workload(WORKLOAD); LAT = Lattice(DIMS)
    COL, _ = colouring(LAT, (RGAP,) * 4, 0)
    c0, c, QS, _ = zolotarev(POLES, 0.14, 2.73)
    S0 = float(QS.min())
    t0 = time.perf_counter(); apply_dw(U, LAT, KAPPA, np.ones((LAT.volume, 4, 3), dtype=np.complex128))
    t_dw = time.perf_counter() - t0
    t0 = time.perf_counter()
    with ctx.Pool(P) as pool:
        per = pool.map(big_source, list(range(P)))
    wall = time.perf_counter() - t0
    print(json.dumps({"part": "sample", "wall_s": wall, "worker_s": per, "dw_s": t_dw}), flush=True)
    del U
    # part 2: one whole small map (every class), classes spread over the cores
    U4 = si.workload(SMALL["workload"]); LAT4 = Lattice(tuple(SMALL["dims"]))
    COL4, ncls = colouring(LAT4, (SMALL["r"],) * 4, 0)
    Z4 = zolotarev(POLES, SMALL["lo"], SMALL["hi"])
    t0 = time.perf_counter()
    with ctx.Pool(P) as pool:
        parts = pool.map(small_class, list(range(int(ncls))))
    wall = time.perf_counter() - t0
    q = np.sum(parts, axis=0).real
    print(json.dumps({"part": "small_map", "wall_s": wall, "classes": int(ncls), "q": q.tolist()}), flush=True)
"""


def cpu_baseline(workload, dims, r_gap, total_iters, n_sources, iters_sample, small, timeout_s):
    """The FP64 oracle on the host cores, one process per core: (1) `iters_sample` multi-shift CG
    iterations of one source of the workload on every core at once, scaled by the map's measured
    iteration count to seconds per map; (2) one whole small map (every class of `small`) timed
    as it runs.  Parts that do not finish within timeout_s are left out."""
    P = host_cores()
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    arg = json.dumps([P, workload, list(dims), r_gap, iters_sample, POLES, KAPPA, TOL, small])
    proc = subprocess.Popen([sys.executable, "-c", CPU_LEG.replace("ROOT", repr(ROOT), 1), arg],
                            stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env)
    try:
        out, err = proc.communicate(timeout=timeout_s)
    except subprocess.TimeoutExpired:
        proc.kill()
        out, err = proc.communicate()
    parts = {}
    for ln in out.splitlines():
        try:
            d = json.loads(ln)
            parts[d["part"]] = d
        except (ValueError, KeyError):
            pass
    res = {"value": None, "unit": "s/map", "cores": P, "kind": "oracle", "host_cpu": cpu_model(),
           "host_nproc": os.cpu_count()}
    if "sample" in parts:
        p = parts["sample"]
        rate = P * iters_sample / p["wall_s"]        # CG iterations per second over all cores
        V = int(np.prod(dims))
        res.update(value=total_iters / rate,
                   sample=f"{iters_sample} multi-shift CG iterations of {P} sources of the {workload} field, "
                          f"one per core at once ({p['wall_s']:.1f} s), scaled by the map's {total_iters} "
                          f"iterations over {n_sources} sources (extrapolated)",
                   seconds_per_iteration_per_core=float(np.mean(p["worker_s"])) / iters_sample,
                   oracle_dw_ns_per_site=1e9 * p["dw_s"] / V,
                   oracle_dw_GBs=V * (72 + 48) * 8 / p["dw_s"] / 1e9)
    else:
        res["sample"] = f"not finished within {timeout_s:.0f} s"
    if "small_map" in parts:
        p = parts["small_map"]
        res["whole_small_map"] = {"workload": small["label"], "s_per_map": round(p["wall_s"], 3),
                                  "classes": p["classes"], "extrapolated": False,
                                  "q": np.asarray(p["q"])}
    if proc.returncode not in (0, None) and not parts:
        res["error"] = err.strip().splitlines()[-1] if err.strip() else f"exit {proc.returncode}"
    return res


class Clock:
    """Wall clock of the whole process against a budget (seconds from the import of bench.py)."""

    def __init__(self, budget_s, now=None, t0=None):
        self.now = now if now is not None else (lambda: time.perf_counter())
        self.t0 = now() if t0 is None else t0
        self.budget = budget_s

    def elapsed(self):
        return self.now() - self.t0

    def left(self):
        return self.budget - self.elapsed()


def timed_maps(one_map, steps, clock, reserve, estimate_s=None):
    """Time whole maps: at most `steps`, at least one, and no further map once the next one (at
    the mean duration so far) would leave less than reserve(duration) seconds of the budget.
    one_map() returns a tuple whose first entry is its duration.  Returns the per-map results."""
    out = []
    for _ in range(steps):
        est = float(np.mean([r[0] for r in out])) if out else estimate_s
        if out and clock.left() - 1.05 * est < reserve(est):
            break
        out.append(one_map())
    return out


SMALL_MAP = {"workload": "noise4", "label": "4^4 near-identity SU(3) eps=0.3 seed 0, SMP normal mode r=2 "
                                         "(192 sources), interval [0.13, 2.62]",
             "dims": [4, 4, 4, 4], "r": 2, "lo": 0.13, "hi": 2.62}
FP64_OVER_MIXED = 2.4      # expected FP64 / mixed map time, for planning only (measured: 2.23)
CPU_LEG_S = 50.0           # time allowed for the CPU leg (measured: 15 s on 16 cores)
EXTRAS_S = 20.0            # standalone stencil, copy, small-map and slack


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed maps requested (an upper bound under --budget-s)")
    ap.add_argument("--warmup", type=int, default=0, help="untimed maps requested (at most one is run)")
    ap.add_argument("--budget-s", type=float, default=470.0,
                    help="wall-clock budget of the whole process; timed maps stop early to keep it")
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
    clock = Clock(args.budget_s, t0=T_START)

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
    whole_fp64 = args.full_fp64 or args.classes == 0    # whole maps: compare whole maps
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
        print(f"bench: map {t2 - t0:.2f} s, Q = {Q:.6f}, iters {st['total_iters']}, batches {st['n_batches']} "
              f"({clock.elapsed():.0f} s of {clock.budget:.0f})", file=sys.stderr, flush=True)
        return t2 - t0, q, Q, st

    # untimed set-up: workspace allocation and first launches of every kernel
    smpq.smpq_set_zolotarev(ctx, POLES, 0.14, 2.73)
    tuning = smpq.smpq_autotune(ctx, 0)            # at the map's batch size
    print(f"bench: stencil variants {tuning} ({clock.elapsed():.0f} s)", file=sys.stderr, flush=True)
    smpq.smpq_prepare(ctx)
    smpq.smpq_compute_qx_classes(ctx, [0])
    smpq.smpq_set_timing(ctx, True)
    est = None
    warm = 0
    if args.warmup > 0:     # one untimed map: workspaces and graphs are already primed above
        print("bench: warmup map", file=sys.stderr, flush=True)
        est = one_map()[0]
        warm = 1
    # what must still fit after the timed maps: the FP64 map (whole or sampled), the CPU leg
    # and the standalone figures
    fp64_est = lambda m: FP64_OVER_MIXED * m * (1.0 if whole_fp64 else min(1.0, args.fp64_classes / len(classes)))
    cpu_s = 0.0 if args.no_cpu else CPU_LEG_S
    reserve = lambda m: fp64_est(m) + cpu_s + EXTRAS_S
    runs = timed_maps(one_map, args.steps, clock, reserve, est)
    times = [r[0] for r in runs]
    _, q_mixed, Q, st = runs[-1]
    map_s = float(np.mean(times))
    ms_per_step = 1000.0 * map_s * scale

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
    stream_GBs = {}
    if hasattr(smpq, "smpq_bench_stream"):
        for nt in (False, True):
            ms = smpq.smpq_bench_stream(ctx, 1 << 31, 20, nt)
            stream_GBs["nontemporal" if nt else "cached"] = round(2.0 * (1 << 31) / (ms * 1e-3) / 1e9, 1)
    ms32, by32 = smpq.smpq_bench_dslash(ctx, smpq.SMPQ_MIXED_FP32, 24, 4, 50)
    ms64, by64 = smpq.smpq_bench_dslash(ctx, smpq.SMPQ_FP64, 24, 4, 50)
    dslash = {"insitu_GBs": round(ds_insitu, 1), "insitu_frac": round(ds_insitu / HBM_PEAK_GBS, 4),
              "launches": st["dslash_launches"], "algorithmic_bytes": st["dslash_bytes"],
              "traffic_over_algorithmic": trd["traffic_over_algorithmic"] if trd else None,
              "standalone_fp32_n24_GBs": round(by32 / ms32 / 1e6, 1),
              "standalone_fp64_n24_GBs": round(by64 / ms64 / 1e6, 1),
              "standalone_note": "24 right-hand sides, 4 rotating input/output/link sets (> 1 GB)"}

    # plain FP64 GPU path: the whole map when it fits the budget, else a sample of classes
    fcls = list(range(min(args.fp64_classes, len(classes))))
    if whole_fp64 and clock.left() - FP64_OVER_MIXED * map_s * scale >= cpu_s + 10.0:
        fcls = list(classes)
    print(f"bench: FP64 comparison on {len(fcls)} classes ({clock.elapsed():.0f} s)", file=sys.stderr, flush=True)
    smpq.smpq_set_solver(ctx, smpq.SMPQ_FP64, TOL, 10000, 0)
    smpq.smpq_set_timing(ctx, False)
    t0 = time.perf_counter()
    q64, qi64, st64 = smpq.smpq_compute_qx_classes(ctx, fcls)
    t64 = time.perf_counter() - t0
    colour = smpq.smpq_get_coloring(ctx)
    mask = np.isin(colour, fcls)
    fp64_whole = len(fcls) == ncls
    fp64 = {"seconds": round(t64, 3), "classes": len(fcls),
            "s_per_map": round(t64 * ncls / len(fcls), 3),
            "scaled": not fp64_whole, "total_iters": st64["total_iters"]}
    accuracy = {"max_abs_dq_mixed_vs_fp64": float(np.abs(q_mixed[mask] - q64[mask]).max()),
                "dQ_mixed_vs_fp64": float(q_mixed[mask].sum() - q64[mask].sum()),
                "dQ_over": "whole map" if fp64_whole else f"{len(fcls)} classes",
                "Q": Q if scale == 1.0 else None,
                "abs_Q_minus_round": abs(Q - round(Q)) if scale == 1.0 else None,
                "max_abs_imag_q": st["max_abs_imag_q"], "sum_imag_q": st["sum_imag_q"],
                "lam_min": st["lam_min"], "lam_max": st["lam_max"], "zolo_delta": st["zolo_delta"],
                "max_true_resid_base_fp64": st["max_true_resid"],
                "deflation": dict(modes=args.deflate, **defl_info) if args.deflate else None}
    if fp64_whole:
        Q64 = float(q64.sum())
        accuracy["Q_fp64"] = Q64
        accuracy["abs_Q_minus_round_fp64"] = abs(Q64 - round(Q64))

    cpu = None
    if not args.no_cpu:
        # the small whole map on the GPU too (both precisions), beside the oracle's
        print(f"bench: CPU oracle ({host_cores()} cores, {clock.elapsed():.0f} s)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(WORKLOAD, DIMS, R_GAP, round(st["total_iters"] * scale), round(st["n_sources"] * scale),
                           args.cpu_iters, SMALL_MAP, max(20.0, min(CPU_LEG_S, clock.left() - 10.0)))
        small = cpu.get("whole_small_map")
        if small is not None:
            c4 = smpq.smpq_create(SMALL_MAP["dims"], 0)
            smpq.smpq_load_gauge(c4, si.workload(SMALL_MAP["workload"]))
            smpq.smpq_set_scheme(c4, (SMALL_MAP["r"],) * 4, 0)
            smpq.smpq_set_zolotarev(c4, POLES, SMALL_MAP["lo"], SMALL_MAP["hi"])
            qcpu = small.pop("q")
            for name, prec, rel in (("fp64", smpq.SMPQ_FP64, 0), ("mixed", smpq.SMPQ_MIXED_FP32, RELIABLE)):
                smpq.smpq_set_solver(c4, prec, TOL, 10000, rel)
                smpq.smpq_compute_qx(c4)                  # untimed: workspace and graphs
                t0 = time.perf_counter()
                q4 = smpq.smpq_compute_qx(c4)[0]
                small[f"gpu_{name}_s_per_map"] = round(time.perf_counter() - t0, 4)
                small[f"gpu_{name}_max_abs_dq_vs_oracle"] = float(np.abs(q4 - qcpu).max())
            smpq.smpq_destroy(c4)

    solve_s = st["t_solve_s"]
    line = {
        "metric": "sec per q(x) map + D_W HBM GB/s; mixed/batched vs plain FP64 at 16^3x32"
                  if WORKLOAD == "noise16x32" else f"sec per q(x) map, {WORKLOAD}",
        "value": round(ms_per_step / 1000.0, 3), "unit": "s/map",
        "n_gpus": 1, "steps": len(times), "warmup": warm, "ms_per_step": round(ms_per_step, 1),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": ("one whole q(x) map: " if scale == 1.0 else "") + desc,
                   "lattice": list(DIMS), "n_sources": st["n_sources"], "n_batches": st["n_batches"],
                   "kappa": KAPPA, "zolotarev_poles": POLES, "cg_tol": TOL, "reliable_interval": RELIABLE,
                   "precision": "FP32 stencil and CG body, FP64 scalars/reliable updates/accumulation"
                                + DIR_STORAGE[args.dir_storage][1],
                   "classes": len(classes), "classes_per_map": ncls,
                   "extrapolated": scale != 1.0,
                   "stencil_variants": {"f32_kind": F32_KINDS[tuning["f32_kind"]],
                                        "f32_rhs_per_thread": tuning["f32_nr"],
                                        "plane_band": tuning["plane_band"],
                                        "f64_kind": ["lanes", "xy-tile"][tuning.get("f64_kind", 0)],
                                        "f64_rhs_per_block": (tuning["f64_nr"] if tuning.get("f64_kind", 0) == 1
                                                              else 1 << tuning["f64_lgr"]),
                                        "f32_interleave": tuning.get("f32_interleave", 1),
                                        "f64_interleave": tuning.get("f64_interleave", 1),
                                        "f32_dag_kind": F32_KINDS[tuning.get("f32_dag_kind", tuning["f32_kind"])],
                                        "f32_dag_rhs_per_thread": tuning.get("f32_dag_nr", tuning["f32_nr"]),
                                        "f32_dag_interleave": tuning.get("f32_dag_interleave",
                                                                         tuning.get("f32_interleave", 1))}},
        "steps_requested": args.steps, "warmup_requested": args.warmup, "budget_s": args.budget_s,
        "speedup_vs_fp64": round(fp64["s_per_map"] / (ms_per_step / 1000.0), 3),
        "roofline": roofline, "dslash": dslash, "fp64": fp64, "accuracy": accuracy,
        "bandwidth_context": {"device_copy_GBs": round(copy_GBs, 1),
                              "device_copy_note": "hipMemcpyAsync device to device, 2 GiB, read + write bytes",
                              "stream_copy_GBs": stream_GBs or None,
                              "stream_copy_note": "the library's float4 copy kernel (cached / non-temporal loads and "
                                                  "stores), 2 GiB, read + write bytes",
                              "map_stencil_and_update_GBs": round(map_GBs, 1),
                              "map_note": "stencil + shift-update algorithmic bytes over the whole solve time"},
        "step_s": [round(t * scale, 3) for t in times],
        "median_s": round(float(np.median(times)) * scale, 3),
        "breakdown_s": {"bounds": round(st["t_bounds_s"], 3), "solve": round(solve_s, 3),
                        "contract": round(st["t_contract_s"], 3),
                        "solve_stencil": round(st["dslash_ms"] * 1e-3, 3),
                        "solve_shift_update": round(st["update_ms"] * 1e-3, 3),
                        "solve_rest": round(solve_s - (st["dslash_ms"] + st["update_ms"]) * 1e-3, 3)},
        "iterations": {"total": st["total_iters"], "max": st["max_iters"], "reliable_updates": st["n_reliable_updates"],
                       "mean_active_shifts": round(st["shift_updates"] / max(1, st["total_iters"]), 2)},
        "cpu_baseline": cpu,
        "wall_s": round(clock.elapsed(), 1),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
