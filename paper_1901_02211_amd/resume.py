"""A q(x) map in chunks of classes with checkpoint and resume, for maps that take hours
(32^3 x 64 at r = 8: 49152 sources).  After every chunk the partial q(x), Im q(x), the
finished classes and the solve statistics so far are written to an .npz file (atomically: a
temporary file, then a rename); a later call with the same file continues after the last
finished chunk, on this or another machine.  The classes of a scheme cover disjoint sites, so
the partial maps add up to the whole map exactly.

The file also records a fingerprint of everything the map depends on: the lattice, the
scheme's colouring, the Zolotarev coefficients, kappa, the solver's precision, tolerance,
iteration limit and reliable-update interval, and a hash of the gauge field the context loaded;
resuming with anything different raises ValueError.

Command line (a time-boxed job that can be run again until the map is complete):

    python -m paper_1901_02211_amd.resume --workload flux24x48 --gauge-seed 55 --state map.npz \\
        --time-limit 900

prints one line per chunk on stderr and, once the map is complete, one JSON line with Q,
|Q - round Q|, the summed solve time and the iteration count.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

from . import binding as smpq


def _fingerprint(ctx):
    col = smpq.smpq_get_coloring(ctx)
    c0, c, q, _ = smpq.smpq_get_zolotarev(ctx)
    s = smpq.smpq_get_settings(ctx)
    h = hashlib.sha256()
    h.update(np.asarray(ctx.dims, dtype=np.int64).tobytes())
    h.update(col.tobytes())
    h.update(np.array([c0, *c, *q], dtype=np.float64).tobytes())
    h.update(np.array([s["kappa"], s["tol"]], dtype=np.float64).tobytes())
    h.update(np.array([s["precision"], s["max_iter"], s["reliable_interval"]], dtype=np.int64).tobytes())
    h.update(np.array([s["gauge_hash"]], dtype=np.uint64).tobytes())
    return h.hexdigest()


_KEYS = ("qx", "qx_imag", "done", "fingerprint", "seconds", "iters")


def compute_qx_resumable(ctx, path, chunk=64, stop_after=None, deadline=None, log=None, extra=None):
    """q(x) of every class of the context's scheme, chunk classes per call of the library.
    Needs the gauge field, the scheme, the Zolotarev coefficients and the solver settings set
    (they are part of the fingerprint).
    stop_after: return after that many new chunks; deadline: a time.monotonic() value after
    which no new chunk starts.  Either leaves the map incomplete and returns None.  Returns
    (qx, qx_imag, Q) when complete.  log(k, classes, seconds, stats) is called after each chunk;
    extra: further arrays kept in the file (with those a previous call stored)."""
    V = ctx.volume
    fp = _fingerprint(ctx)
    ncls = int(smpq.smpq_get_coloring(ctx).max()) + 1
    if os.path.exists(path):
        st = np.load(path)
        if str(st["fingerprint"]) != fp:
            raise ValueError(f"{path} belongs to another lattice, scheme, set of coefficients, gauge field, "
                             f"kappa or solver setting")
        qx, qi, done = st["qx"].copy(), st["qx_imag"].copy(), st["done"].copy()
        secs = float(st["seconds"]) if "seconds" in st.files else 0.0
        iters = int(st["iters"]) if "iters" in st.files else 0
        keep = {k: st[k] for k in st.files if k not in _KEYS}
    else:
        qx, qi, done = np.zeros(V), np.zeros(V), np.zeros(ncls, dtype=bool)
        secs, iters, keep = 0.0, 0, {}
    keep.update(extra or {})
    todo = np.nonzero(~done)[0]
    chunks = 0
    for k0 in range(0, len(todo), chunk):
        if stop_after is not None and chunks >= stop_after:
            return None
        if deadline is not None and time.monotonic() >= deadline:
            return None
        cls = todo[k0:k0 + chunk]
        t0 = time.perf_counter()
        q, im, stats = smpq.smpq_compute_qx_classes(ctx, cls)
        dt = time.perf_counter() - t0
        qx += q
        qi += im
        done[cls] = True
        secs += dt
        iters += int(stats["total_iters"])
        tmp = path + ".tmp.npz"
        np.savez(tmp, qx=qx, qx_imag=qi, done=done, fingerprint=np.array(fp), seconds=secs, iters=iters, **keep)
        os.replace(tmp, path)
        chunks += 1
        if log:
            log(chunks, cls, dt, stats)
    return qx, qi, float(qx.sum())


def main(argv=None):
    import smpq_inputs as si

    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="flux24x48", choices=sorted(si.WORKLOADS))
    ap.add_argument("--gauge-seed", type=int, default=None, help="Haar gauge transform with this seed")
    ap.add_argument("--r", type=int, default=None, help="gap of the scheme (default: the workload's)")
    ap.add_argument("--mode", type=int, default=0, choices=[0, 1, 2])
    ap.add_argument("--fp64", action="store_true")
    ap.add_argument("--state", required=True, help="checkpoint file (.npz)")
    ap.add_argument("--chunk", type=int, default=64, help="classes per chunk")
    ap.add_argument("--time-limit", type=float, default=0, help="start no chunk after this many seconds")
    a = ap.parse_args(argv)
    t_start = time.monotonic()
    w = si.WORKLOADS[a.workload]
    r = a.r if a.r is not None else (w["r"] if isinstance(w["r"], int) else w["r"][0])
    ctx = smpq.smpq_create(w["dims"], 0)
    smpq.smpq_load_gauge(ctx, si.workload(a.workload, gauge_seed=a.gauge_seed))
    ncls, nsrc = smpq.smpq_set_scheme(ctx, (r,) * 4, a.mode)
    if os.path.exists(a.state) and "interval" in np.load(a.state).files:
        lo, hi = (float(v) for v in np.load(a.state)["interval"])   # the same coefficients as before
    else:
        lo, hi = smpq.smpq_estimate_bounds(ctx, 300)
    smpq.smpq_set_zolotarev(ctx, 14, lo, hi)
    smpq.smpq_set_solver(ctx, smpq.SMPQ_FP64 if a.fp64 else smpq.SMPQ_MIXED_FP32, 1e-12, 10000, 50)
    tuning = smpq.smpq_autotune(ctx, 0)
    chunk = max(1, a.chunk)
    print(f"resume: {a.workload} {w['dims']} r={r} mode {a.mode}: {ncls} classes, {nsrc} sources, "
          f"interval [{lo:.6f}, {hi:.6f}], stencil {tuning}, chunk {chunk}", file=sys.stderr, flush=True)

    def log(k, cls, dt, st):
        print(f"resume: chunk {k}: classes {cls[0]}..{cls[-1]}, {dt:.1f} s, {st['total_iters']} iterations",
              file=sys.stderr, flush=True)

    deadline = t_start + a.time_limit if a.time_limit > 0 else None
    # the interval stays with the state, so that a resumed run uses the same coefficients
    res = compute_qx_resumable(ctx, a.state, chunk=chunk, deadline=deadline, log=log,
                               extra={"interval": np.array([lo, hi])})
    if not os.path.exists(a.state):
        print("resume: no chunk ran before the time limit", file=sys.stderr, flush=True)
        return 3
    st = np.load(a.state)
    left = int((~st["done"]).sum())
    if res is None:
        print(f"resume: stopped with {left} of {ncls} classes left; run again to continue", file=sys.stderr,
              flush=True)
        return 3
    qx, qi, Q = res
    print(json.dumps({"workload": a.workload, "dims": list(w["dims"]), "gauge_seed": a.gauge_seed, "r": r,
                      "mode": a.mode, "n_sources": nsrc, "precision": "fp64" if a.fp64 else "mixed",
                      "Q": Q, "abs_Q_minus_round": abs(Q - round(Q)), "sum_imag_q": float(qi.sum()),
                      "max_abs_imag_q": float(np.abs(qi).max()), "solve_seconds": float(st["seconds"]),
                      "iterations": int(st["iters"]), "interval": [lo, hi]}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
