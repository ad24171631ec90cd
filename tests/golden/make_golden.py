"""Write oracle reference values for the GPU parity tests (calls only oracle/ and smpq_inputs).

    python tests/golden/make_golden.py <job> [--procs N]

Jobs (each writes tests/golden/<job>.npz):
  noise4_smp      4^4 near-identity (eps 0.3, seed 0): Zolotarev interval from the oracle's
                  Lanczos, q(x) with SMP r = 2 (all 16 classes, 192 sources), and the dense
                  exact and dense-Zolotarev q(x).
  noise4_point    same field: point-source q(x) on all 256 sites (3072 sources).
  flux8_smp2      8^4 flux (1,1) + noise 0.1 + random gauge: SMP r = 2 (192 sources).
  flux8_point     same field: point sources on the 64 sites of the seeded subset (768 sources).
  flux8_smp4_part same field: SMP r = 4, classes 0, 85 and 255 (36 of 3072 sources).
  noise16x32_part 16^3 x 32 (eps 0.2, seed 4): SMP r = 4, classes 0 and 129 (24 of 3072 sources).
  noise16_part    16^4 (eps 0.1, seed 6): SMP r = 4, classes 0 and 200 (24 of 3072 sources).
  noise24_part    24^4 (eps 0.2, seed 7): SMP r = 6, class 777 (12 of 15552 sources).
  flux24x48_part  24^3 x 48 flux (1,1) + noise 0.15 (seed 5): SMP r = 6, class 5 (12 of 15552).
  noise32x64_dov  32^3 x 64 (eps 0.3, seed 8): D_ov applied to one SMP r = 8 source (class 0,
                  spin 0, colour 0), kept on the 512 sites of the class and 64 seeded sites.
  rough8_smp4_part  8^4 noise 0.3 (seed 60) with a Haar-random 3^4 block (isolated low modes of
                  H_W), undeflated, on the narrow fixed interval [0.07, 2.62] (k = 0.027, the
                  smallest shift q_1 ~ 3e-5 lam_max^2): SMP r = 4, classes 0, 85 and 170.

Every job uses kappa = 0.21, 14 Zolotarev poles and CG tolerance 1e-12.  Up to 16^3 x 32 the
interval is [0.9 sqrt(theta_min), 1.02 sqrt(theta_max)] from 300 Lanczos steps of the oracle
(start vector: SplitMix64 stream 0); on the larger lattices, where the oracle's fully
reorthogonalised Lanczos would hold 300 vectors of 0.1-0.4 GB, it is the fixed interval
[0.15, 2.75], which contains the free-field range [1 - 4 kappa, 1 + 8 kappa] = [0.16, 2.68] that
near-identity noise narrows (both sides use the same coefficients, so parity does not depend on
how tight the interval is).
Sources run in parallel processes; each site's contributions are summed in (class, alpha, a)
order.
"""
import argparse
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import smpq_inputs as si  # noqa: E402
from oracle.charge import (charge_from_spectrum, dov_apply, eps_dense, h_spectrum, qx_from_eps,  # noqa: E402
                           source_contribution)
from oracle.lanczos import bounds  # noqa: E402
from oracle.lattice import Lattice  # noqa: E402
from oracle.probing import colouring, point_colouring  # noqa: E402
from oracle.zolotarev import eps_scalar, zolotarev  # noqa: E402

KAPPA, TOL, MAXIT, NPOLES, STEPS = 0.21, 1e-12, 5000, 14, 300
HERE = os.path.dirname(os.path.abspath(__file__))

JOBS = {
    "noise4_smp": ("noise4", ("smp", 2), None, True),
    "noise4_point": ("noise4", ("point",), None, False),
    "flux8_smp2": ("flux8", ("smp", 2), None, False),
    "flux8_point": ("flux8", ("point",), "subset", False),
    "flux8_smp4_part": ("flux8", ("smp", 4), [0, 85, 255], False),
    "noise16x32_part": ("noise16x32", ("smp", 4), [0, 129], False),
    "noise16_part": ("noise16", ("smp", 4), [0, 200], False),
    "noise24_part": ("noise24", ("smp", 6), [777], False),
    "flux24x48_part": ("flux24x48", ("smp", 6), [5], False),
    "noise32x64_dov": ("noise32x64", ("dov", 8), [0], False),
    "rough8_smp4_part": ("rough8", ("smp", 4), [0, 85, 170], False),
}
FIXED_INTERVAL = {"noise16": (0.15, 2.75), "noise24": (0.15, 2.75), "flux24x48": (0.15, 2.75),
                  "noise32x64": (0.15, 2.75), "rough8": (0.07, 2.62)}
DOV_SAMPLE_SEED, DOV_SAMPLE_N = 9, 64

_G = {}


def _init(name, scheme):
    U = si.workload(name)
    lat = Lattice(si.WORKLOADS[name]["dims"])
    zo = np.load(os.path.join(HERE, f"{name}_zolo.npz"))
    zolo = (float(zo["c0"]), zo["c"], zo["q"])
    if scheme[0] == "point":
        col, _ = point_colouring(lat)
    else:
        col, _ = colouring(lat, (scheme[1],) * 4, 0)
    _G.update(U=U, lat=lat, zolo=zolo, col=col)


def _one(task):
    c, alpha, a = task
    S, val, iters = source_contribution(_G["U"], _G["lat"], KAPPA, _G["zolo"], _G["col"], c, alpha, a, TOL, MAXIT)
    return task, S, val, iters


def zolo_for(name):
    path = os.path.join(HERE, f"{name}_zolo.npz")
    if os.path.exists(path):
        return
    if name in FIXED_INTERVAL:
        lo, hi = FIXED_INTERVAL[name]
    else:
        U = si.workload(name)
        lat = Lattice(si.WORKLOADS[name]["dims"])
        lo, hi = bounds(U, lat, KAPPA, STEPS, seed=0)
    c0, c, q, delta = zolotarev(NPOLES, lo, hi)
    np.savez(path, lam_min=lo, lam_max=hi, c0=c0, c=c, q=q, delta=delta, n_poles=NPOLES, kappa=KAPPA)
    print(f"{name}: interval [{lo:.6f}, {hi:.6f}], delta {delta:.3e}", flush=True)


def run_dov(job, name, r, cls):
    """One probing source of class cls[0] (spin 0, colour 0): D_ov phi on sampled sites."""
    lat = Lattice(si.WORKLOADS[name]["dims"])
    U = si.workload(name)
    zo = np.load(os.path.join(HERE, f"{name}_zolo.npz"))
    col, _ = colouring(lat, (r,) * 4, 0)
    b = np.zeros((lat.volume, 4, 3), dtype=np.complex128)
    b[col == cls[0], 0, 0] = 1.0
    t0 = time.time()
    out = dov_apply(U, lat, KAPPA, (float(zo["c0"]), zo["c"], zo["q"]), b, TOL, MAXIT)
    rng = np.random.default_rng(DOV_SAMPLE_SEED)
    sites = np.union1d(np.nonzero(col == cls[0])[0], rng.choice(lat.volume, DOV_SAMPLE_N, replace=False))
    np.savez_compressed(os.path.join(HERE, f"{job}.npz"), sites=sites, dov=out[sites], cls=np.array(cls),
                        r=np.array(r), seconds=time.time() - t0)
    print(f"{job}: done in {time.time() - t0:.0f} s", flush=True)


def run(job, procs):
    name, scheme, classes, dense = JOBS[job]
    zolo_for(name)
    if scheme[0] == "dov":
        return run_dov(job, name, scheme[1], classes)
    lat = Lattice(si.WORKLOADS[name]["dims"])
    if scheme[0] == "point":
        sites = si.subset_sites(name) if classes == "subset" else np.arange(lat.volume)
        cls = list(sites)
    else:
        _, ncls = colouring(lat, (scheme[1],) * 4, 0)
        cls = list(range(ncls)) if classes is None else classes
    tasks = [(c, al, a) for c in cls for al in range(4) for a in range(3)]
    q = np.zeros(lat.volume, dtype=np.complex128)
    results = {}
    t0 = time.time()
    with ProcessPoolExecutor(procs, initializer=_init, initargs=(name, scheme)) as ex:
        for i, (task, S, val, iters) in enumerate(ex.map(_one, tasks, chunksize=1)):
            results[task] = (S, val, iters)
            if (i + 1) % max(1, len(tasks) // 20) == 0:
                print(f"{job}: {i + 1}/{len(tasks)} sources, {time.time() - t0:.0f} s", flush=True)
    iters = []
    for task in tasks:
        S, val, it = results[task]
        q[S] += val
        iters.append(it)
    out = dict(qx=q.real, qx_imag=q.imag, classes=np.array(cls), iters=np.array(iters),
               scheme=np.array(scheme[1] if scheme[0] == "smp" else 0), seconds=time.time() - t0)
    if dense:
        U = si.workload(name)
        w, v = h_spectrum(U, lat, KAPPA)
        zo = np.load(os.path.join(HERE, f"{name}_zolo.npz"))
        out["qx_exact"] = qx_from_eps(eps_dense(w, v), lat.volume)
        out["qx_dense_zolo"] = qx_from_eps(eps_dense(w, v, lambda x: eps_scalar(x, zo["c0"], zo["c"], zo["q"])),
                                           lat.volume)
        out["Q_exact"] = charge_from_spectrum(w)
        out["h_abs_min"] = np.abs(w).min()
        out["h_abs_max"] = np.abs(w).max()
    np.savez_compressed(os.path.join(HERE, f"{job}.npz"), **out)
    print(f"{job}: done in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("jobs", nargs="+", choices=sorted(JOBS))
    ap.add_argument("--procs", type=int, default=6)
    args = ap.parse_args()
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    for j in args.jobs:
        run(j, args.procs)
