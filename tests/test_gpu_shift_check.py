"""GPU: the per-shift FP64 true-residual check and refinement of the shifted solves.

Section 2.1, Eqs. 6-8 solve every shifted system M_i v_i = b; the reliable updates of the
mixed path only correct the base system.  smpq_set_shift_check evaluates every shift's FP64
residual ||b - (H^2 + q_i) x_i|| / ||b|| after the solve and refines the shifts above a
threshold.  Checked here: the check alone leaves q(x) bit for bit unchanged; the FP64 path's
shifts are already at the tolerance; the mixed path's shifts sit at FP32 rounding before and
below the threshold after refinement, which moves the mixed q(x) from the 1e-5 class to the
FP64 oracle within 1e-8, on the near-identity 4^4 field and on the ill-conditioned rough8
field without deflation.
"""
import os

import numpy as np
import pytest

import paper_1901_02211_amd as smpq
import smpq_inputs as si
from conftest import GOLDEN

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _golden(name):
    path = os.path.join(GOLDEN, f"{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{name}.npz not generated (tests/golden/make_golden.py {name})")
    return np.load(path)


def _map_ctx(workload, r, prec):
    w = si.WORKLOADS[workload]
    z = _golden(f"{workload}_zolo")
    c = smpq.smpq_create(w["dims"], 0)
    smpq.smpq_load_gauge(c, si.workload(workload))
    smpq.smpq_set_zolotarev(c, int(z["n_poles"]), float(z["lam_min"]), float(z["lam_max"]))
    smpq.smpq_set_solver(c, prec, TOL, 10000, 50 if prec != smpq.SMPQ_FP64 else 0)
    smpq.smpq_set_scheme(c, (r,) * 4, 0)
    return c


def test_fp64_shifts_are_at_the_tolerance():
    print("shift check: noise4 r=2 map, FP64", flush=True)
    g = _golden("noise4_smp")
    c = _map_ctx("noise4", 2, smpq.SMPQ_FP64)
    q0 = smpq.smpq_compute_qx(c)[0]
    smpq.smpq_set_shift_check(c, True, 1e-10)
    q, qi, Q, st = smpq.smpq_compute_qx(c)
    print(f"FP64 per-shift residual {st['max_shift_resid']:.3e}, refined {st['n_refined']}", flush=True)
    assert np.array_equal(q, q0)                   # the x_i accumulators do not touch y
    assert 0.0 < st["max_shift_resid"] <= 10 * TOL and st["n_refined"] == 0
    assert np.abs(q - g["qx"]).max() < 1e-10 * np.abs(g["qx"]).max()


def test_mixed_shifts_refined_to_fp64_accuracy():
    print("shift check: noise4 r=2 map, mixed, check only then refined", flush=True)
    g = _golden("noise4_smp")
    c = _map_ctx("noise4", 2, smpq.SMPQ_MIXED_FP32)
    q0, _, _, st0 = smpq.smpq_compute_qx(c)
    smpq.smpq_set_shift_check(c, True, 0.0)                 # check only
    q1, _, _, st1 = smpq.smpq_compute_qx(c)
    assert np.array_equal(q1, q0) and st1["n_refined"] == 0
    print(f"mixed per-shift residual before refinement {st1['max_shift_resid']:.3e}", flush=True)
    assert 1e-11 < st1["max_shift_resid"] < 1e-4             # FP32 rounding of the shifted solutions
    smpq.smpq_set_shift_check(c, True, 1e-10)
    q2, qi2, Q2, st2 = smpq.smpq_compute_qx(c)
    e0, e2 = np.abs(q0 - g["qx"]).max(), np.abs(q2 - g["qx"]).max()
    print(f"refined: final residual {st2['max_shift_resid_final']:.3e}, {st2['n_refined']} systems, "
          f"{st2['refine_iters']} iterations; max |dq| {e0:.3e} -> {e2:.3e}", flush=True)
    assert st2["max_shift_resid_final"] <= 1e-10
    assert st2["n_refined"] > 0 and st2["refine_iters"] > 0
    assert e2 < 1e-8 and e2 < e0
    assert abs(Q2 - g["qx"].sum()) < 1e-8
    smpq.smpq_set_shift_check(c, False)                      # off again: the plain mixed map
    assert np.array_equal(smpq.smpq_compute_qx(c)[0], q0)


def test_refined_mixed_path_on_ill_conditioned_field():
    """rough8 without deflation (k = 0.027): the refined mixed map equals the oracle's stored
    classes within 1e-8."""
    print("shift check: rough8 r=4 undeflated, mixed, refined", flush=True)
    g = _golden("rough8_smp4_part")
    c = _map_ctx("rough8", 4, smpq.SMPQ_MIXED_FP32)
    smpq.smpq_set_shift_check(c, True, 1e-10)
    cls = [int(k) for k in g["classes"]]
    q, qi, st = smpq.smpq_compute_qx_classes(c, cls)
    mask = np.isin(smpq.smpq_get_coloring(c), cls)
    err = np.abs(q[mask] - g["qx"][mask]).max()
    print(f"rough8 refined: residual {st['max_shift_resid']:.3e} -> {st['max_shift_resid_final']:.3e}, "
          f"max |dq| {err:.3e}", flush=True)
    assert st["max_shift_resid_final"] <= 1e-10
    assert err < 1e-8


def test_shift_check_refuses_16bit_directions():
    c = _map_ctx("noise4", 2, smpq.SMPQ_MIXED_FP16DIR)
    smpq.smpq_set_shift_check(c, True, 1e-10)
    with pytest.raises(smpq.SmpqError) as e:
        smpq.smpq_compute_qx_classes(c, [0])
    assert e.value.status == -1
