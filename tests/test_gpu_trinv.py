"""GPU parity of the probing estimate of Tr D_W^-1 (smpq_compute_trinv) against the oracle.

Reference values: dense inverses of D_W (4^4, 3072 rows) and the oracle's sparse-LU probing
(6x4x4x6, ragged against the 256-site blocks).  Tolerances as for q(x): FP64 1e-10 absolute
(|t(x)| is of order 12), mixed precision 1e-5.
"""
import numpy as np
import pytest

import smpq_inputs as si
from oracle.lattice import Lattice
from oracle.probing import colouring
from oracle.trinv import trinv_dense, trinv_free, trinv_probing, trinv_smp_dense

pytestmark = pytest.mark.gpu

import paper_1901_02211_amd as smpq  # noqa: E402

KAPPA, TOL = 0.21, 1e-12
PRECS = [smpq.SMPQ_FP64, smpq.SMPQ_MIXED_FP32]


def _ctx(dims, U, prec):
    c = smpq.smpq_create(dims, 0)
    smpq.smpq_load_gauge(c, U)
    smpq.smpq_set_solver(c, prec, TOL, 10000, 50 if prec == smpq.SMPQ_MIXED_FP32 else 0)
    return c


def _tol(prec):
    return 1e-10 if prec == smpq.SMPQ_FP64 else 1e-5


@pytest.mark.parametrize("prec", PRECS)
def test_point_trace_noise4_and_free_field(prec):
    """Point scheme: the exact trace density, real, equal to the dense diagonal; the free
    field gives the momentum sum at every site."""
    print(f"trinv point sources on noise4 and the free 4^4 field, precision {prec}", flush=True)
    dims = (4, 4, 4, 4)
    lat = Lattice(dims)
    U = si.workload("noise4")
    c = _ctx(dims, U, prec)
    smpq.smpq_set_point_scheme(c)
    t, st = smpq.smpq_compute_trinv(c)
    ref = trinv_dense(U, lat, KAPPA)
    assert st["n_sources"] == 3072
    assert np.abs(t - ref).max() < _tol(prec)
    assert abs(t.sum() - ref.sum()) < 100 * _tol(prec)
    free = _ctx(dims, si.near_identity_su3(dims, 0.0, 0), prec)
    smpq.smpq_set_point_scheme(free)
    tf, _ = smpq.smpq_compute_trinv(free)
    assert np.abs(tf - trinv_free(dims, KAPPA)).max() < _tol(prec)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_smp_modes_match_dense_class_sums(mode, prec):
    print(f"trinv SMP r=2 mode {mode}, precision {prec}", flush=True)
    dims = (4, 4, 4, 4)
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.4, 21)
    col, n = colouring(lat, (2, 2, 2, 2), mode)
    ref = trinv_smp_dense(U, lat, KAPPA, col)
    c = _ctx(dims, U, prec)
    smpq.smpq_set_scheme(c, (2, 2, 2, 2), mode)
    t, st = smpq.smpq_compute_trinv(c)
    assert st["n_sources"] == 12 * n
    assert np.abs(t - ref).max() < _tol(prec)


def test_ragged_lattice_subset_of_classes():
    """V = 576 (two full 256-site blocks and a ragged one), odd extents, a subset of the
    classes; sites of other classes stay zero."""
    dims = (6, 4, 4, 6)
    print(f"trinv on {dims}", flush=True)
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.3, 24)
    col, n = colouring(lat, (2, 2, 2, 2), 0)
    classes = [0, 5, n - 1]
    ref = trinv_probing(U, lat, KAPPA, col, classes)
    for prec in PRECS:
        c = _ctx(dims, U, prec)
        smpq.smpq_set_scheme(c, (2, 2, 2, 2), 0)
        t, _ = smpq.smpq_compute_trinv(c, classes)
        assert np.abs(t - ref).max() < _tol(prec)
        assert np.all(t[~np.isin(col, classes)] == 0)


def test_trinv_then_qx_on_one_context():
    """Switching between the unshifted solve and the Zolotarev solve on one context (graphs
    and workspace rebuilt) leaves both results unchanged."""
    dims = (4, 4, 4, 4)
    print("trinv and q(x) alternating on one context", flush=True)
    U = si.workload("noise4")
    c = _ctx(dims, U, smpq.SMPQ_MIXED_FP32)
    smpq.smpq_set_zolotarev(c, 14, 0.13, 2.62)
    smpq.smpq_set_scheme(c, (2, 2, 2, 2), 0)
    q1 = smpq.smpq_compute_qx_classes(c, [0, 3])[0]
    t1, _ = smpq.smpq_compute_trinv(c, [0, 3])
    q2 = smpq.smpq_compute_qx_classes(c, [0, 3])[0]
    t2, _ = smpq.smpq_compute_trinv(c, [0, 3])
    assert np.array_equal(q1, q2) and np.array_equal(t1, t2)
    assert np.abs(t1).max() > 1.0 and np.abs(q1).max() > 0.0


def test_trinv_scan_point_row_is_exact():
    """The scan of the trace of D_W^-1 on 4^4: the exact trace is the dense one, and the
    single-site scheme r = 4 reproduces it."""
    from paper_1901_02211_amd.scan import scan
    dims = (4, 4, 4, 4)
    print("trinv scheme scan on noise4", flush=True)
    U = si.workload("noise4")
    res = scan(U, dims, gaps=(2, 4), precision=smpq.SMPQ_FP64, quantity="trinv")
    assert abs(res["Q_exact"] - trinv_dense(U, Lattice(dims), KAPPA).sum().real) < 1e-8
    rows = {(w["r"], w["mode"]): w for w in res["rows"]}
    assert rows[(4, 0)]["max_abs_dq"] < 1e-13
