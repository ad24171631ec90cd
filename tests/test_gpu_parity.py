"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same seeded inputs.

Sizes span several 256-site tiles with a ragged tail (V = 420, 576) plus odd extents.
Tolerances: FP64 stencil 1e-13 and FP32 stencil 2e-6, relative to the largest output
entry; FP64 q(x) within 1e-10 relative to the largest |q| of the oracle; mixed precision
within 1e-5.
"""
import functools

import numpy as np
import pytest

import smpq_inputs as si
from oracle.charge import dov_apply, qx_probing
from oracle.dirac import apply_dw, apply_gamma5, h_dense
from oracle.lanczos import bounds, ritz_extremes
from oracle.lattice import Lattice
from oracle.probing import colouring, point_colouring
from oracle.zolotarev import zolotarev

pytestmark = pytest.mark.gpu

import paper_1901_02211_amd as smpq  # noqa: E402

KAPPA = 0.21
TOL = 1e-12


def _ctx(dims, U):
    c = smpq.smpq_create(dims, 0)
    smpq.smpq_load_gauge(c, U)
    return c


def _zolo_interval(U, lat):
    return bounds(U, lat, KAPPA, 300, seed=0)


SITE_VARIANTS = [(0, nr, lgr) for nr, lgr in ((2, 0), (4, 1), (8, 2))]
PLANE_VARIANTS = [(k, nr, lgr) for k in (1, 3) for nr, lgr in ((4, 0), (8, 1), (16, 2))]
TILE_VARIANTS = [(2, nr, lgr) for nr, lgr in ((4, 0), (8, 1), (16, 2))]
F64_TILE_NR = (1, 2, 4, 8)    # FP64 xy-tile kernel (f64_kind 1): right-hand sides per block
# FP32 xy-tiles with the links read per right-hand side (kind 4): 1, 2, 4, 8 right-hand sides per block
RL_VARIANTS = [(4, nr, lgr) for nr, lgr in ((1, 0), (2, 0), (4, 1), (8, 2))]
# the tile kernels' block order: that many right-hand-side groups of one tile in a row
INTERLEAVES = (2, 8)


@pytest.mark.parametrize("dims", [(6, 4, 4, 6), (5, 3, 4, 7), (4, 4, 4, 4)])
@pytest.mark.parametrize("nrhs", [1, 3, 5])
def test_dslash_parity(dims, nrhs):
    """Every site-major FP32 variant (2, 4, 8 right-hand sides per thread) and every FP64
    interleave (1, 2, 4 right-hand sides per block) against the oracle."""
    print(f"dslash parity dims={dims} nrhs={nrhs}", flush=True)
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.5, 1)
    psi = si.random_spinors(dims, nrhs, 2)
    c = _ctx(dims, U)
    for dag in (False, True):
        ref = np.stack([apply_dw(U, lat, KAPPA, p, dagger=dag) for p in psi])
        scale = np.abs(ref).max()
        for tune in SITE_VARIANTS:
            smpq.smpq_set_tuning(c, *tune)
            out64 = smpq.smpq_apply_dw(c, psi, dagger=dag, precision=smpq.SMPQ_FP64)
            assert np.abs(out64 - ref).max() <= 1e-13 * scale, tune
            out32 = smpq.smpq_apply_dw(c, psi, dagger=dag, precision=smpq.SMPQ_MIXED_FP32)
            assert np.abs(out32 - ref).max() <= 2e-6 * scale, tune
    # the plane kernel needs 16x16 xy-planes
    for kind in (1, 3):
        with pytest.raises(smpq.SmpqError):
            smpq.smpq_set_tuning(c, kind, 8, 1)


@pytest.mark.parametrize("dims", [(16, 16, 2, 2), (16, 16, 3, 2), (16, 16, 4, 3)])
@pytest.mark.parametrize("nrhs", [1, 9, 17])
def test_dslash_parity_plane_tiled(dims, nrhs):
    """16x16 xy-planes: the FP32 kernel that stages one plane per block in LDS, with 4, 8 and
    16 right-hand sides per thread (17 leaves a ragged group for each)."""
    print(f"plane-tiled dslash parity dims={dims} nrhs={nrhs}", flush=True)
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.5, 11)
    psi = si.random_spinors(dims, nrhs, 12)
    c = _ctx(dims, U)
    for dag in (False, True):
        ref = np.stack([apply_dw(U, lat, KAPPA, p, dagger=dag) for p in psi])
        for tune in PLANE_VARIANTS + TILE_VARIANTS + RL_VARIANTS:
            for band in (1, 2, 4):
                if dims[2] % band:
                    continue
                smpq.smpq_set_tuning(c, *tune, band)
                out32 = smpq.smpq_apply_dw(c, psi, dagger=dag, precision=smpq.SMPQ_MIXED_FP32)
                assert np.abs(out32 - ref).max() <= 2e-6 * np.abs(ref).max(), (tune, band)
            out64 = smpq.smpq_apply_dw(c, psi, dagger=dag, precision=smpq.SMPQ_FP64)
            assert np.abs(out64 - ref).max() <= 1e-13 * np.abs(ref).max(), tune
        for tune in RL_VARIANTS:
            for il in INTERLEAVES:
                smpq.smpq_set_tuning(c, *tune, 1, 0, 4, il)
                out32 = smpq.smpq_apply_dw(c, psi, dagger=dag, precision=smpq.SMPQ_MIXED_FP32)
                assert np.abs(out32 - ref).max() <= 2e-6 * np.abs(ref).max(), (tune, il)
        # D_W and D_W^dag on different variants: each direction runs its own
        for d_w, d_dag in (((1, 8, 1), (4, 1, 2)), ((4, 1, 2), (3, 16, 1))):
            smpq.smpq_set_tuning(c, d_w[0], d_w[1], 1, 1, 0, 4, d_w[2], 1, *d_dag)
            out32 = smpq.smpq_apply_dw(c, psi, dagger=dag, precision=smpq.SMPQ_MIXED_FP32)
            assert np.abs(out32 - ref).max() <= 2e-6 * np.abs(ref).max(), (d_w, d_dag)
        # the FP64 xy-tile kernel: here the tile is the whole 16x16 plane (no halo rows)
        for nr in F64_TILE_NR:
            for band, il in ((1, 1), (2, 1), (1, 2), (1, 8)):
                if dims[2] % band:
                    continue
                smpq.smpq_set_tuning(c, 1, 8, 1, band, 1, nr, 1, il)
                out64 = smpq.smpq_apply_dw(c, psi, dagger=dag, precision=smpq.SMPQ_FP64)
                assert np.abs(out64 - ref).max() <= 1e-13 * np.abs(ref).max(), (nr, band, il)


def test_autotune_picks_a_valid_variant_and_keeps_parity():
    dims = (16, 16, 2, 2)
    print(f"autotune on {dims}", flush=True)
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.5, 13)
    psi = si.random_spinors(dims, 3, 14)
    c = _ctx(dims, U)
    t = smpq.smpq_autotune(c, 8)
    assert smpq.smpq_get_tuning(c) == t
    assert (t["f32_kind"], t["f32_nr"]) in [(k, n) for k, n, _ in SITE_VARIANTS + PLANE_VARIANTS + TILE_VARIANTS
                                            + RL_VARIANTS]
    assert t["f64_lgr"] in (0, 1, 2) and t["plane_band"] in (1, 2)
    assert (t["f64_kind"], t["f64_nr"]) in [(0, t["f64_nr"])] + [(1, n) for n in F64_TILE_NR]
    assert t["f32_interleave"] in ((1, 2, 4, 8) if t["f32_kind"] == 4 else (1,))
    assert (t["f32_dag_kind"], t["f32_dag_nr"]) in [(k, n) for k, n, _ in SITE_VARIANTS + PLANE_VARIANTS
                                                    + TILE_VARIANTS + RL_VARIANTS]
    assert t["f32_dag_interleave"] in ((1, 2, 4, 8) if t["f32_dag_kind"] == 4 else (1,))
    assert t["f64_interleave"] in ((1, 2, 4, 8) if t["f64_kind"] == 1 else (1,))
    ref = np.stack([apply_dw(U, lat, KAPPA, p) for p in psi])
    out32 = smpq.smpq_apply_dw(c, psi, precision=smpq.SMPQ_MIXED_FP32)
    assert np.abs(out32 - ref).max() <= 2e-6 * np.abs(ref).max()
    out64 = smpq.smpq_apply_dw(c, psi, precision=smpq.SMPQ_FP64)
    assert np.abs(out64 - ref).max() <= 1e-13 * np.abs(ref).max()
    # n_rhs = 0: timed on the batch a whole map would use, which needs a scheme and coefficients
    with pytest.raises(smpq.SmpqError) as e:
        smpq.smpq_autotune(c, 0)
    assert e.value.status == -6
    smpq.smpq_set_scheme(c, (2, 2, 2, 2), 0)
    smpq.smpq_set_zolotarev(c, 14, 0.15, 2.75)
    t0 = smpq.smpq_autotune(c, 0)
    assert (t0["f32_kind"], t0["f32_nr"]) in [(k, n) for k, n, _ in SITE_VARIANTS + PLANE_VARIANTS + TILE_VARIANTS
                                              + RL_VARIANTS]
    out32 = smpq.smpq_apply_dw(c, psi, precision=smpq.SMPQ_MIXED_FP32)
    assert np.abs(out32 - ref).max() <= 2e-6 * np.abs(ref).max()


@pytest.mark.parametrize("dims", [(24, 16, 2, 2), (32, 16, 4, 3), (8, 64, 2, 2)])
@pytest.mark.parametrize("nrhs", [1, 9, 17])
def test_dslash_parity_xy_tiles(dims, nrhs):
    """xy-tiles of ty < ny rows with halo rows staged in LDS (ty = 8, 8, 32), 4, 8 and 16
    right-hand sides per thread, against the oracle."""
    print(f"xy-tile dslash parity dims={dims} nrhs={nrhs}", flush=True)
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.5, 15)
    psi = si.random_spinors(dims, nrhs, 16)
    c = _ctx(dims, U)
    for kind in (1, 3):
        with pytest.raises(smpq.SmpqError):
            smpq.smpq_set_tuning(c, kind, 8, 1)
    for dag in (False, True):
        ref = np.stack([apply_dw(U, lat, KAPPA, p, dagger=dag) for p in psi])
        for tune in TILE_VARIANTS + RL_VARIANTS:
            for band in (1, 2, 4):
                if dims[2] % band:
                    continue
                smpq.smpq_set_tuning(c, *tune, band)
                out32 = smpq.smpq_apply_dw(c, psi, dagger=dag, precision=smpq.SMPQ_MIXED_FP32)
                assert np.abs(out32 - ref).max() <= 2e-6 * np.abs(ref).max(), (tune, band)
        for tune in RL_VARIANTS:
            for il in INTERLEAVES:
                smpq.smpq_set_tuning(c, *tune, 1, 0, 4, il)
                out32 = smpq.smpq_apply_dw(c, psi, dagger=dag, precision=smpq.SMPQ_MIXED_FP32)
                assert np.abs(out32 - ref).max() <= 2e-6 * np.abs(ref).max(), (tune, il)
        # the FP64 xy-tile kernel with its halo rows
        for nr in F64_TILE_NR:
            for il in (1,) + INTERLEAVES:
                smpq.smpq_set_tuning(c, 2, 8, 1, 1, 1, nr, 1, il)
                out64 = smpq.smpq_apply_dw(c, psi, dagger=dag, precision=smpq.SMPQ_FP64)
                assert np.abs(out64 - ref).max() <= 1e-13 * np.abs(ref).max(), (nr, il)
    with pytest.raises(smpq.SmpqError):           # FP64 tile: 2, 4 or 8 right-hand sides per block
        smpq.smpq_set_tuning(c, 2, 8, 1, 1, 1, 16)
    with pytest.raises(smpq.SmpqError):           # the band must divide nz
        smpq.smpq_set_tuning(c, 2, 8, 1, 3)


@functools.lru_cache(maxsize=None)
def _tiled_qx_reference(dims):
    """The oracle's q(x) of class 5 (r = 2) on a near-identity field: one solve per lattice,
    shared by every stencil variant below."""
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.3, 13)
    lo, hi = _zolo_interval(U, lat)
    col, _ = colouring(lat, (2, 2, 2, 2), 0)
    return U, lo, hi, qx_probing(U, lat, KAPPA, zolotarev(14, lo, hi), col, [5], TOL, 5000)


@pytest.mark.parametrize("dims,kind,band,il", [((16, 16, 2, 2), 1, 1, 1), ((16, 16, 2, 2), 2, 2, 1),
                                                ((24, 16, 2, 2), 2, 2, 1), ((16, 16, 2, 2), 3, 2, 1),
                                                ((16, 16, 2, 2), 4, 1, 1), ((24, 16, 2, 2), 4, 2, 1),
                                                ((16, 16, 2, 2), 4, 1, 4), ((24, 16, 2, 2), 4, 2, 2)])
def test_qx_plane_tiled_mixed(dims, kind, band, il):
    print(f"q(x) of class 5 on {dims}, kind {kind}, band {band}, interleave {il}", flush=True)
    U, lo, hi, ref = _tiled_qx_reference(dims)
    c = _ctx(dims, U)
    # with kind 4 the reliable updates' FP64 stencils run on the FP64 tile kernel with one
    # right-hand side per block (the solver's pick at 16^3x32), else on the lane kernel
    tile64 = kind == 4
    smpq.smpq_set_tuning(c, kind, 8, 1, band, 1 if tile64 else 0, 1 if tile64 else 4, il if tile64 else 1,
                         il if tile64 else 1)
    smpq.smpq_set_scheme(c, (2, 2, 2, 2), 0)
    smpq.smpq_set_zolotarev(c, 14, lo, hi)
    smpq.smpq_set_solver(c, smpq.SMPQ_MIXED_FP32, TOL, 5000, 50)
    q32 = smpq.smpq_compute_qx_classes(c, [5])[0]
    assert np.abs(q32 - ref.real).max() < 1e-5
    # the FP64 path with the FP64 xy-tile stencil (in the solver: both fused epilogues)
    smpq.smpq_set_tuning(c, kind, 8, 1, band, 1, 1 if tile64 else 4, il if tile64 else 1, il)
    smpq.smpq_set_solver(c, smpq.SMPQ_FP64, TOL, 5000, 0)
    q64 = smpq.smpq_compute_qx_classes(c, [5])[0]
    assert np.abs(q64 - ref.real).max() < 1e-10 * np.abs(ref.real).max()


@pytest.mark.parametrize("d_w,d_dag", [((1, 8, 1), (4, 1, 2)), ((4, 1, 2), (3, 16, 1))])
def test_qx_split_stencil_variants(d_w, d_dag):
    """The first stencil of each CG iteration (D_W p with its partial sums) and the second (D_W^dag
    with the residual update) on different variants, each with its own partial count: the mixed
    q(x) of class 5 against the oracle."""
    dims = (16, 16, 2, 2)
    print(f"q(x) with D_W on {d_w} and D_W^dag on {d_dag}", flush=True)
    U, lo, hi, ref = _tiled_qx_reference(dims)
    c = _ctx(dims, U)
    smpq.smpq_set_tuning(c, d_w[0], d_w[1], 1, 1, 0, 4, d_w[2], 1, *d_dag)
    smpq.smpq_set_scheme(c, (2, 2, 2, 2), 0)
    smpq.smpq_set_zolotarev(c, 14, lo, hi)
    smpq.smpq_set_solver(c, smpq.SMPQ_MIXED_FP32, TOL, 5000, 50)
    q32 = smpq.smpq_compute_qx_classes(c, [5])[0]
    assert np.abs(q32 - ref.real).max() < 1e-5


def test_dslash_gamma5_hermiticity_and_adjoint():
    dims = (6, 4, 4, 6)
    U = si.near_identity_su3(dims, 0.5, 3)
    chi, psi = si.random_spinors(dims, 2, 4)
    c = _ctx(dims, U)
    d = smpq.smpq_apply_dw(c, psi)[0]
    dd = smpq.smpq_apply_dw(c, chi, dagger=True)[0]
    assert abs(np.vdot(chi, d) - np.vdot(dd, psi)) < 1e-12 * abs(np.vdot(chi, d))
    g5 = apply_gamma5(smpq.smpq_apply_dw(c, apply_gamma5(psi))[0])
    assert np.abs(g5 - smpq.smpq_apply_dw(c, psi, dagger=True)[0]).max() < 1e-13


def test_lanczos_matches_dense_and_oracle():
    dims = (4, 4, 2, 2)
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.3, 5)
    w = np.linalg.eigvalsh(h_dense(U, lat, KAPPA))
    c = _ctx(dims, U)
    tmin, tmax = smpq.smpq_lanczos(c, 300, 0)
    assert abs(tmin - (w ** 2).min()) < 1e-5 * (w ** 2).min()   # no reorthogonalisation on the GPU
    assert abs(tmax - (w ** 2).max()) < 1e-10 * (w ** 2).max()
    omin, omax = ritz_extremes(U, lat, KAPPA, 40, seed=0)
    gmin, gmax = smpq.smpq_lanczos(c, 40, 0)
    assert abs(gmax - omax) < 1e-8 * omax          # same start vector, same steps
    assert abs(gmin - omin) < 1e-3 * omin
    lo, hi = smpq.smpq_estimate_bounds(c, 300)
    assert lo < np.abs(w).min() and hi > np.abs(w).max()


def test_apply_dov_parity():
    dims = (4, 4, 4, 4)
    lat = Lattice(dims)
    U = si.workload("noise4")
    lo, hi = 0.13, 2.62
    zo = zolotarev(14, lo, hi)
    b = si.random_spinors(dims, 2, 6)
    c = _ctx(dims, U)
    smpq.smpq_set_zolotarev(c, 14, lo, hi)
    smpq.smpq_set_solver(c, smpq.SMPQ_FP64, TOL, 5000, 0)
    out = smpq.smpq_apply_dov(c, b)
    for k in range(2):
        ref = dov_apply(U, lat, KAPPA, zo, b[k], TOL, 5000)
        assert np.abs(out[k] - ref).max() < 1e-10 * np.abs(ref).max()
    # eps^2 = 1 on the GPU: eps = gamma5 (D_ov - 1)
    e1 = apply_gamma5(out - b)
    e2 = apply_gamma5(smpq.smpq_apply_dov(c, e1) - e1)
    assert np.abs(e2 - b).max() < 1e-9 * np.abs(b).max()


def _ragged_setup():
    dims = (6, 4, 4, 6)
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.3, 7)
    lo, hi = _zolo_interval(U, lat)
    return dims, lat, U, lo, hi


def test_qx_point_sources_fp64():
    dims, lat, U, lo, hi = _ragged_setup()
    zo = zolotarev(14, lo, hi)
    sites = np.array([0, 300, 575])
    c = _ctx(dims, U)
    smpq.smpq_set_zolotarev(c, 14, lo, hi)
    smpq.smpq_set_solver(c, smpq.SMPQ_FP64, TOL, 5000, 0)
    q, st = smpq.smpq_compute_qx_points(c, sites)
    col, _ = point_colouring(lat)
    ref = qx_probing(U, lat, KAPPA, zo, col, sites, TOL, 5000)[sites].real
    err = np.abs(q - ref).max()
    print(f"point sources: max |dq| {err:.3e}, largest |q| {np.abs(ref).max():.3e}", flush=True)
    assert err < 1e-10 * np.abs(ref).max()
    assert st["n_sources"] == 36


@pytest.mark.parametrize("mode,r", [(0, 2), (1, 2), (2, 2)])
def test_qx_smp_classes_fp64_and_mixed(mode, r):
    dims = (4, 4, 4, 8) if mode != 0 else (6, 4, 4, 6)
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.3, 8)
    lo, hi = _zolo_interval(U, lat)
    zo = zolotarev(14, lo, hi)
    col, ncls = colouring(lat, (r,) * 4, mode)
    classes = [0, ncls - 1]
    c = _ctx(dims, U)
    nc, ns = smpq.smpq_set_scheme(c, (r,) * 4, mode)
    assert nc == ncls and ns == 12 * ncls
    assert np.array_equal(smpq.smpq_get_coloring(c), col)
    smpq.smpq_set_zolotarev(c, 14, lo, hi)
    ref = qx_probing(U, lat, KAPPA, zo, col, classes, TOL, 5000)
    smpq.smpq_set_solver(c, smpq.SMPQ_FP64, TOL, 5000, 0)
    q64, qi64, st = smpq.smpq_compute_qx_classes(c, classes)
    scale = np.abs(ref.real).max()
    err = np.abs(q64 - ref.real).max()
    print(f"mode {mode}: max |dq| {err:.3e}, largest |q| {scale:.3e}", flush=True)
    assert err < 1e-10 * scale
    assert np.abs(qi64 - ref.imag).max() < 1e-10 * scale
    smpq.smpq_set_solver(c, smpq.SMPQ_MIXED_FP32, TOL, 5000, 50)
    q32, qi32, st32 = smpq.smpq_compute_qx_classes(c, classes)
    assert np.abs(q32 - ref.real).max() < 1e-5
    assert st32["n_reliable_updates"] > 0


def test_free_field_density_is_zero():
    dims = (6, 4, 4, 6)
    V = int(np.prod(dims))
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:] = np.eye(3)
    c = _ctx(dims, U)
    smpq.smpq_set_zolotarev(c, 14, 0.15, 2.7)
    smpq.smpq_set_scheme(c, (2, 2, 2, 2), 0)
    for prec in (smpq.SMPQ_FP64, smpq.SMPQ_MIXED_FP32):
        smpq.smpq_set_solver(c, prec, TOL, 5000, 50)
        q, qi, Q, st = smpq.smpq_compute_qx(c)
        assert np.abs(q).max() < (1e-12 if prec == smpq.SMPQ_FP64 else 1e-6)
        assert abs(Q) < (1e-10 if prec == smpq.SMPQ_FP64 else 1e-4)


def test_gauge_covariance_of_point_density():
    dims, lat, U, lo, hi = _ragged_setup()
    Ug = si.gauge_transform(U, dims, si.haar_su3(lat.volume, 9))
    sites = np.array([5, 402])
    out = []
    for field in (U, Ug):
        c = _ctx(dims, field)
        smpq.smpq_set_zolotarev(c, 14, lo, hi)
        out.append(smpq.smpq_compute_qx_points(c, sites)[0])
    assert np.abs(out[0] - out[1]).max() < 1e-11


def test_deterministic_and_errors():
    dims, lat, U, lo, hi = _ragged_setup()
    c = _ctx(dims, U)
    smpq.smpq_set_zolotarev(c, 14, lo, hi)
    smpq.smpq_set_scheme(c, (2, 2, 2, 2), 0)
    a = smpq.smpq_compute_qx_classes(c, [3])[0]
    b = smpq.smpq_compute_qx_classes(c, [3])[0]
    assert np.array_equal(a, b)
    smpq.smpq_set_solver(c, smpq.SMPQ_FP64, TOL, 3, 0)
    with pytest.raises(smpq.SmpqError) as e:
        smpq.smpq_compute_qx_classes(c, [3])
    assert e.value.status == -5
    with pytest.raises(smpq.SmpqError):
        smpq.smpq_compute_qx_classes(c, [99])
    bad = U.copy()
    bad[0, 0] *= 1.01
    with pytest.raises(smpq.SmpqError) as e:
        smpq.smpq_load_gauge(c, bad)
    assert e.value.status == -7


@pytest.mark.parametrize("prec", [0, 1])
def test_graphs_match_eager_and_timed(prec):
    """Captured groups of iterations (with and without event nodes) give bitwise the same q(x)
    as eager launches; a smaller batch afterwards re-captures against the new layout."""
    dims, lat, U, lo, hi = _ragged_setup()
    c = _ctx(dims, U)
    smpq.smpq_set_zolotarev(c, 14, lo, hi)
    smpq.smpq_set_scheme(c, (2, 2, 2, 2), 0)
    smpq.smpq_set_solver(c, prec, TOL, 5000, 50)
    out = []
    for graphs, timing in ((True, False), (False, False), (True, True), (False, True)):
        smpq.smpq_set_graphs(c, graphs)
        smpq.smpq_set_timing(c, timing)
        q, qi, st = smpq.smpq_compute_qx_classes(c, [1, 6, 9])
        out.append(q)
        if timing:
            assert st["dslash_ms"] > 0 and st["update_ms"] > 0 and st["dslash_launches"] > 0
    for q in out[1:]:
        assert np.array_equal(q, out[0])
    smpq.smpq_set_graphs(c, True)
    smpq.smpq_set_timing(c, False)
    smpq.smpq_set_batch(c, 12)
    q2 = smpq.smpq_compute_qx_classes(c, [1, 6, 9])[0]
    assert np.abs(q2 - out[0]).max() < (1e-13 if prec == 0 else 1e-6)


@pytest.mark.parametrize("prec", [smpq.SMPQ_FP64, smpq.SMPQ_MIXED_FP32])
def test_dov_locality_matches_oracle(prec):
    """Mean absolute block entries of D_ov around one site (Eq. 12) against the oracle's twelve
    point-source columns; FP64 1e-10, mixed 2e-6 (entries are at most ~1)."""
    from oracle.locality import block_mean_abs
    dims = (4, 4, 4, 4)
    print(f"D_ov locality on noise4, precision {prec}", flush=True)
    lat = Lattice(dims)
    U = si.workload("noise4")
    lo, hi = 0.13, 2.62
    zo = zolotarev(14, lo, hi)
    site = 37
    ref = block_mean_abs(U, lat, KAPPA, zo[:3], site, TOL, 5000)
    c = _ctx(dims, U)
    smpq.smpq_set_zolotarev(c, 14, lo, hi)
    smpq.smpq_set_solver(c, prec, TOL, 5000, 50 if prec == smpq.SMPQ_MIXED_FP32 else 0)
    m, st = smpq.smpq_dov_locality(c, site)
    assert st["n_sources"] == 12
    assert np.abs(m - ref).max() < (1e-10 if prec == smpq.SMPQ_FP64 else 2e-6)
    assert m[site] == m.max()
