"""Pins of the oracle's q(x) (Eqs. 2, 3, 5, 16): dense sign function, invariants, closed forms."""
import numpy as np
import pytest

import smpq_inputs as si
from oracle.charge import (charge_from_spectrum, dov_apply, eps_apply, eps_dense, h_spectrum,
                           qx_from_eps, qx_probing, qx_smp_from_eps)
from oracle.dirac import GAMMA5, apply_gamma5, h_dense
from oracle.lattice import Lattice
from oracle.probing import colouring, point_colouring
from oracle.zolotarev import eps_scalar, zolotarev

KAPPA = 0.21
TOL = 1e-12


def _zolo(U, lat):
    w = np.linalg.eigvalsh(h_dense(U, lat, KAPPA))
    return zolotarev(14, 0.9 * np.abs(w).min(), 1.02 * np.abs(w).max())


def test_free_field_density_vanishes():
    """Free field: tr_s gamma5 (M + i gamma.s) R = 0, so q(x) = 0 for points and probes."""
    dims = (2, 2, 2, 4)
    lat = Lattice(dims)
    U = np.zeros((lat.volume, 4, 3, 3), dtype=np.complex128)
    U[:] = np.eye(3)
    zo = zolotarev(14, 0.15, 2.7)
    col, _ = point_colouring(lat)
    q = qx_probing(U, lat, KAPPA, zo, col, [0, 9], TOL, 1000)
    assert np.abs(q).max() < 1e-12
    col, _ = colouring(lat, (2, 2, 2, 2), 0)
    q = qx_probing(U, lat, KAPPA, zo, col, [1], TOL, 1000)
    assert np.abs(q).max() < 1e-12


def test_point_sources_match_dense_sign():
    """Point-source q(x) through the multi-shift CG equals the dense eps_Z diagonal (Eq. 5)."""
    dims = (4, 2, 2, 2)
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.4, 3)
    w, v = h_spectrum(U, lat, KAPPA)
    zo = zolotarev(14, 0.9 * np.abs(w).min(), 1.02 * np.abs(w).max())
    exact = qx_from_eps(eps_dense(w, v), lat.volume)
    zq = qx_from_eps(eps_dense(w, v, lambda x: eps_scalar(x, *zo[:3])), lat.volume)
    assert np.abs(zq - exact).max() <= 6 * zo[3] + 1e-13           # 12 diagonal entries / 2
    col, _ = point_colouring(lat)
    sites = [0, 5, 30]
    q = qx_probing(U, lat, KAPPA, zo, col, sites, TOL, 2000)
    assert np.abs(q[sites].real - zq[sites]).max() < 1e-11
    assert np.abs(q[sites].imag).max() < 1e-14
    # exact charge is the spectral asymmetry (an integer), and sum_x q(x) equals it
    assert abs(exact.sum() - charge_from_spectrum(w)) < 1e-11


def test_sign_squares_to_one_and_ginsparg_wilson():
    """eps^2 = 1 and gamma5 D + D gamma5 = D gamma5 D, to the Zolotarev + CG error."""
    dims = (2, 4, 2, 2)
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.3, 5)
    zo = _zolo(U, lat)
    (b,) = si.random_spinors(dims, 1, 6)
    e1, _ = eps_apply(U, lat, KAPPA, zo, b, TOL, 2000)
    e2, _ = eps_apply(U, lat, KAPPA, zo, e1, TOL, 2000)
    nb = np.abs(b).max()
    assert np.abs(e2 - b).max() < 1e-9 * nb
    d = lambda v: dov_apply(U, lat, KAPPA, zo, v, TOL, 2000)
    lhs = apply_gamma5(d(b)) + d(apply_gamma5(b))
    rhs = d(apply_gamma5(d(b)))
    assert np.abs(lhs - rhs).max() < 1e-9 * nb


def test_gauge_invariance_of_point_density():
    dims = (2, 2, 4, 2)
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.3, 7)
    Ug = si.gauge_transform(U, dims, si.haar_su3(lat.volume, 8))
    zo = _zolo(U, lat)
    col, _ = point_colouring(lat)
    sites = [3, 17]
    q0 = qx_probing(U, lat, KAPPA, zo, col, sites, TOL, 2000)
    q1 = qx_probing(Ug, lat, KAPPA, zo, col, sites, TOL, 2000)
    assert np.abs(q0 - q1).max() < 1e-11


def test_flux_background_charge():
    """U(1) flux (n12, n34) = (1, 1) embedded with charges (+1, -1, 0): Q = 2 (index theorem)."""
    dims = (4, 4, 4, 4)
    lat = Lattice(dims)
    U = si.u1_flux(dims, 1, 1)
    w = np.linalg.eigvalsh(h_dense(U, lat, KAPPA))
    assert charge_from_spectrum(w) == 2.0
    U = si.u1_flux(dims, 1, -1)
    w = np.linalg.eigvalsh(h_dense(U, lat, KAPPA))
    assert charge_from_spectrum(w) == -2.0


def test_smp_matches_dense_identity():
    """Eq. 16 from CG-probed sources equals the same sum taken from the dense eps_Z."""
    dims = (4, 4, 2, 2)
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.3, 9)
    w, v = h_spectrum(U, lat, KAPPA)
    zo = zolotarev(14, 0.9 * np.abs(w).min(), 1.02 * np.abs(w).max())
    epsz = eps_dense(w, v, lambda x: eps_scalar(x, *zo[:3]))
    col, ncls = colouring(lat, (2, 2, 2, 2), 0)
    dense = qx_smp_from_eps(epsz, col)
    cls = [0, 7]
    q = qx_probing(U, lat, KAPPA, zo, col, cls, TOL, 2000)
    mask = np.isin(col, cls)
    assert np.abs(q[mask] - dense[mask]).max() < 1e-11
    # the imaginary parts of one class sum to zero (phi^dag eps phi is real)
    for c in cls:
        assert abs(q[col == c].imag.sum()) < 1e-13
    # probing differs from the exact density only by off-diagonal terms
    exact = qx_from_eps(epsz, lat.volume)
    off = np.zeros(lat.volume, dtype=complex)
    g5d = np.kron(np.eye(lat.volume), np.kron(GAMMA5, np.eye(3))) + epsz
    for x in np.nonzero(mask)[0]:
        for y in np.nonzero(col == col[x])[0]:
            if y != x:
                off[x] += 0.5 * sum(g5d[12 * x + j, 12 * y + j] for j in range(12))
    assert np.abs(q[mask] - exact[mask] - off[mask]).max() < 1e-11


def test_single_site_classes_reduce_to_point_sources():
    """r = n in every direction (or a 2^4 lattice with r = 2) gives one site per class."""
    dims = (2, 2, 2, 2)
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.3, 12)
    zo = _zolo(U, lat)
    col, ncls = colouring(lat, (2, 2, 2, 2), 0)
    assert ncls == lat.volume
    qs = qx_probing(U, lat, KAPPA, zo, col, [col[4]], TOL, 2000)
    pc, _ = point_colouring(lat)
    qp = qx_probing(U, lat, KAPPA, zo, pc, [4], TOL, 2000)
    assert qs[4] == qp[4]
