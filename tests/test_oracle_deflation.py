"""Pins of the oracle's low-mode deflation of eps(H_W)."""
import numpy as np
import pytest

import smpq_inputs as si
from oracle.charge import eps_apply, eps_dense, h_spectrum, qx_from_eps
from oracle.deflation import eps_apply_deflated, eps_dense_deflated, low_modes, qx_probing_deflated
from oracle.lattice import Lattice
from oracle.probing import point_colouring
from oracle.zolotarev import eps_scalar, zolotarev

KAPPA, TOL = 0.21, 1e-12
K = 6          # rough4: |lambda| jumps from 0.1160 to 0.1272 after the sixth mode


@pytest.fixture(scope="module")
def rough4():
    dims = (4, 4, 4, 4)
    lat = Lattice(dims)
    U = si.workload("rough4")
    w, v = h_spectrum(U, lat, KAPPA)
    a = np.sort(np.abs(w))
    lo, hi = 0.9 * a[K], 1.02 * a[-1]
    zo = zolotarev(14, lo, hi)
    theta, u = low_modes(U, lat, KAPPA, K)
    return dims, lat, U, w, v, zo, theta, u


def test_low_modes_are_eigenpairs_of_h2(rough4):
    dims, lat, U, w, v, zo, theta, u = rough4
    a = np.sort(np.abs(w))
    assert np.abs(np.sqrt(theta) - a[:K]).max() < 1e-12
    from oracle.dirac import apply_h2
    for th, ui in zip(theta, u):
        assert np.abs(apply_h2(U, lat, KAPPA, ui) - th * ui).max() < 1e-12


def test_deflated_eps_equals_dense_construction(rough4):
    """The projection formula against V f(Lambda) V^dag with the exact sign on the deflated
    modes and the scalar Zolotarev function on the rest."""
    dims, lat, U, w, v, zo, theta, u = rough4
    dense = eps_dense_deflated(w, v, K, lambda x: eps_scalar(x, zo[0], zo[1], zo[2]))
    b = si.random_spinors(dims, 1, 33)[0]
    got = eps_apply_deflated(U, lat, KAPPA, zo[:3], theta, u, b, TOL, 5000)
    ref = (dense @ b.reshape(-1)).reshape(b.shape)
    assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max()


def test_deflation_repairs_the_narrow_interval(rough4):
    """With the interval above the low modes, eps^2 = 1 holds only with deflation."""
    dims, lat, U, w, v, zo, theta, u = rough4
    b = si.random_spinors(dims, 1, 34)[0]
    e1 = eps_apply_deflated(U, lat, KAPPA, zo[:3], theta, u, b, TOL, 5000)
    e2 = eps_apply_deflated(U, lat, KAPPA, zo[:3], theta, u, e1, TOL, 5000)
    err_defl = np.abs(e2 - b).max() / np.abs(b).max()
    f1, _ = eps_apply(U, lat, KAPPA, zo[:3], b, TOL, 5000)
    f2, _ = eps_apply(U, lat, KAPPA, zo[:3], f1, TOL, 5000)
    err_plain = np.abs(f2 - b).max() / np.abs(b).max()
    print(f"|eps^2 b - b| / |b|: deflated {err_defl:.2e}, not deflated {err_plain:.2e}")
    assert err_defl < 1e-10 and err_plain > 100 * err_defl
    # and with no modes it is the plain Zolotarev application
    g, _ = eps_apply(U, lat, KAPPA, zo[:3], b, TOL, 5000)
    assert np.array_equal(eps_apply_deflated(U, lat, KAPPA, zo[:3], theta[:0], u[:0], b, TOL, 5000), g)


def test_deflated_point_density_is_the_exact_density(rough4):
    """Point sources with deflation give the exact q(x) of the sign function (Eq. 5) to the
    Zolotarev error on the undeflated part."""
    dims, lat, U, w, v, zo, theta, u = rough4
    col, n = point_colouring(lat)
    sites = [0, 1, 17, 200]
    q = qx_probing_deflated(U, lat, KAPPA, zo[:3], theta, u, col, sites, TOL, 5000)
    exact = qx_from_eps(eps_dense(w, v), lat.volume)
    assert np.abs(q[sites].real - exact[sites]).max() < 1e-10
