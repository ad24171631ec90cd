"""Pins of the oracle's Lanczos bounds and multi-shift CG (Eq. 4, Eqs. 6-8)."""
import numpy as np
import pytest

import smpq_inputs as si
from oracle.dirac import apply_h2, h_dense
from oracle.lanczos import bounds, ritz_extremes, splitmix64_uniform, start_vector
from oracle.lattice import Lattice
from oracle.mscg import NotConverged, cg, multishift_cg

KAPPA = 0.21


def test_splitmix64_reference_outputs():
    """First outputs of SplitMix64 from state 0, as published with the generator."""
    u = splitmix64_uniform(0, 4)
    words = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    assert np.array_equal(u, np.array([(w >> 11) * 2.0 ** -53 for w in words]))
    v = start_vector(3, 5)
    assert v.shape == (3, 4, 3) and np.abs(v.real).max() <= 1 and np.abs(v.imag).max() <= 1


def test_lanczos_extremes_match_dense_spectrum():
    dims = (4, 2, 2, 4)
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.3, 2)
    w = np.linalg.eigvalsh(h_dense(U, lat, KAPPA))
    tmin, tmax = ritz_extremes(U, lat, KAPPA, 300)
    assert abs(tmin - (w ** 2).min()) < 1e-7 * (w ** 2).min()
    assert abs(tmax - (w ** 2).max()) < 1e-10 * (w ** 2).max()
    # Ritz values lie inside the spectrum
    t60 = ritz_extremes(U, lat, KAPPA, 60)
    assert t60[0] >= (w ** 2).min() and t60[1] <= (w ** 2).max()
    lo, hi = bounds(U, lat, KAPPA, 100)
    assert lo < np.abs(w).min() and hi > np.abs(w).max()


def _setup(dims=(2, 2, 2, 4), seed=4):
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.3, seed)
    (b,) = si.random_spinors(dims, 1, seed + 1)
    return lat, U, b


def test_multishift_matches_dense_solves():
    lat, U, b = _setup()
    h2 = h_dense(U, lat, KAPPA)
    h2 = h2 @ h2
    shifts = np.array([1e-4, 3e-3, 0.05, 0.7, 9.0])
    s = shifts.min()
    x, iters = multishift_cg(lambda v: apply_h2(U, lat, KAPPA, v) + s * v, b, shifts - s, 1e-12, 1000)
    for xi, qi in zip(x, shifts):
        exact = np.linalg.solve(h2 + qi * np.eye(len(h2)), b.reshape(-1))
        assert np.abs(xi.reshape(-1) - exact).max() < 1e-9 * np.abs(exact).max()
    # larger shifts are better conditioned and stop earlier
    assert np.all(np.diff(iters) <= 0)


def test_multishift_true_residuals_and_single_shift_cg():
    lat, U, b = _setup((2, 4, 2, 2), 8)
    shifts = np.array([2e-3, 0.1, 1.5])
    s = shifts.min()
    tol = 1e-11
    x, iters = multishift_cg(lambda v: apply_h2(U, lat, KAPPA, v) + s * v, b, shifts - s, tol, 1000)
    bn = np.sqrt(np.vdot(b, b).real)
    for xi, qi, it in zip(x, shifts, iters):
        res = b - apply_h2(U, lat, KAPPA, xi) - qi * xi
        assert np.sqrt(np.vdot(res, res).real) <= 10 * tol * bn
        xc, itc = cg(lambda v: apply_h2(U, lat, KAPPA, v) + qi * v, b, tol, 1000)
        assert abs(itc - it) <= 1
        assert np.abs(xc - xi).max() < 1e-8 * np.abs(xc).max()


def test_multishift_errors():
    lat, U, b = _setup()
    with pytest.raises(NotConverged):
        multishift_cg(lambda v: apply_h2(U, lat, KAPPA, v), b, [0.0, 1.0], 1e-12, 3)
    with pytest.raises(FloatingPointError):
        multishift_cg(lambda v: -v, b, [0.0], 1e-12, 10)
    x, iters = multishift_cg(lambda v: v, np.zeros_like(b), [0.0, 1.0], 1e-12, 10)
    assert all(np.all(xi == 0) for xi in x)
