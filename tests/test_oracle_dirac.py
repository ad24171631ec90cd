"""Pins of the oracle's Wilson kernel (section 1, Eq. 3) against closed forms and invariants."""
import itertools

import numpy as np
import pytest

import smpq_inputs as si
from oracle.dirac import GAMMA, GAMMA5, apply_dw, apply_gamma5, apply_h, apply_h2, dw_sparse, h_dense
from oracle.lattice import Lattice

KAPPA = 0.21


def test_gamma_algebra():
    """Euclidean hermitian gamma matrices: {g_mu, g_nu} = 2 delta, g5 = g1 g2 g3 g4 = diag(1,1,-1,-1)."""
    for mu, nu in itertools.product(range(4), repeat=2):
        anti = GAMMA[mu] @ GAMMA[nu] + GAMMA[nu] @ GAMMA[mu]
        assert np.allclose(anti, 2.0 * np.eye(4) * (mu == nu), atol=0)
        assert np.allclose(GAMMA[mu], GAMMA[mu].conj().T, atol=0)
    assert np.array_equal(GAMMA5, np.diag([1, 1, -1, -1]).astype(complex))
    for mu in range(4):
        assert np.allclose(GAMMA5 @ GAMMA[mu], -GAMMA[mu] @ GAMMA5, atol=0)


def _free(lat):
    U = np.zeros((lat.volume, 4, 3, 3), dtype=np.complex128)
    U[:] = np.eye(3)
    return U


def test_free_field_plane_waves():
    """Free field: D_W e^{ipx} u = [1 - 2k sum cos p + 2ik sum gamma sin p] e^{ipx} u."""
    dims = (4, 6, 2, 8)
    lat = Lattice(dims)
    U = _free(lat)
    rng = np.random.default_rng(7)
    for _ in range(5):
        n = [rng.integers(0, d) for d in dims]
        p = 2 * np.pi * np.array(n) / np.array(dims)
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        wave = np.exp(1j * lat.coords @ p)
        psi = wave[:, None, None] * u[None]
        dp = (1 - 2 * KAPPA * np.cos(p).sum()) * np.eye(4) + 2j * KAPPA * sum(
            GAMMA[mu] * np.sin(p[mu]) for mu in range(4))
        expect = wave[:, None, None] * (dp @ u)[None]
        assert np.abs(apply_dw(U, lat, KAPPA, psi) - expect).max() < 1e-13


def test_free_field_spectrum_dense():
    """|H_W(p)| = sqrt((1 - 2k sum cos p)^2 + 4 k^2 sum sin^2 p), 6 times with each sign."""
    dims = (4, 2, 2, 4)
    lat = Lattice(dims)
    w = np.linalg.eigvalsh(h_dense(_free(lat), lat, KAPPA))
    expect = []
    for n in itertools.product(*[range(d) for d in dims]):
        p = 2 * np.pi * np.array(n) / np.array(dims)
        e = np.sqrt((1 - 2 * KAPPA * np.cos(p).sum()) ** 2 + 4 * KAPPA ** 2 * (np.sin(p) ** 2).sum())
        expect += [e] * 6 + [-e] * 6
    assert np.abs(np.sort(w) - np.sort(expect)).max() < 1e-12
    # spectrum of |H_W| on the free field: [|1 - 4 kappa|, 1 + 8 kappa] for even extents
    assert abs(np.abs(w).min() - abs(1 - 4 * KAPPA)) < 1e-12
    assert abs(np.abs(w).max() - (1 + 8 * KAPPA)) < 1e-12


def _rand_field(dims, seed):
    return si.near_identity_su3(dims, 0.5, seed)


def test_adjoint_and_gamma5_hermiticity():
    """<chi, D_W psi> = <D_W^dag chi, psi> and D_W^dag = gamma5 D_W gamma5."""
    dims = (4, 2, 6, 2)
    lat = Lattice(dims)
    U = _rand_field(dims, 3)
    chi, psi = si.random_spinors(dims, 2, 11)
    lhs = np.vdot(chi, apply_dw(U, lat, KAPPA, psi))
    rhs = np.vdot(apply_dw(U, lat, KAPPA, chi, dagger=True), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    g5dg5 = apply_gamma5(apply_dw(U, lat, KAPPA, apply_gamma5(psi)))
    assert np.abs(g5dg5 - apply_dw(U, lat, KAPPA, psi, dagger=True)).max() < 1e-13
    # H = gamma5 D_W is hermitian and H^2 = D_W^dag D_W is positive
    assert abs(np.vdot(chi, apply_h(U, lat, KAPPA, psi)) - np.vdot(apply_h(U, lat, KAPPA, chi), psi)) < 1e-12
    assert np.vdot(psi, apply_h2(U, lat, KAPPA, psi)).real > 0


def test_gauge_covariance():
    """D_W[U^g] (g psi) = g D_W[U] psi with U_mu(x) -> g(x) U_mu(x) g(x+mu)^dag."""
    dims = (4, 4, 2, 6)
    lat = Lattice(dims)
    U = _rand_field(dims, 5)
    g = si.haar_su3(lat.volume, 9)
    Ug = si.gauge_transform(U, dims, g)
    (psi,) = si.random_spinors(dims, 1, 13)
    gpsi = np.einsum("xab,xsb->xsa", g, psi)
    for dag in (False, True):
        lhs = apply_dw(Ug, lat, KAPPA, gpsi, dagger=dag)
        rhs = np.einsum("xab,xsb->xsa", g, apply_dw(U, lat, KAPPA, psi, dagger=dag))
        assert np.abs(lhs - rhs).max() < 1e-13


def test_sparse_assembly_matches_matrix_free():
    dims = (2, 4, 2, 4)
    lat = Lattice(dims)
    U = _rand_field(dims, 21)
    (psi,) = si.random_spinors(dims, 1, 22)
    dense = dw_sparse(U, lat, KAPPA) @ psi.reshape(-1)
    assert np.abs(dense.reshape(psi.shape) - apply_dw(U, lat, KAPPA, psi)).max() < 1e-13


def test_translation_covariance():
    """Shifting the gauge field by one site shifts D_W psi the same way (periodic lattice)."""
    dims = (4, 2, 2, 6)
    lat = Lattice(dims)
    U = _rand_field(dims, 31)
    (psi,) = si.random_spinors(dims, 1, 32)
    t = lat.fwd[3]                      # site x -> x + t-hat
    Ut, psit = U[t], psi[t]
    assert np.abs(apply_dw(Ut, lat, KAPPA, psit) - apply_dw(U, lat, KAPPA, psi)[t]).max() < 1e-13


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 2)])
def test_inputs_are_su3(dims):
    U = si.near_identity_su3(dims, 0.3, 0)
    eye = np.eye(3)
    assert np.abs(U @ np.conj(np.swapaxes(U, -1, -2)) - eye).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    g = si.haar_su3(50, 1)
    assert np.abs(g @ np.conj(np.swapaxes(g, -1, -2)) - eye).max() < 1e-14
    assert np.abs(np.linalg.det(g) - 1).max() < 1e-14
