"""Seeded synthetic inputs: SU(3) gauge fields, gauge transforms and test spinors.

This module only *builds inputs*.  It holds none of the arithmetic of the method
(no Dirac operator, no sign function, no solver, no colouring), so both the CPU
oracle and the GPU path may draw their inputs from it without sharing any of the
computation they are compared on.

Field layouts (host, numpy):
  * gauge field  U[site, mu, row, col]  complex128, shape (V, 4, 3, 3)
  * spinor       psi[site, spin, colour] complex128, shape (V, 4, 3)
  * site index   s = x + nx*(y + ny*(z + nz*t)), dims = (nx, ny, nz, nt)

The paper's Iwasaki ensembles (section 3, Table 1) are not available; the
workloads below are synthetic stand-ins with the paper's lattice shapes:

  near-identity SU(3) noise  U = exp(i eps H), H Hermitian traceless, Gaussian
  U(1) constant-field-strength background embedded as diag(e^{i phi}, e^{-i phi}, 1),
      with integer flux quanta (n12, n34) in the (x,y) and (z,t) planes;
      its topological charge is 2 * n12 * n34 (two colour charges of +-1).
  Haar-random SU(3) gauge transformations.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "volume", "coords", "forward_index",
    "near_identity_su3", "u1_flux", "haar_su3", "gauge_transform", "left_multiply",
    "random_spinors", "workload",
    "WORKLOADS",
]


def volume(dims) -> int:
    nx, ny, nz, nt = (int(d) for d in dims)
    return nx * ny * nz * nt


def coords(dims) -> np.ndarray:
    """(V, 4) integer coordinates (x, y, z, t) of every site, x fastest."""
    nx, ny, nz, nt = (int(d) for d in dims)
    s = np.arange(volume(dims), dtype=np.int64)
    return np.stack([s % nx, (s // nx) % ny, (s // (nx * ny)) % nz, s // (nx * ny * nz)], axis=1)


def forward_index(dims, mu: int) -> np.ndarray:
    """Index of the site x + mu-hat (periodic) for every site x."""
    c = coords(dims).copy()
    c[:, mu] = (c[:, mu] + 1) % int(dims[mu])
    nx, ny, nz, _ = (int(d) for d in dims)
    return c[:, 0] + nx * (c[:, 1] + ny * (c[:, 2] + nz * c[:, 3]))


def _gaussian_complex(rng: np.random.Generator, shape) -> np.ndarray:
    g = rng.standard_normal(tuple(shape) + (2,))
    return g[..., 0] + 1j * g[..., 1]


def near_identity_su3(dims, eps: float, seed: int) -> np.ndarray:
    """U_mu(x) = exp(i eps H) with H random Hermitian traceless (Gaussian entries).

    A has i.i.d. N(0,1) real and imaginary parts, H = (A + A^dag)/2 - tr(.)/3,
    U = W diag(exp(i eps lambda)) W^dag from the eigendecomposition of H, so U is
    unitary with det U = exp(i eps tr H) = 1.  Draw order: numpy PCG64 with the
    given seed, one (4, V, 3, 3) array, i.e. links drawn in (mu, site) order.
    """
    V = volume(dims)
    rng = np.random.default_rng(seed)
    A = _gaussian_complex(rng, (4, V, 3, 3))
    H = 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))
    tr = np.trace(H, axis1=-2, axis2=-1)
    H = H - (tr / 3.0)[..., None, None] * np.eye(3)
    lam, W = np.linalg.eigh(H)
    U = (W * np.exp(1j * eps * lam)[..., None, :]) @ np.conj(np.swapaxes(W, -1, -2))
    return np.ascontiguousarray(np.transpose(U, (1, 0, 2, 3)))


def u1_flux(dims, n12: int, n34: int) -> np.ndarray:
    """Constant U(1) field strength embedded in SU(3) as diag(e^{i phi}, e^{-i phi}, 1).

    For the plane (a, b) with flux quanta n_ab, theta = 2 pi n_ab / (L_a L_b):
      U_b(x) <- U_b(x) E(theta x_a)                     at every site,
      U_a(x) <- U_a(x) E(-theta L_a x_b)                where x_a = L_a - 1,
    with E(phi) = diag(e^{i phi}, e^{-i phi}, 1).  Every plaquette of the plane is
    then E(theta), including the ones that wrap around the torus.
    """
    dims = tuple(int(d) for d in dims)
    V = volume(dims)
    c = coords(dims)
    phase = np.zeros((V, 4))
    for (a, b), n in (((0, 1), n12), ((2, 3), n34)):
        if n == 0:
            continue
        theta = 2.0 * np.pi * n / (dims[a] * dims[b])
        phase[:, b] += theta * c[:, a]
        edge = c[:, a] == dims[a] - 1
        phase[edge, a] += -theta * dims[a] * c[edge, b]
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = np.exp(1j * phase)
    U[:, :, 1, 1] = np.exp(-1j * phase)
    U[:, :, 2, 2] = 1.0
    return U


def haar_su3(n: int, seed: int) -> np.ndarray:
    """n Haar-random SU(3) matrices (QR of a complex Gaussian, phase-fixed, det -> 1)."""
    rng = np.random.default_rng(seed)
    Z = _gaussian_complex(rng, (n, 3, 3))
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(Q)
    return Q / (det ** (1.0 / 3.0))[..., None, None]


def rough_block(dims, eps: float, seed: int, block: int) -> np.ndarray:
    """Near-identity links (eps, seed) with the links of the sites whose four coordinates are
    all < block replaced by Haar-random SU(3) (seed + 100): a smooth field with one rough
    spot, which pulls a few eigenvalues of H_W below the rest of its spectrum."""
    U = near_identity_su3(dims, eps, seed)
    V = volume(dims)
    H = haar_su3(4 * V, seed + 100).reshape(V, 4, 3, 3)
    idx = np.arange(V)
    inside = np.ones(V, dtype=bool)
    for n in dims:
        inside &= (idx % n) < block
        idx = idx // n
    U[inside] = H[inside]
    return U


def left_multiply(N: np.ndarray, U: np.ndarray) -> np.ndarray:
    """U_mu(x) <- N_mu(x) U_mu(x) (noise applied on the left)."""
    return N @ U


def gauge_transform(U: np.ndarray, dims, g: np.ndarray) -> np.ndarray:
    """U_mu(x) <- g(x) U_mu(x) g(x + mu)^dag for g of shape (V, 3, 3)."""
    out = np.empty_like(U)
    for mu in range(4):
        gf = g[forward_index(dims, mu)]
        out[:, mu] = g @ U[:, mu] @ np.conj(np.swapaxes(gf, -1, -2))
    return out


def random_spinors(dims, n: int, seed: int) -> np.ndarray:
    """n Gaussian spinor fields, shape (n, V, 4, 3) complex128."""
    rng = np.random.default_rng(seed)
    return _gaussian_complex(rng, (n, volume(dims), 4, 3))


# ---------------------------------------------------------------------------
# Named synthetic workloads.  Each entry records the lattice, how the links are
# made and the probing gap r used for it (normal mode, r_min = r).
WORKLOADS = {
    # 4^4, near-identity noise eps=0.3, seed 0; SMP r=2 plus a full point-source trace.
    "noise4": dict(dims=(4, 4, 4, 4), kind="noise", eps=0.3, seed=0, r=2),
    # 4^4 and 8^4 near-identity (eps 0.3) with a Haar-random 2^4 / 3^4 block: isolated low modes
    "rough4": dict(dims=(4, 4, 4, 4), kind="rough", eps=0.3, seed=50, block=2, r=2),
    "rough8": dict(dims=(8, 8, 8, 8), kind="rough", eps=0.3, seed=60, block=3, r=(2, 4)),
    # 12^4 (the smallest lattice of Tables 1 and 2), noise eps=0.3, seed 12, Haar gauge seed 13
    "noise12": dict(dims=(12, 12, 12, 12), kind="noise", eps=0.3, seed=12, gauge_seed=13, r=(2, 3, 4, 6)),
    # 8^4, near-identity noise eps=0.3, seed 10 (scheme scans; Haar gauge transform seed 11 on request)
    "noise8": dict(dims=(8, 8, 8, 8), kind="noise", eps=0.3, seed=10, r=(2, 4)),
    # 8^4, U(1) flux (1,1) (Q = 2), noise eps=0.1 seed 1, Haar gauge transform seed 2;
    # SMP r in {2, 4}; point sources on 64 sites drawn with seed 3.
    "flux8": dict(dims=(8, 8, 8, 8), kind="flux", flux=(1, 1), eps=0.1, seed=1, gauge_seed=2,
                  subset_seed=3, subset_n=64, r=(2, 4)),
    # 16^3 x 32, near-identity noise eps=0.2, seed 4; SMP r=4 (3072 sources).
    "noise16x32": dict(dims=(16, 16, 16, 32), kind="noise", eps=0.2, seed=4, r=4),
    # 24^3 x 48, flux (1,1) with noise eps=0.15 seed 5; SMP r=6 (15552 sources).
    "flux24x48": dict(dims=(24, 24, 24, 48), kind="flux", flux=(1, 1), eps=0.15, seed=5, r=6),
    # uneven mix: 16^4 (eps 0.1, seed 6, r 4), 24^4 (eps 0.2, seed 7, r 6), 32^3x64 (eps 0.3, seed 8, r 8)
    "noise16": dict(dims=(16, 16, 16, 16), kind="noise", eps=0.1, seed=6, r=4),
    "noise24": dict(dims=(24, 24, 24, 24), kind="noise", eps=0.2, seed=7, r=6),
    "noise32x64": dict(dims=(32, 32, 32, 64), kind="noise", eps=0.3, seed=8, r=8),
}


def workload(name: str, gauge=True, gauge_seed=None) -> np.ndarray:
    """Build the gauge field of a named workload (deterministic).  gauge=False leaves out the
    workload's random gauge transform; gauge_seed applies a Haar transform with that seed
    (in place of the workload's own, if it has one)."""
    w = WORKLOADS[name]
    dims = w["dims"]
    if w["kind"] == "noise":
        U = near_identity_su3(dims, w["eps"], w["seed"])
    elif w["kind"] == "rough":
        U = rough_block(dims, w["eps"], w["seed"], w["block"])
    else:
        U = u1_flux(dims, *w["flux"])
        U = left_multiply(near_identity_su3(dims, w["eps"], w["seed"]), U)
    seed = gauge_seed if gauge_seed is not None else w.get("gauge_seed")
    if gauge and seed is not None:
        U = gauge_transform(U, dims, haar_su3(volume(dims), seed))
    return U


def subset_sites(name: str) -> np.ndarray:
    """Sorted random site subset of a workload (uniform, without replacement)."""
    w = WORKLOADS[name]
    rng = np.random.default_rng(w["subset_seed"])
    return np.sort(rng.choice(volume(w["dims"]), size=w["subset_n"], replace=False))
