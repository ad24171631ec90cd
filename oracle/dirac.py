"""Wilson kernel D_W and the hermitian H_W = gamma5 D_W (section 1, Eqs. 3-4).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper names only gamma5, the hopping parameter kappa = 0.21 and the Wilson
kernel.  The reading fixed here (and used everywhere):

  Euclidean hermitian gamma matrices in the chiral basis,
      gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]  (k = 1, 2, 3 -> x, y, z)
      gamma_4 = [[0, 1], [1, 0]]                   (t)
      gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 = diag(1, 1, -1, -1)
  D_W psi(x) = psi(x) - kappa sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
                                     + (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu) ]
  periodic boundary conditions in all four directions.

Spinors have shape (V, 4, 3) (site, spin, colour); links (V, 4, 3, 3)
(site, mu, row, col).
"""
import numpy as np
import scipy.sparse as sp

SIGMA = np.array([[[0, 1], [1, 0]],
                  [[0, -1j], [1j, 0]],
                  [[1, 0], [0, -1]]], dtype=np.complex128)


def gamma_matrices():
    """(gamma_1..gamma_4, gamma_5) in the chiral basis described above."""
    z = np.zeros((2, 2), dtype=np.complex128)
    one = np.eye(2, dtype=np.complex128)
    g = [np.block([[z, -1j * SIGMA[k]], [1j * SIGMA[k], z]]) for k in range(3)]
    g.append(np.block([[z, one], [one, z]]))
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    return np.array(g), g5


GAMMA, GAMMA5 = gamma_matrices()
ID4 = np.eye(4, dtype=np.complex128)


def apply_gamma5(psi):
    """gamma5 acting on the spin index of psi (..., V, 4, 3)."""
    return np.einsum("st,...xta->...xsa", GAMMA5, psi)


def _hop_terms(U, lat, psi, dagger):
    """sum_mu [P-_mu U_mu(x) psi(x+mu) + P+_mu U_mu(x-mu)^dag psi(x-mu)]; P-+ = 1 -+ gamma_mu.

    The adjoint D_W^dag swaps the two projectors (the links stay in place).
    """
    out = np.zeros_like(psi)
    for mu in range(4):
        pm, pp = ID4 - GAMMA[mu], ID4 + GAMMA[mu]
        if dagger:
            pm, pp = pp, pm
        fwd = np.einsum("xab,xsb->xsa", U[:, mu], psi[lat.fwd[mu]])
        out += np.einsum("st,xta->xsa", pm, fwd)
        ub = np.conj(np.swapaxes(U[lat.bwd[mu], mu], -1, -2))
        bwd = np.einsum("xab,xsb->xsa", ub, psi[lat.bwd[mu]])
        out += np.einsum("st,xta->xsa", pp, bwd)
    return out


def apply_dw(U, lat, kappa, psi, dagger=False):
    """D_W psi, or D_W^dag psi when dagger is set (section 1, Eq. 3)."""
    return psi - kappa * _hop_terms(U, lat, psi, dagger)


def apply_h(U, lat, kappa, psi):
    """H_W psi = gamma5 D_W psi (the argument of the sign function in Eq. 3)."""
    return apply_gamma5(apply_dw(U, lat, kappa, psi))


def apply_h2(U, lat, kappa, psi):
    """H_W^2 psi = D_W^dag D_W psi (the operator of Eq. 4's denominators)."""
    return apply_dw(U, lat, kappa, apply_dw(U, lat, kappa, psi), dagger=True)


def dw_sparse(U, lat, kappa):
    """D_W as a (12V x 12V) sparse matrix, assembled site by site from its definition.

    Row/column index = 12*site + 3*spin + colour.  Used for dense checks on tiny
    lattices; independent of the matrix-free apply_dw above.
    """
    V = lat.volume
    rows, cols, vals = [], [], []

    def add_block(x, y, block):  # block is 12x12 acting on psi(y), landing at x
        r, c = np.nonzero(block)
        rows.extend(12 * x + r)
        cols.extend(12 * y + c)
        vals.extend(block[r, c])

    for x in range(V):
        add_block(x, x, np.eye(12, dtype=np.complex128))
        for mu in range(4):
            xf = lat.fwd[mu][x]
            add_block(x, xf, -kappa * np.kron(ID4 - GAMMA[mu], U[x, mu]))
            xb = lat.bwd[mu][x]
            add_block(x, xb, -kappa * np.kron(ID4 + GAMMA[mu], np.conj(U[xb, mu].T)))
    return sp.csr_matrix((vals, (rows, cols)), shape=(12 * V, 12 * V))


def h_dense(U, lat, kappa):
    """Dense H_W = gamma5 D_W, (12V x 12V)."""
    g5 = np.kron(np.eye(lat.volume), np.kron(GAMMA5, np.eye(3)))
    return g5 @ dw_sparse(U, lat, kappa).toarray()
