"""Probing estimate of the trace of the inverse Wilson kernel (Conclusion: the same probing
applies to Tr D_W^-1, the application the paper proposes; probing vectors as in Eqs. 15-16).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

For a colouring with classes S_c and the probing vectors phi_{c,alpha,a} = sum_{y in S_c}
e_{y,alpha,a}, the estimate of the spin-colour trace of D_W^-1 at x in S_c is
    t(x) = sum_{alpha,a} [D_W^-1 phi_{c,alpha,a}](x, alpha, a)
         = sum_{alpha,a} sum_{y in S_c} D_W^-1(x alpha a; y alpha a),
the diagonal block trace plus the off-diagonal terms inside the class (the analogue of
Eq. 16 without the factor 1/2 and gamma5).  With one site per class (point sources) it is
exact: t(x) = tr_sc D_W^-1(x, x) and Tr D_W^-1 = sum_x t(x).

Each probing vector is solved with D_W z = phi directly, by a sparse LU factorisation of the
matrix assembled from the definition of D_W (dirac.dw_sparse), or by CG on the normal
equations D_W^dag D_W z = D_W^dag phi where the factorisation would be too large.
"""
import numpy as np
import scipy.sparse.linalg as spla

from .dirac import apply_dw, dw_sparse
from .mscg import cg


def dw_solver(U, lat, kappa, method="lu", tol=1e-13, max_iter=20000):
    """A function phi -> D_W^-1 phi on spinors of shape (V, 4, 3)."""
    V = lat.volume
    if method == "lu":
        lu = spla.splu(dw_sparse(U, lat, kappa).tocsc())
        return lambda phi: lu.solve(phi.reshape(12 * V)).reshape(V, 4, 3)

    def solve(phi):
        rhs = apply_dw(U, lat, kappa, phi, dagger=True)
        z, _ = cg(lambda v: apply_dw(U, lat, kappa, apply_dw(U, lat, kappa, v), dagger=True), rhs, tol, max_iter)
        return z
    return solve


def trinv_probing(U, lat, kappa, colour, classes, method="lu"):
    """t(x) (complex) on the sites of the listed classes, zero elsewhere."""
    solve = dw_solver(U, lat, kappa, method)
    t = np.zeros(lat.volume, dtype=np.complex128)
    for c in classes:
        S = np.nonzero(colour == c)[0]
        for alpha in range(4):
            for a in range(3):
                phi = np.zeros((lat.volume, 4, 3), dtype=np.complex128)
                phi[S, alpha, a] = 1.0
                t[S] += solve(phi)[S, alpha, a]
    return t


def trinv_dense(U, lat, kappa):
    """tr_sc D_W^-1(x, x) for every x from the dense inverse (tiny lattices)."""
    inv = np.linalg.inv(dw_sparse(U, lat, kappa).toarray())
    return np.diagonal(inv).reshape(lat.volume, 12).sum(axis=1)


def trinv_smp_dense(U, lat, kappa, colour):
    """The probing estimate from the dense inverse: for x in S_c, sum over y in S_c and the
    twelve spin-colour components of D_W^-1(x j; y j)."""
    V = lat.volume
    inv = np.linalg.inv(dw_sparse(U, lat, kappa).toarray()).reshape(V, 12, V, 12)
    diag = np.einsum("xjyj->xy", inv)                  # sum over the component j
    same = colour[:, None] == colour[None, :]
    return (diag * same).sum(axis=1)


def trinv_free(dims, kappa):
    """Free field (U = 1): D_W(p) = M(p) + i sum_mu gamma_mu s_mu(p) with M = 1 - 2 kappa
    sum cos p_mu and s_mu = 2 kappa sin p_mu, so D_W(p)^-1 = (M - i gamma.s) / (M^2 + s^2)
    and tr_sc D_W^-1(x, x) = (12 / V) sum_p M / (M^2 + s^2), p_mu = 2 pi k / n_mu."""
    ps = np.meshgrid(*[2 * np.pi * np.arange(n) / n for n in dims], indexing="ij")
    M = 1.0 - 2.0 * kappa * sum(np.cos(p) for p in ps)
    s2 = 4.0 * kappa ** 2 * sum(np.sin(p) ** 2 for p in ps)
    return 12.0 * np.mean(M / (M ** 2 + s2))
