"""Low-mode deflation of the sign function (the exact sign on the lowest eigenmodes and the
Zolotarev function on the rest: the usual companion of the Zolotarev construction the paper
takes for Eq. 4, needed when |H_W| has a few eigenvalues far below the others).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

For eigenpairs (u_i, theta_i) at the bottom of the spectrum of H^2 = D_W^dag D_W,
eps(H) = H (H^2)^(-1/2) gives eps(H) u_i = H u_i / sqrt(theta_i) exactly, whether or not u_i is
an eigenvector of H itself.  With P b = b - sum_i u_i <u_i, b> the projection on the rest of
the spectrum (H commutes with H^2, so H maps it into itself):
    eps b = sum_i (H u_i / sqrt(theta_i)) <u_i, b> + eps_Z(H) P b,
where the Zolotarev interval need only cover the eigenvalues left in P.
"""
import numpy as np

from .charge import eps_apply
from .dirac import apply_gamma5, apply_h, h_dense


def low_modes(U, lat, kappa, k):
    """The k smallest eigenvalues theta_i of H^2 and orthonormal eigenvectors u_i (k, V, 4, 3),
    from the dense H_W (tiny lattices): theta = lambda^2 for the k smallest |lambda|."""
    w, v = np.linalg.eigh(h_dense(U, lat, kappa))
    order = np.argsort(np.abs(w))[:k]
    u = v[:, order].T.reshape(k, lat.volume, 4, 3)
    return w[order] ** 2, u


def eps_apply_deflated(U, lat, kappa, zolo, theta, u, b, tol, max_iter):
    """eps(H) b with the modes (theta, u) deflated."""
    coef = [np.vdot(ui, b) for ui in u]
    pb = b.copy()
    for ci, ui in zip(coef, u):
        pb = pb - ci * ui
    eb, _ = eps_apply(U, lat, kappa, zolo, pb, tol, max_iter)
    for ci, ui, th in zip(coef, u, theta):
        eb = eb + (ci / np.sqrt(th)) * apply_h(U, lat, kappa, ui)
    return eb


def qx_probing_deflated(U, lat, kappa, zolo, theta, u, colour, classes, tol, max_iter):
    """q(x) of Eq. 16 on the listed classes with the deflated sign function."""
    q = np.zeros(lat.volume, dtype=np.complex128)
    for c in classes:
        S = np.nonzero(colour == c)[0]
        for alpha in range(4):
            for a in range(3):
                b = np.zeros((lat.volume, 4, 3), dtype=np.complex128)
                b[S, alpha, a] = 1.0
                out = apply_gamma5(b) + eps_apply_deflated(U, lat, kappa, zolo, theta, u, b, tol, max_iter)
                q[S] += 0.5 * out[S, alpha, a]
    return q


def eps_dense_deflated(w, v, k, eps_z):
    """Dense reference: V diag(f) V^dag with f = sign on the k smallest |lambda| of H_W and the
    scalar Zolotarev function eps_z elsewhere."""
    f = eps_z(w)
    low = np.argsort(np.abs(w))[:k]
    f[low] = np.sign(w[low])
    return (v * f) @ np.conj(v.T)



