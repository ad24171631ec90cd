"""Topological charge density q(x) = 1/2 tr(gamma5 D_ov)(x, x) (Eqs. 2, 3, 5, 16).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

  D_ov = 1 + gamma5 eps(H_W)                                    (Eq. 3)
  eps(H) b ~ H (c_0 b + sum_i c_i x_i),  (H^2 + q_i) x_i = b     (Eq. 4, Eqs. 6-8)
  point source e_{x,alpha,a}:   q(x) = 1/2 sum_{alpha,a} <e|gamma5 D_ov|e>   (Eq. 5)
  probing source phi = sum_{y in S} e_{y,alpha,a}, for x in S:
      q(x) += 1/2 [gamma5 D_ov phi](x, alpha, a)                              (Eq. 16)

q is returned complex: the real part is q(x); the imaginary part, which comes
only from the off-diagonal terms of a probing source, is kept as a diagnostic
(its sum over one class is zero).  Q = sum_x Re q(x).
"""
import numpy as np

from .dirac import GAMMA5, apply_gamma5, apply_h, apply_h2, h_dense
from .mscg import multishift_cg


def eps_apply(U, lat, kappa, zolo, b, tol, max_iter):
    """eps_Z(H_W) b through the multi-shift CG (Eq. 4); returns (eps b, per-shift iterations)."""
    c0, c, q = zolo[:3]
    s = float(np.min(q))
    x, iters = multishift_cg(lambda v: apply_h2(U, lat, kappa, v) + s * v,
                             b, np.asarray(q) - s, tol, max_iter)
    y = c0 * b
    for ci, xi in zip(c, x):
        y = y + ci * xi
    return apply_h(U, lat, kappa, y), iters


def dov_apply(U, lat, kappa, zolo, b, tol, max_iter):
    """D_ov b = b + gamma5 eps_Z(H_W) b (Eq. 3)."""
    eb, _ = eps_apply(U, lat, kappa, zolo, b, tol, max_iter)
    return b + apply_gamma5(eb)


def source_contribution(U, lat, kappa, zolo, colour, c, alpha, a, tol, max_iter):
    """One probing source phi = sum_{y in S_c} e_{y,alpha,a} (Eq. 15): returns the sites S_c,
    the values 1/2 [gamma5 D_ov phi](x, alpha, a) for x in S_c (Eq. 16) and the CG iterations."""
    V = lat.volume
    S = np.nonzero(colour == c)[0]
    b = np.zeros((V, 4, 3), dtype=np.complex128)
    b[S, alpha, a] = 1.0
    eb, iters = eps_apply(U, lat, kappa, zolo, b, tol, max_iter)
    out = apply_gamma5(b) + eb                           # gamma5 D_ov phi
    return S, 0.5 * out[S, alpha, a], iters


def qx_probing(U, lat, kappa, zolo, colour, classes, tol, max_iter, stats=None):
    """q(x) on the sites of the given classes, one source per (class, alpha, a) (Eq. 16).

    With the point colouring this is the exact point-source trace of Eq. 5.
    Sites outside the given classes are left at zero.
    """
    q = np.zeros(lat.volume, dtype=np.complex128)
    for c in classes:
        for alpha in range(4):
            for a in range(3):
                S, val, iters = source_contribution(U, lat, kappa, zolo, colour, c, alpha, a, tol, max_iter)
                q[S] += val
                if stats is not None:
                    stats.append(iters)
    return q


# ---------------------------------------------------------------- dense checks
def h_spectrum(U, lat, kappa):
    """Eigenvalues and eigenvectors of the dense H_W (tiny lattices only)."""
    return np.linalg.eigh(h_dense(U, lat, kappa))


def eps_dense(w, v, fn=np.sign):
    """eps = V f(Lambda) V^dag for a function f of the eigenvalues of H_W."""
    return (v * fn(w)) @ np.conj(v.T)


def qx_from_eps(eps, V):
    """Exact q(x) = 1/2 tr_{s,c} eps(x, x) (gamma5 is traceless in spin)."""
    return 0.5 * np.real(np.diagonal(eps)).reshape(V, 12).sum(axis=1)


def qx_smp_from_eps(eps, colour):
    """Eq. 16 summed from a dense eps: 1/2 sum_{alpha,a} sum_{y in S(x)} [gamma5 D_ov](x a; y a)."""
    V = len(colour)
    g5d = np.kron(np.eye(V), np.kron(GAMMA5, np.eye(3)))
    m = g5d + eps                                     # gamma5 D_ov = gamma5 + eps
    q = np.zeros(V, dtype=np.complex128)
    for x in range(V):
        S = np.nonzero(colour == colour[x])[0]
        for j in range(12):
            q[x] += 0.5 * m[12 * x + j, 12 * S + j].sum()
    return q


def charge_from_spectrum(w):
    """Q = 1/2 Tr eps(H_W) = (N_+ - N_-)/2 (index theorem, Eq. 2)."""
    return 0.5 * (np.sum(w > 0) - np.sum(w < 0))
