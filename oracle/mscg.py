"""Multi-shift conjugate gradient for (D_W^dag D_W + q_i) x_i = b (section 2.1, Eqs. 6-8).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper solves each shifted system M_i v_i = b "with CG".  All 14 systems share
one Krylov space, so they are solved together (Jegerlehner, hep-lat/9612014;
Frommer, Computing 70 (2003)).  Base matrix A = H^2 + s with s = min_i q_i, relative
shifts d_i = q_i - s >= 0.  Textbook CG on A:
    alpha_k = |r_k|^2 / <p_k, A p_k>,  r_{k+1} = r_k - alpha_k A p_k,
    beta_k = |r_{k+1}|^2 / |r_k|^2,    p_{k+1} = r_{k+1} + beta_k p_k,
and the shifted residuals stay collinear, r^i_k = zeta^i_k r_k, with
    zeta^i_{k+1} = zeta^i_k zeta^i_{k-1} alpha_{k-1} /
                   (alpha_k beta_{k-1} (zeta^i_{k-1} - zeta^i_k)
                    + zeta^i_{k-1} alpha_{k-1} (1 + d_i alpha_k)),
    alpha^i_k = alpha_k zeta^i_{k+1} / zeta^i_k,     x^i_{k+1} = x^i_k + alpha^i_k p^i_k,
    beta^i_k = beta_k (zeta^i_{k+1} / zeta^i_k)^2,   p^i_{k+1} = zeta^i_{k+1} r_{k+1} + beta^i_k p^i_k,
starting from x = 0, r = p = p^i = b, zeta_{-1} = zeta_0 = 1, alpha_{-1} = 1, beta_{-1} = 0.

Stopping rule (the paper gives none; reading): shift i is frozen after the first
iteration with zeta^i_{k+1} |r_{k+1}| <= tol |b|; the solve ends when every shift is
frozen, and raises after max_iter iterations.
"""
import numpy as np


class NotConverged(RuntimeError):
    pass


def multishift_cg(apply_a, b, deltas, tol, max_iter):
    """Solve (A + d_i) x_i = b for every d_i >= 0 at once.

    apply_a(v) applies the base matrix A.  Returns (x, iters) with x[i] the solution
    of shift i and iters[i] the iteration after which it was frozen.
    """
    deltas = np.asarray(deltas, dtype=np.float64)
    n = len(deltas)
    x = [np.zeros_like(b) for _ in range(n)]
    p_s = [b.copy() for _ in range(n)]
    r = b.copy()
    p = b.copy()
    zeta = np.ones(n)
    zeta_prev = np.ones(n)
    alpha_prev, beta_prev = 1.0, 0.0
    rr = np.vdot(r, r).real
    bnorm = np.sqrt(rr)
    active = np.ones(n, dtype=bool)
    iters = np.zeros(n, dtype=np.int64)
    if bnorm == 0.0:
        return x, iters
    for k in range(max_iter):
        ap = apply_a(p)
        pap = np.vdot(p, ap).real
        if not (pap > 0.0):
            raise FloatingPointError("CG breakdown: <p, A p> <= 0")
        alpha = rr / pap
        zeta_new = zeta.copy()
        for i in np.nonzero(active)[0]:
            zeta_new[i] = (zeta[i] * zeta_prev[i] * alpha_prev /
                           (alpha * beta_prev * (zeta_prev[i] - zeta[i]) +
                            zeta_prev[i] * alpha_prev * (1.0 + deltas[i] * alpha)))
            x[i] = x[i] + (alpha * zeta_new[i] / zeta[i]) * p_s[i]
        r = r - alpha * ap
        rr_new = np.vdot(r, r).real
        beta = rr_new / rr
        for i in np.nonzero(active)[0]:
            if zeta_new[i] * np.sqrt(rr_new) <= tol * bnorm:
                active[i] = False
                iters[i] = k + 1
            else:
                p_s[i] = zeta_new[i] * r + (beta * (zeta_new[i] / zeta[i]) ** 2) * p_s[i]
        p = r + beta * p
        zeta_prev, zeta = zeta, zeta_new
        alpha_prev, beta_prev, rr = alpha, beta, rr_new
        if not active.any():
            return x, iters
    raise NotConverged(f"multi-shift CG: {int(active.sum())} shifts not converged after {max_iter} iterations")


def cg(apply_m, b, tol, max_iter):
    """Plain CG for a single hermitian positive matrix (used to check the shifted solver)."""
    x = np.zeros_like(b)
    r = b.copy()
    p = b.copy()
    rr = np.vdot(r, r).real
    bnorm = np.sqrt(rr)
    for k in range(max_iter):
        mp = apply_m(p)
        alpha = rr / np.vdot(p, mp).real
        x = x + alpha * p
        r = r - alpha * mp
        rr_new = np.vdot(r, r).real
        if np.sqrt(rr_new) <= tol * bnorm:
            return x, k + 1
        p = r + (rr_new / rr) * p
        rr = rr_new
    raise NotConverged("CG not converged")
