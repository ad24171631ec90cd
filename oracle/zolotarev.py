"""Zolotarev rational approximation of the sign function (section 1, Eq. 4).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Eq. 4 writes eps(H) = H (c_0 + sum_i c_i / (H^2 + q_i)) and the paper uses a
"14th-order" Zolotarev expansion, read here as n = 14 poles q_i with a constant
term c_0 (a type (2n+1, 2n) rational function of H).

Zolotarev's optimal approximation of sign(x) on [-1, -k] u [k, 1]:
    x R(x^2),  R(x^2) = d prod_{l=1}^{n} (x^2 + a_{2l}) / (x^2 + a_{2l-1}),
    a_l = k^2 sn^2(l K'/(2n+1); k') / cn^2(l K'/(2n+1); k'),  l = 1..2n,
with k' = sqrt(1 - k^2), K' = K(k') the complete elliptic integral of the first
kind; sn, cn are Jacobi elliptic functions of modulus k'.  The constant d is
fixed by symmetric equioscillation: with m, M the minimum and maximum of
x R(x^2)/d on [k, 1] (attained at the alternation points below), d = 2/(m + M)
and the maximal error is delta = (M - m)/(M + m).

Partial fractions: R(x^2) = b_0 + sum_l b_l/(x^2 + a_{2l-1}) with b_0 = d and
    b_l = d prod_j (a_{2j} - a_{2l-1}) / prod_{j != l} (a_{2j-1} - a_{2l-1}).
For H with |H| in [lam_min, lam_max], x = H/lam_max and k = lam_min/lam_max, so
    c_0 = b_0/lam_max,  c_i = b_i lam_max,  q_i = a_{2i-1} lam_max^2.
"""
import numpy as np
from scipy.special import ellipj, ellipk


def _a_coefficients(n, k):
    kp2 = 1.0 - k * k                       # parameter m = k'^2 as scipy expects
    Kp = ellipk(kp2)
    u = np.arange(1, 2 * n + 1) * Kp / (2 * n + 1)
    sn, cn, _, _ = ellipj(u, kp2)
    return k * k * sn * sn / (cn * cn)


def _unnormalised(x, a):
    x = np.asarray(x, dtype=np.float64)
    x2 = x * x
    r = x.copy()
    for l in range(len(a) // 2):
        r = r * (x2 + a[2 * l + 1]) / (x2 + a[2 * l])
    return r


def alternation_points(n, k):
    """The 2n+2 points x_l = k / dn(l K'/(2n+1); k'), l = 0..2n+1, running from k to 1,
    where the error of the optimal approximation alternates in sign (Zolotarev;
    Akhiezer, Elements of the theory of elliptic functions)."""
    kp2 = 1.0 - k * k
    u = np.arange(0, 2 * n + 2) * ellipk(kp2) / (2 * n + 1)
    _, _, dn, _ = ellipj(u, kp2)
    return k / dn


def zolotarev(n, lam_min, lam_max):
    """Coefficients (c0, c[n], q[n], delta) of eps(H) ~ H (c0 + sum c_i/(H^2 + q_i)).

    Follows Eq. 4 with the Zolotarev construction in the module docstring.
    Shifts are returned in increasing order.
    """
    if not (0.0 < lam_min < lam_max):
        raise ValueError("need 0 < lam_min < lam_max")
    if n < 1:
        raise ValueError("need at least one pole")
    k = lam_min / lam_max
    a = _a_coefficients(n, k)
    ext = _unnormalised(alternation_points(n, k), a)
    m, M = ext.min(), ext.max()
    d = 2.0 / (m + M)
    delta = (M - m) / (M + m)
    num = a[1::2]            # a_{2l},   l = 1..n
    den = a[0::2]            # a_{2l-1}, l = 1..n
    b = np.empty(n)
    for l in range(n):
        others = np.delete(den, l)
        b[l] = d * np.prod(num - den[l]) / np.prod(others - den[l])
    c0 = d / lam_max
    c = b * lam_max
    q = den * lam_max ** 2
    order = np.argsort(q)
    return c0, c[order], q[order], delta


def eps_scalar(x, c0, c, q):
    """The rational function x (c0 + sum c_i/(x^2 + q_i)) on real x (for checks)."""
    x = np.asarray(x, dtype=np.float64)
    s = np.full_like(x, c0)
    for ci, qi in zip(c, q):
        s = s + ci / (x * x + qi)
    return x * s


def eps_product_form(x, n, lam_min, lam_max):
    """Same function from the product form x R(x^2) (used to check the partial fractions)."""
    k = lam_min / lam_max
    a = _a_coefficients(n, k)
    ext = _unnormalised(alternation_points(n, k), a)
    d = 2.0 / (ext.min() + ext.max())
    return d * _unnormalised(np.asarray(x, dtype=np.float64) / lam_max, a)
