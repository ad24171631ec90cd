"""Pins of the oracle's Zolotarev coefficients (section 1, Eq. 4).

The optimal approximation is characterised by Chebyshev alternation: the error
sign(x) - eps(x) on [k, 1] attains its maximum modulus at 2n+2 points with
alternating signs.  These tests find the extrema by a dense grid search (not by
the closed-form alternation points the oracle uses) and check the count, the
equal moduli and the alternation, plus the error bound, positivity, scaling and
the partial-fraction form.
"""
import numpy as np
import pytest

from oracle.zolotarev import alternation_points, eps_product_form, eps_scalar, zolotarev


def _grid_extrema(err, x):
    idx = [0]
    d = np.diff(err)
    idx += list(np.nonzero(d[:-1] * d[1:] < 0)[0] + 1)
    idx.append(len(x) - 1)
    return np.array(idx)


@pytest.mark.parametrize("n,k", [(3, 0.1), (4, 0.05), (6, 0.01), (5, 0.02), (8, 0.005)])
def test_equioscillation(n, k):
    c0, c, q, delta = zolotarev(n, k, 1.0)
    x = np.exp(np.linspace(np.log(k), 0.0, 400001))
    err = 1.0 - eps_scalar(x, c0, c, q)
    idx = _grid_extrema(err, x)
    assert len(idx) == 2 * n + 2
    vals = err[idx]
    assert np.all(np.sign(vals[1:]) == -np.sign(vals[:-1]))
    assert np.allclose(np.abs(vals), delta, rtol=1e-5)
    assert np.abs(err).max() <= delta * (1 + 1e-6)
    # the grid extrema sit at the closed-form alternation points
    assert np.allclose(x[idx], alternation_points(n, k), rtol=1e-3)


@pytest.mark.parametrize("k", [0.01, 0.03])
def test_fourteen_poles_error_bound(k):
    c0, c, q, delta = zolotarev(14, k, 1.0)
    x = np.exp(np.linspace(np.log(k), 0.0, 200001))
    err = np.abs(1.0 - eps_scalar(x, c0, c, q))
    assert err.max() <= delta * (1 + 1e-3) + 1e-15
    assert delta < 1e-9
    # error decreases with the number of poles
    assert zolotarev(10, k, 1.0)[3] > 10 * delta


def test_scaling_and_positivity():
    lo, hi = 0.15, 2.7
    c0, c, q, delta = zolotarev(14, lo, hi)
    assert c0 > 0 and np.all(c > 0) and np.all(q > 0)
    assert np.all(np.diff(q) > 0)
    c0u, cu, qu, du = zolotarev(14, lo / hi, 1.0)
    assert abs(delta - du) < 1e-15
    x = np.linspace(lo, hi, 1001)
    assert np.abs(eps_scalar(x, c0, c, q) - eps_scalar(x / hi, c0u, cu, qu)).max() < 1e-13
    # odd function
    assert np.abs(eps_scalar(-x, c0, c, q) + eps_scalar(x, c0, c, q)).max() == 0.0


def test_partial_fractions_match_product_form():
    lo, hi = 0.2, 2.5
    for n in (4, 14):
        c0, c, q, _ = zolotarev(n, lo, hi)
        x = np.linspace(0.05, 4.0, 777)
        assert np.abs(eps_scalar(x, c0, c, q) - eps_product_form(x, n, lo, hi)).max() < 1e-12


def test_normalisation_is_optimal():
    """Scaling eps by (1 +- 1e-6) away from the symmetric choice increases the max error."""
    n, k = 4, 0.1
    c0, c, q, delta = zolotarev(n, k, 1.0)
    x = np.exp(np.linspace(np.log(k), 0.0, 100001))
    for s in (1 + 1e-6, 1 - 1e-6):
        assert np.abs(1 - s * eps_scalar(x, c0, c, q)).max() > delta


def test_rejects_bad_interval():
    for lo, hi in ((0.0, 1.0), (-1.0, 1.0), (2.0, 1.0)):
        with pytest.raises(ValueError):
            zolotarev(14, lo, hi)
