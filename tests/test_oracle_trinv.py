"""Pins of the oracle's probing estimate of Tr D_W^-1 (Conclusion; probing as in Eqs. 15-16)."""
import numpy as np
import pytest

import smpq_inputs as si
from oracle.lattice import Lattice
from oracle.probing import colouring, point_colouring
from oracle.trinv import trinv_dense, trinv_free, trinv_probing, trinv_smp_dense

KAPPA = 0.21


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (4, 2, 2, 6)])
def test_free_field_matches_momentum_sum(dims):
    """U = 1: every site carries the closed-form momentum sum; the trace is real."""
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.0, 0)
    t = trinv_dense(U, lat, KAPPA)
    assert np.abs(t - trinv_free(dims, KAPPA)).max() < 1e-12
    col, n = point_colouring(lat)
    tp = trinv_probing(U, lat, KAPPA, col, range(n))
    assert np.abs(tp - t).max() < 1e-12


def test_free_field_closed_form_hand_value():
    """2^4 free field: the momenta are 0 or pi in each direction, so sin p = 0 and
    D_W(p) = 1 - 2 kappa (4 - 2 k) with k the number of pi components; the mean over the
    16 momenta of 12 / (1 - 2 kappa (4 - 2k)) weighted by C(4, k)."""
    from math import comb
    want = 12.0 * sum(comb(4, k) / (1 - 2 * KAPPA * (4 - 2 * k)) for k in range(5)) / 16
    assert abs(trinv_free((2, 2, 2, 2), KAPPA) - want) < 1e-13


def test_point_sources_equal_dense_diagonal_and_real():
    """Interacting 4^4 field: point sources give the dense diagonal trace, which is real
    (gamma5-hermiticity: (D^-1)^dag = gamma5 D^-1 gamma5)."""
    dims = (4, 4, 4, 4)
    lat = Lattice(dims)
    U = si.workload("noise4")
    t = trinv_dense(U, lat, KAPPA)
    assert np.abs(t.imag).max() < 1e-12
    col, n = point_colouring(lat)
    tp = trinv_probing(U, lat, KAPPA, col, range(0, n, 7))
    m = np.zeros(lat.volume, bool)
    m[::7] = True
    assert np.abs(tp[m] - t[m]).max() < 1e-12 and np.all(tp[~m] == 0)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_probing_equals_dense_class_sums(mode):
    """The probing estimate is the sum over the class of the component-diagonal entries of
    the dense inverse; the CG path agrees with the factorised one."""
    dims = (4, 4, 4, 4)
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.4, 21)
    col, n = colouring(lat, (2, 2, 2, 2), mode)
    ref = trinv_smp_dense(U, lat, KAPPA, col)
    t = trinv_probing(U, lat, KAPPA, col, range(n))
    assert np.abs(t - ref).max() < 1e-12
    t2 = trinv_probing(U, lat, KAPPA, col, [0, n - 1], method="cg")
    m = np.isin(col, [0, n - 1])
    assert np.abs(t2[m] - ref[m]).max() < 1e-10


def test_gauge_invariance_of_exact_trace():
    dims = (4, 4, 2, 2)
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.5, 22)
    Ug = si.gauge_transform(U, dims, si.haar_su3(lat.volume, 23))
    assert np.abs(trinv_dense(U, lat, KAPPA) - trinv_dense(Ug, lat, KAPPA)).max() < 1e-12
