"""Pins of the oracle's locality diagnostic (section 2.2, Eq. 12, Fig. 1)."""
import numpy as np

import smpq_inputs as si
from oracle.charge import eps_dense, h_spectrum
from oracle.dirac import GAMMA5
from oracle.lattice import Lattice
from oracle.lanczos import bounds
from oracle.locality import block_mean_abs, block_mean_abs_dense, distances
from oracle.zolotarev import zolotarev

KAPPA = 0.21


def test_block_means_equal_dense_overlap_on_2x2x2x4():
    """Solver columns against the blocks of the dense D_ov = 1 + gamma5 eps (Eq. 3), eps from
    eigh; also the Ginsparg-Wilson consequence D^dag D = D + D^dag on the dense matrix."""
    dims = (2, 2, 2, 4)
    lat = Lattice(dims)
    U = si.near_identity_su3(dims, 0.4, 31)
    w, v = h_spectrum(U, lat, KAPPA)
    g5 = np.kron(np.eye(lat.volume), np.kron(GAMMA5, np.eye(3)))
    dov = np.eye(12 * lat.volume) + g5 @ eps_dense(w, v)
    assert np.abs(dov.conj().T @ dov - dov - dov.conj().T).max() < 1e-12
    lo, hi = bounds(U, lat, KAPPA, 120, seed=0)
    zo = zolotarev(14, lo, hi)
    for site in (0, 13):
        m = block_mean_abs(U, lat, KAPPA, zo[:3], site, 1e-13, 5000)
        assert np.abs(m - block_mean_abs_dense(dov, lat.volume, site)).max() < 1e-10


def test_distances_min_image():
    lat = Lattice((4, 6, 4, 8))
    eu, tx = distances(lat, 0)
    s = lat.index((3, 4, 2, 5))
    # minimum image: (1, 2, 2, 3)
    assert tx[s] == 8 and abs(eu[s] - np.sqrt(18)) < 1e-15
    assert eu[0] == 0 and tx.max() == 2 + 3 + 2 + 4
