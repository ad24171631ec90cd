"""Locality of the overlap operator (section 2.2, Eq. 12 and Fig. 1).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

For a source site y, the twelve columns D_ov e_{y,beta,b} (Eq. 3) give the blocks
D_ov(x, . ; y, .) for every x; the diagnostic of Fig. 1 is the mean absolute value of the
144 entries of each block, averaged over the sites at one distance |x - y| (Euclidean, or
taxi-driver, minimum image on the torus), whose logarithm falls linearly with the distance,
slope -gamma of Eq. 12.
"""
import numpy as np

from .charge import dov_apply


def block_mean_abs(U, lat, kappa, zolo, site, tol, max_iter):
    """m(x) = (1/144) sum_{alpha,a,beta,b} |D_ov(x alpha a; site beta b)| for every x."""
    V = lat.volume
    m = np.zeros(V)
    for beta in range(4):
        for b in range(3):
            e = np.zeros((V, 4, 3), dtype=np.complex128)
            e[site, beta, b] = 1.0
            col = dov_apply(U, lat, kappa, zolo, e, tol, max_iter)
            m += np.abs(col).reshape(V, 12).sum(axis=1)
    return m / 144.0


def block_mean_abs_dense(dov, V, site):
    """The same from a dense D_ov (12V x 12V, row/column index 12 x + 3 spin + colour)."""
    blocks = np.abs(dov.reshape(V, 12, V, 12)[:, :, site, :])
    return blocks.sum(axis=(1, 2)) / 144.0


def distances(lat, site):
    """(Euclidean, taxi-driver) minimum-image distances of every site from `site`."""
    d = np.abs(lat.coords - lat.coords[site])
    d = np.minimum(d, np.asarray(lat.dims) - d)
    return np.sqrt((d * d).sum(axis=1)), d.sum(axis=1)
