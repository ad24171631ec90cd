"""Host logic of the locality diagnostic (shells and decay fit); no GPU needed."""
import numpy as np

from oracle.lattice import Lattice
from oracle.locality import distances
from paper_1901_02211_amd.locality import fit_decay, shells, site_distances


def test_site_distances_match_oracle_definition():
    dims = (4, 6, 4, 8)
    lat = Lattice(dims)
    for site in (0, 77, lat.volume - 1):
        eu, tx = site_distances(dims, site)
        oe, ot = distances(lat, site)
        assert np.array_equal(tx, ot) and np.abs(eu - oe).max() < 1e-14


def test_shells_and_fit_recover_an_exponential():
    dims = (8, 8, 8, 8)
    eu, tx = site_distances(dims, 5)
    m = 3.0 * np.exp(-1.1 * eu)
    d, mean, cnt = shells(m, eu)
    assert cnt.sum() == 8 ** 4 and d[0] == 0 and cnt[0] == 1 and cnt[1] == 8
    slope, icpt = fit_decay(d, mean)
    assert abs(slope + 1.1) < 1e-9 and abs(icpt - np.log(3.0)) < 1e-9
    d2, mean2, _ = shells(np.exp(-0.5 * tx), tx)
    assert abs(fit_decay(d2, mean2)[0] + 0.5) < 1e-9
