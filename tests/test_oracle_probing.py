"""Pins of the oracle's SMP colourings against the paper's printed integers (Tables 1-2, Eq. 19)."""
import numpy as np
import pytest

from conftest import load_table
from oracle.lattice import Lattice
from oracle.probing import (class_sites, colouring, gaps_from_m, n_sources, nearest_count,
                            point_colouring, r_min)


def _scheme(n, m, mode):
    lat = Lattice((n, n, n, n))
    r = gaps_from_m(lat.dims, (m, m, m, m))
    return lat, colouring(lat, r, mode)


@pytest.mark.parametrize("row", load_table("table2_source_counts.txt"))
def test_table2_source_counts(row):
    """N^SMP and N^SMP/N^PT of every scheme in Table 2."""
    n, m, mode, nsmp, denom = row
    lat, (colour, ncls) = _scheme(n, m, mode) if n <= 24 else (None, (None, None))
    if lat is None:                  # 32^4: the class count depends only on r and the mode
        r = n // m
        ncls = {0: r ** 4, 1: 2 * r ** 4, 2: r ** 4 // 2}[mode]
        assert ncls == len(np.unique(colouring(Lattice((2 * r, 2 * r, 2 * r, 2 * r)), (r,) * 4, mode)[0]))
    else:
        assert len(np.unique(colour)) == ncls
    assert n_sources(ncls) == nsmp
    assert 12 * n ** 4 == nsmp * denom


def _small_classes(row):
    n, m, mode = row[:3]
    return n <= 16 and m ** 4 * (2 if mode == 2 else 1) <= 1296


@pytest.mark.parametrize("row", [r for r in load_table("table1_rmin.txt") if _small_classes(r)])
def test_table1_rmin_brute_force(row):
    """r_min of Table 1 (Eq. 18) by brute force over all pairs of every class."""
    n, m, mode, a, b = row
    lat, (colour, ncls) = _scheme(n, m, mode)
    assert abs(r_min(lat, colour, ncls) - a * np.sqrt(b)) < 1e-12


@pytest.mark.parametrize("row", [r for r in load_table("table1_rmin.txt") if not _small_classes(r)])
def test_table1_rmin_large(row):
    """Large classes: distances from one seed site to its class (classes are translates)."""
    n, m, mode, a, b = row
    lat, (colour, ncls) = _scheme(n, m, mode)
    s = class_sites(colour, colour[0])
    d2 = lat.distance2(0, s[1:])
    assert abs(np.sqrt(d2.min()) - a * np.sqrt(b)) < 1e-12


@pytest.mark.parametrize("n,m,mode", [(12, 6, 0), (12, 6, 1), (12, 3, 2), (8, 2, 0), (8, 2, 1), (8, 2, 2)])
def test_partition_and_class_sizes(n, m, mode):
    """Each site in exactly one set; m^4, m^4/2 or 2 m^4 sites per set (section 2.2)."""
    lat, (colour, ncls) = _scheme(n, m, mode)
    counts = np.bincount(colour, minlength=ncls)
    assert len(counts) == ncls and counts.sum() == lat.volume
    expect = {0: m ** 4, 1: m ** 4 // 2, 2: 2 * m ** 4}[mode]
    assert np.all(counts == expect)


def test_eq19_rmin_by_mode():
    """Eq. 19: r_min = r for modes 0 and 2, r sqrt(2) for mode 1 (here 8^4 and 16^3 x 8, r = 2, 4)."""
    for dims, r in (((8, 8, 8, 8), 2), ((16, 16, 16, 8), 4), ((8, 8, 8, 8), 4)):
        lat = Lattice(dims)
        for mode, expect in ((0, r), (1, r * np.sqrt(2)), (2, r)):
            m = [d // r for d in dims]
            if mode == 1 and any(mm % 2 for mm in m):
                continue
            colour, ncls = colouring(lat, (r,) * 4, mode)
            assert abs(r_min(lat, colour, ncls) - expect) < 1e-12


def test_nearest_neighbour_counts():
    """Section 3: 8 nearest same-class neighbours in mode 0, 24 in mode 1 (and in mode 2)."""
    lat, (colour, _) = _scheme(16, 4, 0)
    assert nearest_count(lat, colour, 0) == 8
    lat, (colour, _) = _scheme(16, 4, 1)
    assert nearest_count(lat, colour, 0) == 24
    lat, (colour, _) = _scheme(16, 4, 2)
    assert nearest_count(lat, colour, 0) == 24
    # with two class sites per direction +r and -r are the same image on the torus
    lat, (colour, _) = _scheme(12, 2, 0)
    assert nearest_count(lat, colour, 0) == 4


def test_combine_offset_and_rejections():
    lat = Lattice((8, 8, 8, 8))
    colour, _ = colouring(lat, (4, 4, 4, 4), 2)
    # the two merged offsets differ by (r/2, r/2, r/2, r/2)
    assert colour[lat.index(np.array([0, 0, 0, 0]))] == colour[lat.index(np.array([2, 2, 2, 2]))]
    assert colour[lat.index(np.array([0, 0, 0, 0]))] != colour[lat.index(np.array([2, 0, 0, 0]))]
    with pytest.raises(ValueError):
        colouring(lat, (3, 4, 4, 4), 0)          # r must divide n (Eq. 19)
    with pytest.raises(ValueError):
        colouring(Lattice((12, 12, 12, 12)), (4, 4, 4, 4), 1)   # odd number of class sites
    with pytest.raises(ValueError):
        colouring(Lattice((12, 12, 12, 12)), (3, 3, 3, 3), 2)   # odd gap in combine mode
    colour, n = point_colouring(lat)
    assert n == lat.volume and np.array_equal(colour, np.arange(lat.volume))
