"""Symmetric multi-probing colourings (section 2.2, Eqs. 15, 18, 19; Figs. 2-5; Tables 1-2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

A scheme P(m_x, m_y, m_z, m_t, mode) marks m_mu sites with the same colour along
direction mu; equivalently the gap is r_mu = n_mu / m_mu.  With the class offset
y_mu = x_mu mod r_mu:

  mode 0 (normal):  colour = y.                    prod(r) classes of prod(m) sites
  mode 1 (split):   colour = (y, sum_mu floor(x_mu / r_mu) mod 2), a checkerboard of
                    each class on its own coarse lattice; needs every m_mu even.
                                                   2 prod(r) classes of prod(m)/2 sites
  mode 2 (combine): the classes y and y + r/2 (all four directions) are merged;
                    needs every r_mu even.        prod(r)/2 classes of 2 prod(m) sites

Colour labels are contiguous: mode 0 uses the lexicographic index of y (x
fastest); mode 1 appends the parity as the lowest bit; mode 2 labels the pair by
its representative with y_t < r_t/2.  The "point" scheme gives every site its
own colour (point sources, section 2.1).
"""
import numpy as np


def gaps_from_m(dims, m):
    """r_mu = n_mu / m_mu for a scheme P(m_x, m_y, m_z, m_t, mode) (section 2.2)."""
    r = []
    for n, mm in zip(dims, m):
        if mm < 1 or n % mm:
            raise ValueError(f"m={mm} does not divide n={n}")
        r.append(n // mm)
    return tuple(r)


def colouring(lat, r, mode):
    """(colour[V], n_classes) of the scheme with gaps r (4-tuple) and mode 0/1/2."""
    r = tuple(int(v) for v in r)
    if len(r) != 4 or min(r) < 1:
        raise ValueError("r must be four positive integers")
    for n, rr in zip(lat.dims, r):
        if n % rr:
            raise ValueError(f"gap r={rr} does not divide n={n} (Eq. 19)")
    m = [n // rr for n, rr in zip(lat.dims, r)]
    x = lat.coords
    y = x % np.asarray(r)
    lex = y[:, 0] + r[0] * (y[:, 1] + r[1] * (y[:, 2] + r[2] * y[:, 3]))
    nbase = r[0] * r[1] * r[2] * r[3]
    if mode == 0:
        return lex, nbase
    if mode == 1:
        if any(mm % 2 for mm in m):
            raise ValueError("split mode needs an even number of class sites per direction")
        parity = (x // np.asarray(r)).sum(axis=1) % 2
        return 2 * lex + parity, 2 * nbase
    if mode == 2:
        if any(rr % 2 for rr in r):
            raise ValueError("combine mode needs an even gap in all four directions")
        half = np.asarray(r) // 2
        partner = (y + half) % np.asarray(r)
        rep = np.where((y[:, 3] < half[3])[:, None], y, partner)
        label = rep[:, 0] + r[0] * (rep[:, 1] + r[1] * (rep[:, 2] + r[2] * rep[:, 3]))
        return label, nbase // 2
    raise ValueError("mode must be 0, 1 or 2")


def point_colouring(lat):
    """Every site its own class: point sources (section 2.1, Eq. 5)."""
    return np.arange(lat.volume), lat.volume


def class_sites(colour, c):
    return np.nonzero(colour == c)[0]


def n_sources(n_classes):
    """One source per (class, Dirac index, colour index): 12 per class (section 2.2)."""
    return 12 * n_classes


def r_min(lat, colour, n_classes):
    """Minimal Euclidean distance between two sites of one class (Eq. 18), by brute force."""
    best = np.inf
    for c in range(n_classes):
        s = class_sites(colour, c)
        if len(s) < 2:
            continue
        d2 = lat.distance2(s[:, None], s[None, :])
        d2[np.arange(len(s)), np.arange(len(s))] = np.iinfo(np.int64).max
        best = min(best, d2.min())
    return np.sqrt(best)


def nearest_count(lat, colour, site):
    """Number of same-class sites at distance r_min from `site` (section 3)."""
    s = class_sites(colour, colour[site])
    d2 = lat.distance2(site, s)
    d2 = d2[s != site]
    return int((d2 == d2.min()).sum())
