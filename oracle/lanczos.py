"""Spectral bounds of |H_W| for the Zolotarev interval (Eq. 4; the paper is silent on how).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Reading: Lanczos on H_W^2 = D_W^dag D_W with full reorthogonalisation; the extreme
Ritz values theta_min, theta_max give |H_W| ~ [sqrt(theta_min), sqrt(theta_max)],
and the Zolotarev interval is widened to [0.9 sqrt(theta_min), 1.02 sqrt(theta_max)]
(Ritz values lie inside the spectrum).  No low-mode projection.

The start vector is drawn from SplitMix64 used as a counter-based generator
(Steele, Lea and Flood 2014; the 64-bit finaliser with multipliers
0xbf58476d1ce4e5b9 and 0x94d049bb133111eb): word i of a stream with seed s is
mix(s + (i + 1) * 0x9e3779b97f4a7c15), mapped to [0, 1) by its top 53 bits and
then to [-1, 1).  Real parts come from even counters, imaginary parts from odd
ones, in the order (site, spin, colour).
"""
import numpy as np
from scipy.linalg import eigvalsh_tridiagonal

from .dirac import apply_h2

LOW_MARGIN = 0.9
HIGH_MARGIN = 1.02


def splitmix64_uniform(seed, n):
    """n doubles in [0, 1) from the counter-based SplitMix64 stream `seed`."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.arange(1, n + 1, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def start_vector(volume, seed):
    u = 2.0 * splitmix64_uniform(seed, 24 * volume) - 1.0
    return (u[0::2] + 1j * u[1::2]).reshape(volume, 4, 3)


def ritz_extremes(U, lat, kappa, steps, seed=0):
    """Extreme Ritz values (theta_min, theta_max) of H_W^2 after `steps` Lanczos steps."""
    v = start_vector(lat.volume, seed)
    v = v / np.sqrt(np.vdot(v, v).real)
    basis = [v]
    alpha, beta = [], []
    for j in range(steps):
        w = apply_h2(U, lat, kappa, basis[-1])
        a = np.vdot(basis[-1], w).real
        w = w - a * basis[-1]
        if j > 0:
            w = w - beta[-1] * basis[-2]
        for _ in range(2):                          # full reorthogonalisation
            for b in basis:
                w = w - np.vdot(b, w) * b
        alpha.append(a)
        bnorm = np.sqrt(np.vdot(w, w).real)
        if j == steps - 1 or bnorm == 0.0:
            break
        beta.append(bnorm)
        basis.append(w / bnorm)
    theta = eigvalsh_tridiagonal(np.array(alpha), np.array(beta[:len(alpha) - 1]))
    return theta[0], theta[-1]


def bounds(U, lat, kappa, steps, seed=0):
    """Zolotarev interval [lam_min, lam_max] for |H_W| (widened Ritz extremes)."""
    tmin, tmax = ritz_extremes(U, lat, kappa, steps, seed)
    return LOW_MARGIN * np.sqrt(tmin), HIGH_MARGIN * np.sqrt(tmax)
