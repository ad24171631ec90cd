"""Lattice geometry (section 2.1): L(nx, ny, nz, nt), periodic in every direction.

Site index s = x + nx*(y + ny*(z + nz*t)); direction mu = 0..3 is x, y, z, t.
TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
import numpy as np


class Lattice:
    def __init__(self, dims):
        self.dims = tuple(int(d) for d in dims)
        if len(self.dims) != 4 or min(self.dims) < 1:
            raise ValueError("dims must be four positive integers")
        nx, ny, nz, nt = self.dims
        self.volume = nx * ny * nz * nt
        s = np.arange(self.volume, dtype=np.int64)
        self.coords = np.stack([s % nx, (s // nx) % ny, (s // (nx * ny)) % nz,
                                s // (nx * ny * nz)], axis=1)
        self.fwd = np.stack([self.shift(mu, +1) for mu in range(4)])
        self.bwd = np.stack([self.shift(mu, -1) for mu in range(4)])

    def index(self, c):
        c = np.asarray(c) % np.asarray(self.dims)
        nx, ny, nz, _ = self.dims
        return c[..., 0] + nx * (c[..., 1] + ny * (c[..., 2] + nz * c[..., 3]))

    def shift(self, mu, step):
        c = self.coords.copy()
        c[:, mu] += step
        return self.index(c)

    def distance2(self, a, b):
        """Squared Euclidean minimum-image distance between sites a and b on the torus."""
        d = np.abs(self.coords[a] - self.coords[b])
        d = np.minimum(d, np.asarray(self.dims) - d)
        return (d * d).sum(axis=-1)
