"""A q(x) map in chunks of classes with checkpoint and resume, for maps that take hours
(32^3 x 64 at r = 8: 49152 sources).  After every chunk the partial q(x), Im q(x) and the
finished classes are written to an .npz file (atomically: a temporary file, then a rename);
a later call with the same file continues after the last finished chunk.  The classes of a
scheme cover disjoint sites, so the partial maps add up to the whole map exactly.

The file also records the lattice, the scheme's colouring and the Zolotarev coefficients;
resuming with anything different raises ValueError.
"""
import hashlib
import os

import numpy as np

from . import binding as smpq


def _fingerprint(ctx):
    col = smpq.smpq_get_coloring(ctx)
    c0, c, q, _ = smpq.smpq_get_zolotarev(ctx)
    h = hashlib.sha256()
    h.update(np.asarray(ctx.dims, dtype=np.int64).tobytes())
    h.update(col.tobytes())
    h.update(np.array([c0, *c, *q], dtype=np.float64).tobytes())
    return h.hexdigest()


def compute_qx_resumable(ctx, path, chunk=64, stop_after=None):
    """q(x) of every class of the context's scheme, chunk classes per call of the library.
    Needs the scheme and the Zolotarev coefficients set (they are part of the fingerprint).
    stop_after: return after that many new chunks (for tests and time-boxed jobs); the map is
    then incomplete and the call returns None.  Returns (qx, qx_imag, Q) when complete."""
    V = ctx.volume
    fp = _fingerprint(ctx)
    ncls = int(smpq.smpq_get_coloring(ctx).max()) + 1
    if os.path.exists(path):
        st = np.load(path)
        if str(st["fingerprint"]) != fp:
            raise ValueError(f"{path} belongs to another lattice, scheme or set of coefficients")
        qx, qi, done = st["qx"].copy(), st["qx_imag"].copy(), st["done"].copy()
    else:
        qx, qi, done = np.zeros(V), np.zeros(V), np.zeros(ncls, dtype=bool)
    todo = np.nonzero(~done)[0]
    chunks = 0
    for k0 in range(0, len(todo), chunk):
        if stop_after is not None and chunks >= stop_after:
            return None
        cls = todo[k0:k0 + chunk]
        q, im, _ = smpq.smpq_compute_qx_classes(ctx, cls)
        qx += q
        qi += im
        done[cls] = True
        tmp = path + ".tmp.npz"
        np.savez(tmp, qx=qx, qx_imag=qi, done=done, fingerprint=np.array(fp))
        os.replace(tmp, path)
        chunks += 1
    return qx, qi, float(qx.sum())
