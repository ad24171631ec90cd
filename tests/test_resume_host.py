"""Host-side checks of the resumable map (no GPU): a checkpoint of another lattice, scheme, set
of coefficients, kappa, solver setting or gauge field is refused before any solve, and a
complete checkpoint is returned as is."""
import numpy as np
import pytest

import paper_1901_02211_amd as smpq
from paper_1901_02211_amd.resume import _fingerprint, compute_qx_resumable


def _host_ctx(dims=(4, 4, 4, 4), r=2, lo=0.15, kappa=0.21, prec=smpq.SMPQ_MIXED_FP32, tol=1e-12):
    c = smpq.smpq_create(dims, -1)
    smpq.smpq_set_scheme(c, (r,) * 4, 0)
    smpq.smpq_set_zolotarev(c, 14, lo, 2.75)
    smpq.smpq_set_kappa(c, kappa)
    smpq.smpq_set_solver(c, prec, tol, 10000, 50)
    return c


def test_fingerprint_separates_lattice_scheme_and_coefficients():
    base = _fingerprint(_host_ctx())
    assert _fingerprint(_host_ctx()) == base
    assert _fingerprint(_host_ctx(dims=(4, 4, 4, 8))) != base
    assert _fingerprint(_host_ctx(r=4)) != base
    assert _fingerprint(_host_ctx(lo=0.2)) != base
    assert _fingerprint(_host_ctx(kappa=0.2)) != base
    assert _fingerprint(_host_ctx(prec=smpq.SMPQ_FP64)) != base
    assert _fingerprint(_host_ctx(tol=1e-10)) != base


def test_fingerprint_separates_gauge_fields(monkeypatch):
    """Two gauge fields (a host-only context cannot load one, so the library's settings are
    stood in for) give two fingerprints; so does no field at all."""
    import paper_1901_02211_amd.resume as res
    c = _host_ctx()
    real = smpq.smpq_get_settings(c)
    assert real["gauge_hash"] == 0 and real["kappa"] == 0.21 and real["reliable_interval"] == 50
    prints = set()
    for h in (0, 1234567, 7654321):
        monkeypatch.setattr(res.smpq, "smpq_get_settings", lambda ctx, h=h: dict(real, gauge_hash=h))
        prints.add(res._fingerprint(c))
    assert len(prints) == 3


def test_foreign_checkpoint_is_refused(tmp_path):
    path = str(tmp_path / "map.npz")
    other = _host_ctx(lo=0.2)
    np.savez(path, qx=np.zeros(256), qx_imag=np.zeros(256), done=np.zeros(16, dtype=bool),
             fingerprint=np.array(_fingerprint(other)))
    with pytest.raises(ValueError):
        compute_qx_resumable(_host_ctx(), path)


def test_complete_checkpoint_needs_no_solve(tmp_path):
    """All classes done: the stored map comes back without a library solve (a host-only context
    could not run one), extra arrays and statistics survive."""
    c = _host_ctx()
    path = str(tmp_path / "map.npz")
    q = np.linspace(-1.0, 1.0, 256)
    np.savez(path, qx=q, qx_imag=np.zeros(256), done=np.ones(16, dtype=bool),
             fingerprint=np.array(_fingerprint(c)), seconds=3.0, iters=7, interval=np.array([0.15, 2.75]))
    qx, qi, Q = compute_qx_resumable(c, path)
    assert np.array_equal(qx, q) and Q == pytest.approx(q.sum())
    st = np.load(path)
    assert float(st["seconds"]) == 3.0 and int(st["iters"]) == 7 and "interval" in st.files
