"""ctypes marshalling for libsmpq.so: numpy arrays in, numpy arrays out.

Host layouts (see include/smpq.h): gauge field complex128 [V, 4, 3, 3]
(site, mu, row, col); spinors complex128 [n, V, 4, 3] (rhs, site, spin, colour).
Errors raise SmpqError carrying the status and the library's message.
"""
import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsmpq.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1901_02211_amd/build.py`")
_lib = ctypes.CDLL(LIB_PATH)

__all__ = [
    "SMPQ_FP64", "SMPQ_MIXED_FP32", "SMPQ_MIXED_FP16DIR", "SMPQ_MIXED_BF16DIR", "SMPQ_MIXED_FP16VEC",
    "SMPQ_MIXED_BF16VEC", "SmpqError", "SmpqStats", "SmpqTuning", "LIB_PATH", "EXPORTS",
    "smpq_create", "smpq_destroy", "smpq_strerror", "smpq_last_error", "smpq_load_gauge",
    "smpq_set_kappa", "smpq_lanczos", "smpq_estimate_bounds", "smpq_set_zolotarev",
    "smpq_get_zolotarev", "smpq_set_solver", "smpq_get_settings", "SmpqSettings", "smpq_set_shift_check", "smpq_set_batch", "smpq_set_scheme",
    "smpq_set_point_scheme", "smpq_get_coloring", "smpq_get_scheme_rmin", "smpq_apply_dw", "smpq_apply_dw_noalloc", "smpq_apply_dw_dev", "smpq_apply_dov",
    "smpq_compute_qx_dev",
    "smpq_compute_qx", "smpq_compute_qx_classes", "smpq_compute_trinv", "smpq_dov_locality", "smpq_deflate", "smpq_compute_qx_points", "smpq_prepare", "smpq_set_stream",
    "smpq_set_timing", "smpq_set_graphs", "smpq_bench_dslash", "smpq_bench_copy", "smpq_bench_stream", "smpq_autotune",
    "smpq_set_tuning", "smpq_get_tuning", "smpq_set_memory_limit", "smpq_compute_qx_multi",
]

SMPQ_FP64 = 0
SMPQ_MIXED_FP32 = 1
SMPQ_MIXED_FP16DIR = 2   # FP32 body, shifted search directions stored in FP16 (scaled)
SMPQ_MIXED_BF16DIR = 3   # the same in BF16
SMPQ_MIXED_FP16VEC = 4   # FP32 body, the stencil's inputs (p and D_W p) rounded to FP16 (scaled)
SMPQ_MIXED_BF16VEC = 5   # the same rounded to BF16
_c_int_p = ctypes.POINTER(ctypes.c_int)
_c_double_p = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class SmpqTuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int) for n in ("f32_kind", "f32_nr", "f64_lgr", "plane_band", "f64_kind", "f64_nr",
                                            "f32_interleave", "f64_interleave", "f32_dag_kind", "f32_dag_nr",
                                            "f32_dag_interleave")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class SmpqSettings(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("precision", ctypes.c_int), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("reliable_interval", ctypes.c_int), ("gauge_hash", ctypes.c_uint64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class SmpqStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("lam_min", "lam_max", "zolo_delta", "t_bounds_s", "t_solve_s",
                                               "t_contract_s", "sum_imag_q", "max_abs_imag_q")] + \
               [(n, ctypes.c_int64) for n in ("n_sources", "n_batches", "total_iters", "max_iters",
                                              "n_reliable_updates", "shift_updates")] + \
               [("dslash_ms", ctypes.c_double), ("dslash_bytes", ctypes.c_double), ("dslash_launches", ctypes.c_int64),
                ("update_ms", ctypes.c_double), ("update_bytes", ctypes.c_double), ("update_launches", ctypes.c_int64),
                ("max_true_resid", ctypes.c_double), ("max_shift_resid", ctypes.c_double),
                ("max_shift_resid_final", ctypes.c_double), ("n_refined", ctypes.c_int64),
                ("refine_iters", ctypes.c_int64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_SIG = {
    "smpq_create": (ctypes.c_int, [_c_int_p, ctypes.c_int, ctypes.POINTER(_vp)]),
    "smpq_destroy": (None, [_vp]),
    "smpq_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "smpq_last_error": (ctypes.c_char_p, [_vp]),
    "smpq_load_gauge": (ctypes.c_int, [_vp, _c_double_p, ctypes.c_size_t]),
    "smpq_set_kappa": (ctypes.c_int, [_vp, ctypes.c_double]),
    "smpq_lanczos": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_uint64, _c_double_p, _c_double_p]),
    "smpq_estimate_bounds": (ctypes.c_int, [_vp, ctypes.c_int, _c_double_p, _c_double_p]),
    "smpq_set_zolotarev": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_double]),
    "smpq_get_zolotarev": (ctypes.c_int, [_vp, _c_int_p, _c_double_p, _c_double_p, _c_double_p, _c_double_p]),
    "smpq_set_solver": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int]),
    "smpq_get_settings": (ctypes.c_int, [_vp, ctypes.POINTER(SmpqSettings)]),
    "smpq_set_shift_check": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double]),
    "smpq_set_batch": (ctypes.c_int, [_vp, ctypes.c_int]),
    "smpq_set_scheme": (ctypes.c_int, [_vp, _c_int_p, ctypes.c_int, _c_int_p, _c_int_p]),
    "smpq_set_point_scheme": (ctypes.c_int, [_vp, _c_int_p, _c_int_p]),
    "smpq_get_coloring": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int32)]),
    "smpq_get_scheme_rmin": (ctypes.c_int, [_vp, _c_double_p, _c_int_p]),
    "smpq_apply_dw": (ctypes.c_int, [_vp, _c_double_p, _c_double_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "smpq_apply_dw_noalloc": (ctypes.c_int, [_vp, _c_double_p, _c_double_p, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int]),
    "smpq_apply_dov": (ctypes.c_int, [_vp, _c_double_p, _c_double_p, ctypes.c_int]),
    "smpq_apply_dw_dev": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "smpq_compute_qx_dev": (ctypes.c_int, [_vp, _vp, _vp, _c_double_p, ctypes.POINTER(SmpqStats)]),
    "smpq_compute_qx": (ctypes.c_int, [_vp, _c_double_p, _c_double_p, _c_double_p, ctypes.POINTER(SmpqStats)]),
    "smpq_compute_qx_classes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int, _c_double_p,
                                               _c_double_p, ctypes.POINTER(SmpqStats)]),
    "smpq_compute_trinv": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int, _c_double_p,
                                          _c_double_p, ctypes.POINTER(SmpqStats)]),
    "smpq_deflate": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _c_double_p, _c_double_p, _c_double_p]),
    "smpq_dov_locality": (ctypes.c_int, [_vp, ctypes.c_int64, _c_double_p, ctypes.POINTER(SmpqStats)]),
    "smpq_compute_qx_points": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, _c_double_p,
                                              ctypes.POINTER(SmpqStats)]),
    "smpq_prepare": (ctypes.c_int, [_vp]),
    "smpq_set_stream": (ctypes.c_int, [_vp, _vp]),
    "smpq_set_timing": (ctypes.c_int, [_vp, ctypes.c_int]),
    "smpq_set_graphs": (ctypes.c_int, [_vp, ctypes.c_int]),
    "smpq_bench_dslash": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _c_double_p,
                                         _c_double_p]),
    "smpq_autotune": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(SmpqTuning)]),
    "smpq_bench_copy": (ctypes.c_int, [_vp, ctypes.c_size_t, ctypes.c_int, _c_double_p]),
    "smpq_bench_stream": (ctypes.c_int, [_vp, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, _c_double_p]),
    "smpq_set_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(SmpqTuning)]),
    "smpq_get_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(SmpqTuning)]),
    "smpq_set_memory_limit": (ctypes.c_int, [_vp, ctypes.c_size_t]),
    "smpq_compute_qx_multi": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int,
                                             ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)), _c_int_p,
                                             ctypes.POINTER(_c_double_p), ctypes.POINTER(_c_double_p),
                                             ctypes.POINTER(SmpqStats), _c_int_p]),
}
EXPORTS = tuple(_SIG)
for _name, (_res, _args) in _SIG.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class SmpqError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_lib.smpq_strerror(status).decode()} ({status}): {message}")
        self.status = status


class _Ctx:
    """Owning handle of a smpq_ctx; destroyed with the object."""

    def __init__(self, ptr, dims):
        self.ptr = ptr
        self.dims = tuple(dims)
        self.volume = int(np.prod(dims))

    def __del__(self):
        if getattr(self, "ptr", None):
            _lib.smpq_destroy(self.ptr)
            self.ptr = None


def _check(ctx, status):
    if status != 0:
        msg = _lib.smpq_last_error(ctx.ptr).decode() if ctx is not None else ""
        raise SmpqError(status, msg)


def _dp(a):
    return a.ctypes.data_as(_c_double_p)


def _real_view(a, shape_tail, n_expected=None):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if a.shape[-len(shape_tail):] != tuple(shape_tail):
        raise ValueError(f"expected trailing shape {shape_tail}, got {a.shape}")
    return a, a.view(np.float64)


def smpq_strerror(status):
    return _lib.smpq_strerror(status).decode()


def smpq_last_error(ctx):
    return _lib.smpq_last_error(ctx.ptr).decode()


def smpq_create(dims, device=0):
    d = (ctypes.c_int * 4)(*[int(v) for v in dims])
    out = _vp()
    st = _lib.smpq_create(d, int(device), ctypes.byref(out))
    if st != 0:
        raise SmpqError(st, "smpq_create failed")
    return _Ctx(out, dims)


def smpq_destroy(ctx):
    if ctx.ptr:
        _lib.smpq_destroy(ctx.ptr)
        ctx.ptr = None


def smpq_load_gauge(ctx, U):
    U, r = _real_view(U, (4, 3, 3))
    _check(ctx, _lib.smpq_load_gauge(ctx.ptr, _dp(r), r.size))


def smpq_set_kappa(ctx, kappa):
    _check(ctx, _lib.smpq_set_kappa(ctx.ptr, float(kappa)))


def smpq_lanczos(ctx, steps, seed=0):
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(ctx, _lib.smpq_lanczos(ctx.ptr, int(steps), int(seed), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def smpq_estimate_bounds(ctx, steps=300):
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(ctx, _lib.smpq_estimate_bounds(ctx.ptr, int(steps), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def smpq_set_zolotarev(ctx, n_poles, lam_min, lam_max):
    _check(ctx, _lib.smpq_set_zolotarev(ctx.ptr, int(n_poles), float(lam_min), float(lam_max)))


def smpq_get_zolotarev(ctx):
    n = ctypes.c_int()
    c0, delta = ctypes.c_double(), ctypes.c_double()
    c = np.zeros(32)
    q = np.zeros(32)
    _check(ctx, _lib.smpq_get_zolotarev(ctx.ptr, ctypes.byref(n), ctypes.byref(c0), _dp(c), _dp(q),
                                        ctypes.byref(delta)))
    return c0.value, c[:n.value].copy(), q[:n.value].copy(), delta.value


def smpq_set_solver(ctx, precision=SMPQ_FP64, tol=1e-12, max_iter=10000, reliable_interval=50):
    _check(ctx, _lib.smpq_set_solver(ctx.ptr, int(precision), float(tol), int(max_iter), int(reliable_interval)))


def smpq_get_settings(ctx):
    """dict: kappa, precision, tol, max_iter, reliable_interval, gauge_hash."""
    out = SmpqSettings()
    _check(ctx, _lib.smpq_get_settings(ctx.ptr, ctypes.byref(out)))
    return out.as_dict()


def smpq_set_shift_check(ctx, enable=True, refine_tol=0.0):
    _check(ctx, _lib.smpq_set_shift_check(ctx.ptr, int(enable), float(refine_tol)))


def smpq_set_batch(ctx, max_rhs):
    _check(ctx, _lib.smpq_set_batch(ctx.ptr, int(max_rhs)))


def smpq_set_scheme(ctx, r, mode=0):
    rr = (ctypes.c_int * 4)(*[int(v) for v in r])
    nc, ns = ctypes.c_int(), ctypes.c_int()
    _check(ctx, _lib.smpq_set_scheme(ctx.ptr, rr, int(mode), ctypes.byref(nc), ctypes.byref(ns)))
    return nc.value, ns.value


def smpq_set_point_scheme(ctx):
    nc, ns = ctypes.c_int(), ctypes.c_int()
    _check(ctx, _lib.smpq_set_point_scheme(ctx.ptr, ctypes.byref(nc), ctypes.byref(ns)))
    return nc.value, ns.value


def smpq_get_coloring(ctx):
    out = np.zeros(ctx.volume, dtype=np.int32)
    _check(ctx, _lib.smpq_get_coloring(ctx.ptr, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return out


def smpq_get_scheme_rmin(ctx):
    """(r_min, number of same-class sites at r_min) of the current scheme."""
    r, n = ctypes.c_double(), ctypes.c_int()
    _check(ctx, _lib.smpq_get_scheme_rmin(ctx.ptr, ctypes.byref(r), ctypes.byref(n)))
    return r.value, n.value


def _spinors(ctx, psi):
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    if psi.ndim == 3:
        psi = psi[None]
    if psi.shape[1:] != (ctx.volume, 4, 3):
        raise ValueError(f"spinors must have shape (n, {ctx.volume}, 4, 3)")
    return psi


def smpq_apply_dw(ctx, psi, dagger=False, precision=SMPQ_FP64):
    psi = _spinors(ctx, psi)
    out = np.empty_like(psi)
    _check(ctx, _lib.smpq_apply_dw(ctx.ptr, _dp(psi.view(np.float64)), _dp(out.view(np.float64)), psi.shape[0],
                                   int(bool(dagger)), int(precision)))
    return out


def smpq_apply_dw_noalloc(ctx, psi, dagger=False, precision=SMPQ_FP64, out=None):
    """smpq_apply_dw through the library's fixed scratch (no device allocation); `out` may be a
    preallocated complex128 array of psi's shape."""
    psi = _spinors(ctx, psi)
    if out is None:
        out = np.empty_like(psi)
    elif out.shape != psi.shape or out.dtype != np.complex128 or not out.flags.c_contiguous:
        raise ValueError("out must be a C-contiguous complex128 array of the input's shape")
    _check(ctx, _lib.smpq_apply_dw_noalloc(ctx.ptr, _dp(psi.view(np.float64)), _dp(out.view(np.float64)),
                                           psi.shape[0], int(bool(dagger)), int(precision)))
    return out


def _dev_ptr(buf):
    """Device address of a caller-owned buffer: an int, or an object with data_ptr().  The memory
    must come from the HIP runtime libsmpq.so is linked to (see include/smpq.h)."""
    if buf is None:
        return None
    return ctypes.c_void_p(int(buf.data_ptr()) if hasattr(buf, "data_ptr") else int(buf))


def smpq_apply_dw_dev(ctx, in_buf, out_buf, n_rhs, dagger=False, precision=SMPQ_FP64):
    """D_W (or D_W^dag) of n_rhs spinors in device buffers of the host layout (24 V float64 each):
    in_buf / out_buf are device addresses or objects with data_ptr()."""
    _check(ctx, _lib.smpq_apply_dw_dev(ctx.ptr, _dev_ptr(in_buf), _dev_ptr(out_buf), int(n_rhs),
                                       int(bool(dagger)), int(precision)))


def smpq_compute_qx_dev(ctx, qx_buf, qxi_buf=None):
    """q(x) into caller-owned device buffers of V float64 (addresses or objects with data_ptr());
    returns (Q, stats)."""
    st = SmpqStats()
    Q = ctypes.c_double()
    _check(ctx, _lib.smpq_compute_qx_dev(ctx.ptr, _dev_ptr(qx_buf), _dev_ptr(qxi_buf), ctypes.byref(Q),
                                         ctypes.byref(st)))
    return Q.value, st.as_dict()


def smpq_apply_dov(ctx, psi):
    psi = _spinors(ctx, psi)
    out = np.empty_like(psi)
    _check(ctx, _lib.smpq_apply_dov(ctx.ptr, _dp(psi.view(np.float64)), _dp(out.view(np.float64)), psi.shape[0]))
    return out


def smpq_compute_qx(ctx):
    """Returns (qx, qx_imag, Q, stats dict)."""
    qx = np.zeros(ctx.volume)
    qi = np.zeros(ctx.volume)
    Q = ctypes.c_double()
    st = SmpqStats()
    _check(ctx, _lib.smpq_compute_qx(ctx.ptr, _dp(qx), _dp(qi), ctypes.byref(Q), ctypes.byref(st)))
    return qx, qi, Q.value, st.as_dict()


def smpq_compute_qx_classes(ctx, classes):
    """Returns (qx, qx_imag, stats dict) with zeros outside the listed classes."""
    cl = np.ascontiguousarray(classes, dtype=np.int32)
    qx = np.zeros(ctx.volume)
    qi = np.zeros(ctx.volume)
    st = SmpqStats()
    _check(ctx, _lib.smpq_compute_qx_classes(ctx.ptr, cl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(cl),
                                             _dp(qx), _dp(qi), ctypes.byref(st)))
    return qx, qi, st.as_dict()


def smpq_compute_trinv(ctx, classes=None):
    """Probing estimate of tr_sc D_W^-1(x, x): returns (t complex array of V, stats dict)."""
    t_re = np.zeros(ctx.volume)
    t_im = np.zeros(ctx.volume)
    st = SmpqStats()
    if classes is None:
        cp, n = None, 0
    else:
        cl = np.ascontiguousarray(classes, dtype=np.int32)
        cp, n = cl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(cl)
    _check(ctx, _lib.smpq_compute_trinv(ctx.ptr, cp, n, _dp(t_re), _dp(t_im), ctypes.byref(st)))
    return t_re + 1j * t_im, st.as_dict()


def smpq_deflate(ctx, n_modes, steps=80):
    """Deflate the n_modes lowest modes of H_W^2; returns (theta[n_modes + 1], theta_max,
    max relative residual)."""
    th = np.zeros(max(n_modes, 0) + 1)
    tmax, res = ctypes.c_double(), ctypes.c_double()
    _check(ctx, _lib.smpq_deflate(ctx.ptr, int(n_modes), int(steps), _dp(th), ctypes.byref(tmax),
                                  ctypes.byref(res)))
    return th, tmax.value, res.value


def smpq_dov_locality(ctx, site):
    """Mean absolute entry of the 12x12 blocks D_ov(x, . ; site, .) for every x: (m, stats)."""
    m = np.zeros(ctx.volume)
    st = SmpqStats()
    _check(ctx, _lib.smpq_dov_locality(ctx.ptr, int(site), _dp(m), ctypes.byref(st)))
    return m, st.as_dict()


def smpq_compute_qx_points(ctx, sites):
    s = np.ascontiguousarray(sites, dtype=np.int64)
    qx = np.zeros(len(s))
    st = SmpqStats()
    _check(ctx, _lib.smpq_compute_qx_points(ctx.ptr, s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(s),
                                            _dp(qx), ctypes.byref(st)))
    return qx, st.as_dict()


def smpq_prepare(ctx):
    _check(ctx, _lib.smpq_prepare(ctx.ptr))


def smpq_set_stream(ctx, stream_handle):
    """stream_handle: integer hipStream_t (e.g. torch.cuda.current_stream().cuda_stream) or None."""
    _check(ctx, _lib.smpq_set_stream(ctx.ptr, _vp(stream_handle) if stream_handle else None))


def smpq_set_timing(ctx, enable=True):
    _check(ctx, _lib.smpq_set_timing(ctx.ptr, int(bool(enable))))


def smpq_set_graphs(ctx, enable=True):
    _check(ctx, _lib.smpq_set_graphs(ctx.ptr, int(bool(enable))))


def smpq_bench_dslash(ctx, precision, n_rhs, n_sets, launches):
    ms, by = ctypes.c_double(), ctypes.c_double()
    _check(ctx, _lib.smpq_bench_dslash(ctx.ptr, int(precision), int(n_rhs), int(n_sets), int(launches),
                                       ctypes.byref(ms), ctypes.byref(by)))
    return ms.value, by.value


def smpq_autotune(ctx, n_rhs=48):
    """Times the stencil variants on this lattice; returns the chosen ones as a dict.
    n_rhs = 0 times them on the batch a whole map of the current scheme would use."""
    t = SmpqTuning()
    _check(ctx, _lib.smpq_autotune(ctx.ptr, int(n_rhs), ctypes.byref(t)))
    return t.as_dict()


def smpq_set_tuning(ctx, f32_kind, f32_nr, f64_lgr, plane_band=1, f64_kind=0, f64_nr=4, f32_interleave=1,
                    f64_interleave=1, f32_dag_kind=None, f32_dag_nr=None, f32_dag_interleave=None):
    """The D_W^dag variant defaults to the D_W one (f32_kind, f32_nr, f32_interleave)."""
    dk = f32_kind if f32_dag_kind is None else f32_dag_kind
    dn = f32_nr if f32_dag_nr is None else f32_dag_nr
    di = f32_interleave if f32_dag_interleave is None else f32_dag_interleave
    t = SmpqTuning(int(f32_kind), int(f32_nr), int(f64_lgr), int(plane_band), int(f64_kind), int(f64_nr),
                   int(f32_interleave), int(f64_interleave), int(dk), int(dn), int(di))
    _check(ctx, _lib.smpq_set_tuning(ctx.ptr, ctypes.byref(t)))


def smpq_get_tuning(ctx):
    t = SmpqTuning()
    _check(ctx, _lib.smpq_get_tuning(ctx.ptr, ctypes.byref(t)))
    return t.as_dict()


def smpq_set_memory_limit(ctx, nbytes):
    _check(ctx, _lib.smpq_set_memory_limit(ctx.ptr, int(nbytes)))


def smpq_compute_qx_multi(ctxs, classes=None):
    """q(x) of several contexts solved concurrently.  classes: None, or one entry per context
    (None for every class).  Returns a list of (qx, qx_imag, stats dict)."""
    n = len(ctxs)
    ptrs = (_vp * n)(*[c.ptr for c in ctxs])
    qx = [np.zeros(c.volume) for c in ctxs]
    qi = [np.zeros(c.volume) for c in ctxs]
    qxp = (_c_double_p * n)(*[_dp(a) for a in qx])
    qip = (_c_double_p * n)(*[_dp(a) for a in qi])
    st = (SmpqStats * n)()
    failed = ctypes.c_int(-1)
    cl_arrays, clp, ncl = [], None, None
    if classes is not None:
        i32p = ctypes.POINTER(ctypes.c_int32)
        clp = (i32p * n)()
        ncl = (ctypes.c_int * n)()
        for k, cl in enumerate(classes):
            if cl is None:
                clp[k] = i32p()
                ncl[k] = -1
            else:
                a = np.ascontiguousarray(cl, dtype=np.int32)
                cl_arrays.append(a)
                clp[k] = a.ctypes.data_as(i32p)
                ncl[k] = len(a)
    rc = _lib.smpq_compute_qx_multi(ptrs, n, clp, ncl, qxp, qip, st, ctypes.byref(failed))
    if rc != 0:
        k = failed.value
        msg = _lib.smpq_last_error(ctxs[k].ptr).decode() if 0 <= k < n else ""
        raise SmpqError(rc, f"context {k}: {msg}")
    return [(qx[k], qi[k], st[k].as_dict()) for k in range(n)]


def smpq_bench_copy(ctx, nbytes, launches=20):
    """Mean ms of one device-to-device copy of nbytes."""
    ms = ctypes.c_double()
    _check(ctx, _lib.smpq_bench_copy(ctx.ptr, int(nbytes), int(launches), ctypes.byref(ms)))
    return ms.value


def smpq_bench_stream(ctx, nbytes, launches=20, nontemporal=False):
    """Mean ms per launch of the library's streaming copy of nbytes (cached or non-temporal)."""
    ms = ctypes.c_double()
    _check(ctx, _lib.smpq_bench_stream(ctx.ptr, int(nbytes), int(launches), int(bool(nontemporal)), ctypes.byref(ms)))
    return ms.value
