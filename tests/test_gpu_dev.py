"""GPU: the entry points on caller-owned device memory give the same results as their host-buffer
counterparts, bit for bit (the same kernels).  The buffers come from hipMalloc of the HIP runtime
the library itself is linked to, called through ctypes: the caller's memory must belong to that
runtime instance."""
import ctypes

import numpy as np
import pytest

import paper_1901_02211_amd as smpq
import smpq_inputs as si

pytestmark = pytest.mark.gpu

H2D, D2H = 1, 2


class DeviceBuffer:
    """hipMalloc'ed memory of the runtime libsmpq.so uses (already loaded with the library)."""
    hip = None

    def __init__(self, nbytes):
        if DeviceBuffer.hip is None:
            DeviceBuffer.hip = ctypes.CDLL("libamdhip64.so.7")
            DeviceBuffer.hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        self.nbytes = nbytes
        self.ptr = ctypes.c_void_p()
        assert DeviceBuffer.hip.hipMalloc(ctypes.byref(self.ptr), ctypes.c_size_t(nbytes)) == 0

    def data_ptr(self):
        return self.ptr.value

    def upload(self, a):
        a = np.ascontiguousarray(a)
        assert a.nbytes == self.nbytes
        assert DeviceBuffer.hip.hipMemcpy(self.ptr, a.ctypes.data, a.nbytes, H2D) == 0

    def download(self, dtype, shape):
        out = np.empty(shape, dtype=dtype)
        assert out.nbytes == self.nbytes
        assert DeviceBuffer.hip.hipMemcpy(out.ctypes.data, self.ptr, out.nbytes, D2H) == 0
        return out

    def free(self):
        DeviceBuffer.hip.hipFree(self.ptr)


@pytest.mark.parametrize("prec", [smpq.SMPQ_FP64, smpq.SMPQ_MIXED_FP32])
def test_apply_dw_dev_equals_host(prec):
    dims = (6, 4, 4, 6)
    print(f"apply_dw on device buffers, {dims}, precision {prec}", flush=True)
    c = smpq.smpq_create(dims, 0)
    smpq.smpq_load_gauge(c, si.near_identity_su3(dims, 0.3, 31))
    psi = si.random_spinors(dims, 3, 32)
    d_in, d_out = DeviceBuffer(psi.nbytes), DeviceBuffer(psi.nbytes)
    d_in.upload(psi)
    try:
        for dag in (False, True):
            want = smpq.smpq_apply_dw(c, psi, dagger=dag, precision=prec)
            smpq.smpq_apply_dw_dev(c, d_in, d_out, 3, dagger=dag, precision=prec)
            got = d_out.download(np.complex128, psi.shape)
            assert np.array_equal(got, want), dag
    finally:
        d_in.free()
        d_out.free()
        smpq.smpq_destroy(c)


def test_compute_qx_dev_equals_host():
    print("compute_qx into device buffers, noise4 r=2", flush=True)
    c = smpq.smpq_create((4, 4, 4, 4), 0)
    smpq.smpq_load_gauge(c, si.workload("noise4"))
    smpq.smpq_set_zolotarev(c, 14, 0.13, 2.62)
    smpq.smpq_set_scheme(c, (2, 2, 2, 2), 0)
    smpq.smpq_set_solver(c, smpq.SMPQ_MIXED_FP32, 1e-12, 10000, 50)
    q, qi, Q, st = smpq.smpq_compute_qx(c)
    dq, dqi = DeviceBuffer(256 * 8), DeviceBuffer(256 * 8)
    try:
        Q2, st2 = smpq.smpq_compute_qx_dev(c, dq, dqi)
        assert np.array_equal(dq.download(np.float64, 256), q) and np.array_equal(dqi.download(np.float64, 256), qi)
        assert Q2 == Q and st2["n_sources"] == st["n_sources"] == 192
        Q3, _ = smpq.smpq_compute_qx_dev(c, dq.data_ptr(), None)   # a plain address, no imaginary part
        assert Q3 == Q and np.array_equal(dq.download(np.float64, 256), q)
    finally:
        dq.free()
        dqi.free()
        smpq.smpq_destroy(c)
