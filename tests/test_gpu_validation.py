"""The C ABI refuses buffers that are not device memory of the context's GPU,
or are shorter than the call implies, before it launches anything (the
pointers below are never dereferenced)."""
import ctypes

import numpy as np
import pytest
import torch

import inputs

pytestmark = pytest.mark.gpu

w = pytest.importorskip("paper_1011_2775_amd")
from paper_1011_2775_amd import _lib  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    dims = (4, 4, 4, 4)
    c = w.Context(dims)
    c.set_gauge(torch.from_numpy(inputs.gauge_field(dims, 0.3, 1001)).cuda())
    c.set_clover(-0.2, 1.0)
    yield c
    c.close()


def test_host_pointer_refused(ctx):
    host = np.zeros((256, 4, 3), np.complex128)
    out = torch.empty((256, 4, 3), dtype=torch.complex128, device="cuda")
    rc = _lib.LIB.wcmg_apply_D(ctx.h, 0, w.OP_FULL, w.F64, ctypes.c_void_p(out.data_ptr()),
                               ctypes.c_void_p(host.ctypes.data), 1)
    msg = _lib.LIB.wcmg_last_error()
    assert rc == _lib.EINVAL and (b"host memory" in msg or b"device pointer" in msg)
    rc = _lib.LIB.wcmg_solve(ctx.h, 0, w.GCR, ctypes.c_void_p(host.ctypes.data), ctypes.c_void_p(out.data_ptr()),
                             1, 1e-10, None)
    assert rc == _lib.EINVAL


def _address_range(ptr):
    """(base, size) of the device allocation holding ptr, from the HIP runtime torch loaded."""
    hip = ctypes.CDLL("libamdhip64.so.7")
    base, size = ctypes.c_void_p(), ctypes.c_size_t()
    rc = hip.hipMemGetAddressRange(ctypes.byref(base), ctypes.byref(size), ctypes.c_void_p(ptr))
    return (base.value, size.value) if rc == 0 and base.value else None


def test_short_device_buffer_refused(ctx):
    out = torch.zeros((256, 4, 3), dtype=torch.complex128, device="cuda")
    big = torch.zeros(1 << 21, dtype=torch.complex128, device="cuda")  # 32 MiB
    rng = _address_range(big.data_ptr())
    if rng is None:
        pytest.skip("the runtime reports no address range: the library cannot check lengths either")
    base, size = rng
    tail = base + size - 256  # 256 bytes before the end of the allocation; a spinor needs 49152
    rc = _lib.LIB.wcmg_apply_D(ctx.h, 0, w.OP_FULL, w.F64, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(tail), 1)
    assert rc == _lib.EINVAL and b"shorter" in _lib.LIB.wcmg_last_error()
    x = torch.randn((1, 4, 4, 4, 4, 4, 3), dtype=torch.complex128, device="cuda")
    y = ctx.apply_D(x)  # a correct call still goes through
    assert torch.isfinite(torch.view_as_real(y)).all()


def test_binding_refuses_wrong_dtype_on_gpu(ctx):
    x = torch.zeros((1, 4, 4, 4, 4, 4, 3), dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError, match="complex128"):
        ctx.apply_D(x)
    with pytest.raises(ValueError):
        ctx.apply_D(torch.zeros(100, dtype=torch.complex128, device="cuda"))
