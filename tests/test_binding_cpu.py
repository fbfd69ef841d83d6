"""The Python binding validates every buffer before it hands a raw pointer
to the C ABI (no GPU needed: every check raises before the library is
called).  The C side repeats the device-memory checks (see the GPU tests)."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1011_2775_amd as w
from paper_1011_2775_amd import _dev, _ptr


def fake_context(dims=(4, 4, 4, 4)):
    """A Context whose handle is null: any call that reached the library would fail there."""
    c = w.Context.__new__(w.Context)
    c.dims = [tuple(dims)]
    c.h = ctypes.c_void_p()
    c.params = {0: w.default_params(block=[(2, 2, 2, 2)], nvec=[4])}
    return c


def test_dev_rejects_cpu_wrong_dtype_and_bad_length():
    t = torch.zeros(24, dtype=torch.complex128)
    with pytest.raises(ValueError, match="CUDA"):
        _dev(t, 12, "x")


def test_ptr_converts_and_keeps_alive():
    a = np.arange(6, dtype=np.float64)[::2]  # non-contiguous, real
    p, dev, keep = _ptr(a, 3, "v")
    assert dev == 0 and keep.dtype == np.complex128 and keep.flags.c_contiguous
    assert p.value == keep.ctypes.data
    assert np.array_equal(keep.real, [0.0, 2.0, 4.0])
    with pytest.raises(ValueError, match="elements"):
        _ptr(np.zeros(4, np.complex128), 3, "v")
    with pytest.raises(ValueError, match="complex128"):
        _ptr(torch.zeros(3, dtype=torch.complex64), 3, "v")
    with pytest.raises(ValueError, match="contiguous"):
        _ptr(torch.zeros((3, 2), dtype=torch.complex128).t(), 6, "v")


@pytest.mark.parametrize("call", ["apply_D", "apply_Ddag", "solve", "solve_dag", "restrict", "force"])
def test_context_calls_reject_host_tensors(call):
    c = fake_context()
    x = torch.zeros((1, 4, 4, 4, 4, 4, 3), dtype=torch.complex128)
    with pytest.raises(ValueError, match="CUDA"):
        if call == "force":
            c.force(x, x)
        else:
            getattr(c, call)(x)


def test_set_gauge_checks_size_and_dtype():
    c = fake_context()
    with pytest.raises(ValueError, match="elements"):
        c.set_gauge(np.zeros((4, 4, 4, 4, 4, 3, 2), np.complex128))
    with pytest.raises(ValueError, match="complex128"):
        c.set_gauge(torch.zeros((4, 4, 4, 4, 4, 3, 3), dtype=torch.complex64))


def test_dot_rejects_mismatched_lengths_before_the_library():
    c = fake_context()
    x = torch.zeros(8, dtype=torch.complex128)
    with pytest.raises(ValueError):
        c.dot(x, x)
