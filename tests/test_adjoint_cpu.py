"""Host-side validation of the adjoint ABI (no kernel runs)."""
import ctypes

import pytest

from paper_1612_02495_amd import _lib


@pytest.mark.parametrize("args,code", [
    ((0, 1024, 1, 1e-6, 1e-3, 100), _lib.SWEPT_EINVAL),        # batch
    ((65536, 1024, 1, 1e-6, 1e-3, 100), _lib.SWEPT_EINVAL),    # batch beyond one grid dimension
    ((2, 1000, 1, 1e-6, 1e-3, 100), _lib.SWEPT_EUNSUPPORTED),  # n not a multiple of 64
    ((2, 1024, 0, 1e-6, 1e-3, 100), _lib.SWEPT_EUNSUPPORTED),  # f32
    ((2, 1024, 1, 1e-6, 1e-3, 0), _lib.SWEPT_EINVAL),          # steps
    ((2, 1024, 1, 1e-6, 0.0, 10), _lib.SWEPT_EINVAL),          # dx
    ((65535, 65600, 1, 1e-6, 1e-3, 10), _lib.SWEPT_EUNSUPPORTED),  # batch x n beyond one launch
])
def test_adjoint_create_rejects(args, code):
    h = ctypes.c_void_p()
    assert _lib.lib().swept_adjoint_create(ctypes.byref(h), *args) == code
    assert not h.value


def test_adjoint_null_handles():
    lib = _lib.lib()
    assert lib.swept_forward_ckpt(None, None, None, None, None) == _lib.SWEPT_EINVAL
    assert lib.swept_adjoint_run(None, None, None, None, None) == _lib.SWEPT_EINVAL
    assert lib.swept_adjoint_info(None, None, None, None, None) == _lib.SWEPT_EINVAL
    lib.swept_adjoint_destroy(None)


@pytest.mark.parametrize("args,code", [
    ((0, 1024, 1, 0.005, 0.5, 100), _lib.SWEPT_EINVAL),        # batch
    ((65536, 1024, 1, 0.005, 0.5, 100), _lib.SWEPT_EINVAL),    # batch beyond one grid dimension
    ((1, 1000, 1, 0.005, 0.5, 100), _lib.SWEPT_EUNSUPPORTED),  # n not a multiple of 64
    ((1, 32, 1, 0.005, 0.5, 100), _lib.SWEPT_EUNSUPPORTED),    # n below one tile
    ((1, 1024, 0, 0.005, 0.5, 100), _lib.SWEPT_EUNSUPPORTED),  # f32
    ((1, 1024, 1, 0.005, 0.5, 0), _lib.SWEPT_EINVAL),          # steps
    ((1, 1024, 1, 0.005, 0.0, 10), _lib.SWEPT_EINVAL),         # dx
    ((1, 1024, 1, float("nan"), 0.5, 10), _lib.SWEPT_EINVAL),  # dt
    ((65535, 65600, 1, 0.005, 0.5, 10), _lib.SWEPT_EUNSUPPORTED),  # batch x n beyond one launch
])
def test_ks_adjoint_create_rejects(args, code):
    h = ctypes.c_void_p()
    assert _lib.lib().swept_ks_adjoint_create(ctypes.byref(h), *args) == code
    assert not h.value


def test_ks_adjoint_null_handles():
    lib = _lib.lib()
    assert lib.swept_ks_forward_ckpt(None, None, None, None) == _lib.SWEPT_EINVAL
    assert lib.swept_ks_adjoint_run(None, None, None, None) == _lib.SWEPT_EINVAL
    assert lib.swept_ks_adjoint_info(None, None, None, None, None) == _lib.SWEPT_EINVAL
    lib.swept_ks_adjoint_destroy(None)


def test_segmented_create_rejects_before_any_device_call():
    import ctypes
    h = ctypes.c_void_p()
    lib = _lib.lib()
    assert lib.swept_adjoint_create_segmented(ctypes.byref(h), 2, 256, 1, 1e-5, 1e-2, 100, -1) == _lib.SWEPT_EINVAL
    assert lib.swept_adjoint_create_segmented(ctypes.byref(h), 0, 256, 1, 1e-5, 1e-2, 100, 0) == _lib.SWEPT_EINVAL
    assert lib.swept_adjoint_create_segmented(None, 2, 256, 1, 1e-5, 1e-2, 100, 0) == _lib.SWEPT_EINVAL
