"""Host-side checks of the batched ABI: argument validation before any
device call, and the size lattice of the batched inputs."""
import ctypes

import numpy as np
import pytest

from paper_1612_02495_amd import _lib, inputs


def _create(n, kind=0, dtype=1, steps=10, dt=None, dx=None, alpha=None):
    n = np.asarray(n, dtype=np.int64)
    m = n.size
    dt = np.full(m, 1e-6) if dt is None else np.asarray(dt, dtype=np.float64)
    dx = np.full(m, 1e-2) if dx is None else np.asarray(dx, dtype=np.float64)
    alpha = np.ones(m) if alpha is None else np.asarray(alpha, dtype=np.float64)
    pd = ctypes.POINTER(ctypes.c_double)
    h = ctypes.c_void_p()
    rc = _lib.lib().swept_batch_create(ctypes.byref(h), m, n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), kind,
                                       dtype, dt.ctypes.data_as(pd), dx.ctypes.data_as(pd),
                                       alpha.ctypes.data_as(pd), steps)
    return rc, h


@pytest.mark.parametrize("kw,code", [
    (dict(n=[256, 31]), _lib.SWEPT_EUNSUPPORTED),    # below 32
    (dict(n=[16]), _lib.SWEPT_EUNSUPPORTED),
    (dict(n=[(1 << 30) + 1]), _lib.SWEPT_EUNSUPPORTED),  # above 2^30
    (dict(n=[256], kind=4), _lib.SWEPT_EINVAL),
    (dict(n=[256], dtype=9), _lib.SWEPT_EINVAL),
    (dict(n=[256], steps=-1), _lib.SWEPT_EINVAL),
    (dict(n=[256, 512], dx=[1e-2, 0.0]), _lib.SWEPT_EINVAL),
    (dict(n=[256], dt=[float("nan")]), _lib.SWEPT_EINVAL),
])
def test_batch_create_rejects(kw, code):
    rc, h = _create(**kw)
    assert rc == code and not h.value


def test_batch_null_handles():
    lib = _lib.lib()
    assert lib.swept_batch_run(None, None, 1, None) == _lib.SWEPT_EINVAL
    assert lib.swept_batch_info(None, None, None, None, None) == _lib.SWEPT_EINVAL
    assert lib.swept_batch_set_engine(None, _lib.SWEPT_ENGINE_COMPACT) == _lib.SWEPT_EINVAL
    lib.swept_batch_destroy(None)
    h = ctypes.c_void_p()
    assert lib.swept_batch_create(ctypes.byref(h), 0, None, 0, 1, None, None, None, 1) == _lib.SWEPT_EINVAL


def test_batch_sizes_log_uniform_integers():
    probs = inputs.heat_batch(nprob=4096)
    n = np.array([p.n for p in probs])
    assert n.min() >= 256 and n.max() <= 65536
    # round(2^U(8,16)): integers of every residue, odd ones included
    assert 0.45 < np.mean(n % 2 == 1) < 0.55
    assert len(set((n % 16).tolist())) == 16
    # log-uniform: about a quarter of the sizes in each of [2^8,2^10), ..., [2^14,2^16]
    frac = np.histogram(np.log2(n), bins=[8, 10, 12, 14, 16.01])[0] / n.size
    assert np.all(np.abs(frac - 0.25) < 0.03)
    fo = np.array([p.extra["fo_drawn"] for p in probs])
    assert fo.min() >= 0.05 and fo.max() <= 0.45
