"""The opt-in non-finite check (swept_plan_set_checks, swept_batch_set_checks):
a NaN or Inf put into the initial state reaches the result, and the run then
returns SWEPT_ENONFINITE through the C ABI; a clean run returns SWEPT_OK with
the same bits as an unchecked run."""
import ctypes

import numpy as np
import pytest

from paper_1612_02495_amd import Batch, Plan, SweptError, _lib, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _stream():
    return ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind,n,w", [("heat", 4096, 1024), ("ks", 3001, 1024), ("heat", 1024, 64)])
def test_plan_check(kind, n, w, dtype):
    p = inputs.heat_large(n=n, steps=300) if kind == "heat" else inputs.ks(n=n, steps=60)
    plan = Plan(n, kind, dtype, p.dt, p.dx, p.alpha, tile_width=w)
    ref = torch.tensor(p.u0, dtype=dtype, device="cuda")
    plan.run(ref, p.steps)                       # unchecked
    plan.set_checks(True)
    u = torch.tensor(p.u0, dtype=dtype, device="cuda")
    rc = _lib.lib().swept_run(plan._h, ctypes.c_void_p(u.data_ptr()), p.steps, _stream())
    assert rc == _lib.SWEPT_OK
    torch.cuda.synchronize()
    assert torch.equal(u, ref)
    for bad in (float("nan"), float("inf")):
        u0 = p.u0.copy()
        u0[n // 3] = bad
        u = torch.tensor(u0, dtype=dtype, device="cuda")
        rc = _lib.lib().swept_run(plan._h, ctypes.c_void_p(u.data_ptr()), p.steps, _stream())
        assert rc == _lib.SWEPT_ENONFINITE
        assert "non-finite" in _lib.last_error()
        v = torch.tensor(u0, dtype=dtype, device="cuda")
        with pytest.raises(SweptError) as ei:
            plan.naive(v, p.steps)
        assert ei.value.code == _lib.SWEPT_ENONFINITE
    # switched off, the same run returns OK (and the grid holds NaN)
    plan.set_checks(False)
    u = torch.tensor(u0, dtype=dtype, device="cuda")
    plan.run(u, p.steps)
    torch.cuda.synchronize()
    assert not bool(torch.isfinite(u).all())


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_check(use_graph):
    sizes = np.array([33, 1025, 4099, 20001, 40000], dtype=np.int64)
    rng = np.random.default_rng(5)
    dx = 1.0 / sizes
    dt = rng.uniform(0.05, 0.45, size=sizes.size) * dx * dx
    u0 = [rng.standard_normal(int(m)) for m in sizes]
    b = Batch(sizes, "heat", torch.float64, dt, dx, np.ones(sizes.size), 150)
    ref = torch.tensor(np.concatenate(u0), device="cuda")
    b.run(ref, use_graph=use_graph)
    b.set_checks(True)
    u = torch.tensor(np.concatenate(u0), device="cuda")
    b.run(u, use_graph=use_graph)
    torch.cuda.synchronize()
    assert torch.equal(u, ref)
    for g in (0, 3):
        bad = [x.copy() for x in u0]
        bad[g][7] = np.nan
        u = torch.tensor(np.concatenate(bad), device="cuda")
        with pytest.raises(SweptError) as ei:
            b.run(u, use_graph=use_graph)
        assert ei.value.code == _lib.SWEPT_ENONFINITE
    b.set_checks(False)
    b.run(u, use_graph=use_graph)
    torch.cuda.synchronize()
