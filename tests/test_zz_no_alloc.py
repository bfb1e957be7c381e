"""The allocation-free entry point, swept_run_noalloc, against swept_run.

swept_run_noalloc runs the same phase kernels as swept_run, with its edge
slots in the library's static per-device array instead of a plan's
allocation.  Two calls in a row on one GPU (the second on a smaller grid,
so it reuses the array left over by the first) must each give swept_run's
result bit for bit, and equal the naive run.
"""
import numpy as np
import pytest

from paper_1612_02495_amd import Plan, inputs
from paper_1612_02495_amd import _lib
from paper_1612_02495_amd import swept as sw

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _plan_run(p, kind, tile, steps, u0, engine=None):
    plan = Plan(p.n, kind, torch.float64, p.dt, p.dx, p.alpha if kind == "heat" else 0.0, tile_width=tile,
                engine=engine)
    u = torch.tensor(u0, device="cuda")
    plan.run(u, steps)
    v = torch.tensor(u0, device="cuda")
    plan.naive(v, steps)
    torch.cuda.synchronize()
    out = u.cpu().numpy(), v.cpu().numpy()
    plan.close()
    return out


def _noalloc_run(p, kind, tile, steps, u0, dtype=torch.float64):
    u = torch.tensor(u0, dtype=dtype, device="cuda")
    sw.swept_run_noalloc(p.n, kind, dtype, p.dt, p.dx, p.alpha if kind == "heat" else 0.0, tile, 0, u, steps)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def test_two_calls_in_a_row_match_swept_run():
    # first call: heat at 2^20 points, tile width 1024 (16.8 MB of edge slots,
    # the compacted engine), 700 steps (a remainder phase)
    h = inputs.heat_large(n=1 << 20, steps=700)
    got1 = _noalloc_run(h, "heat", 1024, h.steps, h.u0)
    want1, naive1 = _plan_run(h, "heat", 1024, h.steps, h.u0)
    assert np.array_equal(got1, want1)
    assert np.array_equal(got1, naive1)
    # second call: a smaller KS grid (tile width 512) in the array the first
    # call left behind
    k = inputs.ks(n=1 << 15, steps=150)
    got2 = _noalloc_run(k, "ks", 512, k.steps, k.u0)
    want2, naive2 = _plan_run(k, "ks", 512, k.steps, k.u0)
    assert np.array_equal(got2, want2)
    assert np.array_equal(got2, naive2)


def test_repeat_and_engines_and_fp32():
    # register engine width (w = 256) and the LDS engine width (w = 32), then
    # FP32, each against swept_run of a plan with the same configuration
    h = inputs.heat_large(n=1 << 14, steps=333)
    for tile in (256, 32):
        got = _noalloc_run(h, "heat", tile, h.steps, h.u0)
        want, naive = _plan_run(h, "heat", tile, h.steps, h.u0)
        assert np.array_equal(got, want), tile
        assert np.array_equal(got, naive), tile
    u0 = h.u0.astype(np.float32)
    got = _noalloc_run(h, "heat", 512, h.steps, u0, dtype=torch.float32)
    plan = Plan(h.n, "heat", torch.float32, h.dt, h.dx, h.alpha, tile_width=512)
    u = torch.tensor(u0, device="cuda")
    plan.run(u, h.steps)
    torch.cuda.synchronize()
    assert np.array_equal(got, u.cpu().numpy())
    plan.close()


def test_size_limit_is_refused_before_launch():
    # 2^22 FP64 points at tile width 1024 need 2 * 4096 * 1026 * 8 bytes of
    # slots, beyond the 32 MiB array: refused, the grid untouched
    n = 1 << 22
    u = torch.ones(n, dtype=torch.float64, device="cuda")
    with pytest.raises(sw.SweptError) as ei:
        sw.swept_run_noalloc(n, "heat", torch.float64, 1e-12, 1.0 / n, 1.0, 1024, 0, u, 10)
    assert ei.value.code == _lib.SWEPT_EUNSUPPORTED
    assert "static workspace" in str(ei.value)
    torch.cuda.synchronize()
    assert bool(torch.all(u == 1.0))
