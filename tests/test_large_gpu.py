"""Grids past 32-bit indexing: a heat FP32 ring of 2^31 + 2^20 points and a KS
FP64 ring of 2^28 + 2^20 points (more than 2^31 bytes).  The swept run equals
the naive run bit for bit (compared on the device), and sampled points -- some
beyond index 2^31 -- equal the oracle: after T steps a point depends only on
the 2sT + 1 points around it, so the oracle run on that window as a periodic
ring of exactly that length reproduces it (every point of the window enters
its dependency cone once, through the same operations in the same order).
Inputs are drawn on the device from a seeded generator.  A plan whose phase
launch would exceed the 32-bit work-item count of one dispatch is refused
before it allocates."""
import numpy as np
import pytest

import oracle
from paper_1612_02495_amd import Plan, SweptError

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _window(u, x, half):
    n = u.numel()
    idx = (torch.arange(x - half, x + half + 1, device=u.device) % n)
    return u[idx].cpu().numpy()


def _run_pair(n, kind, dtype, dt, dx, alpha, steps, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    u0 = torch.rand(n, generator=g, device="cuda", dtype=dtype) * 2 - 1
    plan = Plan(n, kind, dtype, dt, dx, alpha, tile_width=1024)
    us = u0.clone()
    plan.run(us, steps)
    un = u0.clone()
    plan.naive(un, steps)
    torch.cuda.synchronize()
    return plan, u0, us, un


def test_heat_fp32_beyond_2p31_points():
    n = 2 ** 31 + 2 ** 20
    steps = 600  # phases of 512 and 88 steps
    print(f"heat f32 n={n} steps={steps}", flush=True)
    dx = 1.0 / n
    plan, u0, us, un = _run_pair(n, "heat", torch.float32, 0.25 * dx * dx, dx, 1.0, steps, seed=31)
    assert torch.equal(us, un)
    for x in (0, 12345, 2 ** 31 - 1, 2 ** 31 + 7, n - 1):
        w = _window(u0, x, steps).astype(np.float32)
        ref = oracle.heat(w, 1.0, 0.25 * dx * dx, dx, steps, dtype=np.float32)
        assert ref[steps] == us[x].item(), f"point {x}"
    del u0, us, un
    plan.close()
    torch.cuda.empty_cache()


def test_ks_fp64_beyond_2p31_bytes():
    n = 2 ** 28 + 2 ** 20
    steps = 200
    print(f"ks f64 n={n} steps={steps}", flush=True)
    plan, u0, us, un = _run_pair(n, "ks", torch.float64, 0.005, 0.5, 0.0, steps, seed=28)
    assert torch.equal(us, un)
    half = 2 * 2 * steps  # radius 2 per sub-step, two sub-steps per step
    for x in (3, 2 ** 28 - 5, 2 ** 28 + 4099, n - 2):
        w = _window(u0, x, half)
        ref = oracle.ks(w, 0.005, 0.5, steps)
        assert ref[half] == us[x].item(), f"point {x}"
    del u0, us, un
    plan.close()
    torch.cuda.empty_cache()


def test_too_many_tiles_for_one_launch_is_refused():
    # 2^28 tiles of 16 points, one wave64 each: 2^34 work-items in one phase
    with pytest.raises(SweptError, match="exceed one launch"):
        Plan(2 ** 32, "heat", torch.float32, 1e-6, 1e-3, 1.0, tile_width=16)
    print("2^32 points at tile width 16 refused", flush=True)
