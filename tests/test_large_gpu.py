"""Grids past 32-bit indexing: a heat FP32 ring of 2^31 + 2^20 points and a KS
FP64 ring of 2^28 + 2^20 points (more than 2^31 bytes).  The swept run equals
the naive run bit for bit (compared on the device), and sampled points -- some
beyond index 2^31 -- equal the oracle: after T steps a point depends only on
the 2sT + 1 points around it, so the oracle run on that window as a periodic
ring of exactly that length reproduces it (every point of the window enters
its dependency cone once, through the same operations in the same order).
A batch with two grids of the maximum 2^30 points puts its other grids past
element offset 2^31.  Inputs are drawn on the device from a seeded generator.
A plan whose phase launch would exceed the 32-bit work-item count of one
dispatch is refused before it allocates."""
import numpy as np
import pytest

import oracle
from paper_1612_02495_amd import Batch, Plan, SweptError

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


def test_batch_grids_beyond_2p31_offsets():
    # two grids of the maximum 2^30 points (compacted swept tiles) put the two
    # small grids behind them (register-resident) past element offset 2^31
    sizes = np.array([2 ** 30, 2 ** 30, 4096, 48], dtype=np.int64)
    steps = 3
    print(f"batch f32 sizes={sizes.tolist()} steps={steps}", flush=True)
    dx = 1.0 / sizes
    dt = 0.3 * dx * dx
    alpha = np.ones(sizes.size)
    b = Batch(sizes, "heat", torch.float32, dt, dx, alpha, steps)
    assert b.offsets[2] >= 2 ** 31  # beyond the int32 index range
    g = torch.Generator(device="cuda")
    g.manual_seed(30)
    u0 = torch.rand(b.total_points, generator=g, device="cuda", dtype=torch.float32) * 2 - 1
    u = u0.clone()
    b.run(u)
    torch.cuda.synchronize()
    for i, (got, start) in enumerate(zip(b.split(u), b.split(u0))):
        plan = Plan(int(sizes[i]), "heat", torch.float32, dt[i], dx[i], 1.0)  # naive only: any width
        v = start.clone()
        plan.naive(v, steps)
        torch.cuda.synchronize()
        assert torch.equal(got, v), f"grid {i} (n={sizes[i]})"
        # the oracle on the periodic window around a few points of the grid
        for x in (0, int(sizes[i]) // 2 + 3, int(sizes[i]) - 1):
            w = _window(start, x, steps).astype(np.float32)
            ref = oracle.heat(w, 1.0, dt[i], dx[i], steps, dtype=np.float32)
            assert ref[steps] == got[x].item(), f"grid {i} point {x}"
        plan.close()
        del v
    b.close()
    del u, u0
    torch.cuda.empty_cache()
