"""GPU parity of the insulated rod (arXiv 1612.02495, Sec. 4.1: heat
conduction in a rod with insulated ends): the swept run on the compacted
engine equals the naive kernel and the CPU oracle bit for bit.

The rod is laid on the same ring of tiles as the periodic grids; the ring
closes between nodes n-1 and 0, which sit at the middle of one tile in the
shifted tilings and at the outer points of the first and last tile in the
others.  Cases cover one-tile rods (both ends in one tile), several tiles,
trapezoid phases, remainder phases and runs shorter than one phase.
"""
import zlib

import numpy as np
import pytest

import oracle
from paper_1612_02495_amd import Plan, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    # n, w, steps_per_cycle, steps
    (512, 512, 0, 700),
    (1024, 512, 0, 600),
    (1536, 512, 100, 333),
    (1024, 512, 37, 200),
    (1024, 1024, 0, 1100),
    (2048, 1024, 0, 1300),
    (3072, 1024, 200, 900),
    (2048, 1024, 0, 17),
    (512, 512, 0, 3),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n,w,spc,steps", CASES)
def test_insulated_swept_equals_naive_and_oracle(n, w, spc, steps, dtype):
    print(f"insulated n={n} w={w} spc={spc} steps={steps} {dtype}", flush=True)
    rng = np.random.default_rng(zlib.crc32(repr(("ins", n, w, spc, steps)).encode()))
    u0 = rng.standard_normal(n)
    dx = 1.0 / (n - 1)
    dt = 0.3 * dx * dx
    plan = Plan(n, "heat_insulated", dtype, dt, dx, 1.0, tile_width=w, steps_per_cycle=spc)
    us = torch.tensor(u0, dtype=dtype, device="cuda")
    un = us.clone()
    plan.run(us, steps)
    plan.naive(un, steps)
    torch.cuda.synchronize()
    s, nv = us.cpu().numpy(), un.cpu().numpy()
    assert np.array_equal(s, nv), f"swept vs naive max diff {np.max(np.abs(s - nv))}"
    np_dtype = np.float64 if dtype == torch.float64 else np.float32
    ref = oracle.heat_insulated(u0.astype(np_dtype), 1.0, dt, dx, steps, dtype=np_dtype)
    assert np.array_equal(s, ref)


def test_insulated_rod_2p20_vs_oracle():
    p = inputs.heat_rod(n=2 ** 20, steps=1000)
    print("insulated rod n=2^20 steps=1000", flush=True)
    plan = Plan(p.n, "heat_insulated", torch.float64, p.dt, p.dx, p.alpha)
    assert plan.info()["tile_width"] == 1024
    u = torch.tensor(p.u0, device="cuda")
    plan.run(u, p.steps)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    assert np.array_equal(got, oracle.heat_insulated(p.u0, p.alpha, p.dt, p.dx, p.steps))
    # the trapezoid-weighted heat content is conserved by insulated ends
    w = np.ones(p.n)
    w[0] = w[-1] = 0.5
    assert abs(w @ got - w @ p.u0) <= 1e-9 * np.abs(p.u0).sum()


def test_insulated_rejects_other_engines_and_widths():
    plan = Plan(4096, "heat_insulated", torch.float64, 1e-7, 1e-3, 1.0, tile_width=1024)
    with pytest.raises(Exception):
        plan.set_engine("wave")
    with pytest.raises(Exception):
        plan.set_engine("lds")
    plan.set_engine("compact")
    with pytest.raises(Exception):
        Plan(4096, "heat_insulated", torch.float64, 1e-7, 1e-3, 1.0, tile_width=256)
