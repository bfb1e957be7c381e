"""Single grids of any size: when no tile width divides n, the swept run uses
tiles of uneven width (two halves of floor(n / 2nt) or ceil(n / 2nt) points
each, on the compacted engine).  The paper's grids are powers of two
(Sec. 5), but the edge passing of Sec. 4.2 does not need that; the scheme is
unchanged, so every result equals the naive run and the oracle bit for bit.
"""
import zlib

import numpy as np
import pytest

import oracle
from paper_1612_02495_amd import Plan, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _params(kind, n):
    if kind == "heat":
        dx = 1.0 / n
        return dict(dt=0.3 * dx * dx, dx=dx, alpha=1.0)
    return dict(dt=0.005, dx=0.5, alpha=0.0)


def _oracle(kind, u0, prm, steps, np_dtype):
    if kind == "heat":
        return oracle.heat(u0, prm["alpha"], prm["dt"], prm["dx"], steps, dtype=np_dtype)
    return oracle.ks(u0, prm["dt"], prm["dx"], steps, dtype=np_dtype)


GENERAL_CASES = [
    # kind, n, w, steps_per_cycle, steps
    ("heat", 32, 0, 0, 50),       # one tile of halves 16 + 16
    ("heat", 33, 0, 0, 70),       # odd: one tile of 33 points (halves 16, 17)
    ("heat", 97, 512, 0, 333),    # prime, one tile
    ("heat", 1000, 0, 0, 1200),   # 8 x 125: no width of 256 or more divides it
    ("heat", 1025, 1024, 0, 999),  # two tiles, odd
    ("heat", 3001, 1024, 0, 2100),  # prime, three tiles of odd widths
    ("heat", 5003, 512, 37, 700),  # prime, short phases
    ("heat", 65537, 1024, 0, 800),  # prime, 65 tiles
    ("ks", 33, 0, 0, 41),
    ("ks", 97, 512, 0, 90),
    ("ks", 1001, 0, 0, 170),       # widths mod 4 = 1, 2, 3 appear
    ("ks", 1026, 1024, 0, 133),
    ("ks", 3001, 1024, 3, 77),
    ("ks", 7919, 512, 0, 260),     # prime
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind,n,w,spc,steps", GENERAL_CASES)
def test_uneven_tiles_equal_naive_and_oracle(kind, n, w, spc, steps, dtype):
    print(f"general {kind} n={n} w={w} spc={spc} steps={steps} {dtype}", flush=True)
    rng = np.random.default_rng(zlib.crc32(repr(("general", kind, n, w, spc, steps)).encode()))
    u0 = rng.standard_normal(n)
    prm = _params(kind, n)
    plan = Plan(n, kind, dtype, prm["dt"], prm["dx"], prm["alpha"], tile_width=w, steps_per_cycle=spc)
    us, un = _dev(u0, dtype), _dev(u0, dtype)
    plan.run(us, steps)
    plan.naive(un, steps)
    s, nv = _host(us), _host(un)
    assert np.array_equal(s, nv), f"max diff {np.max(np.abs(s - nv))}"
    np_dtype = np.float64 if dtype == torch.float64 else np.float32
    ref = _oracle(kind, u0.astype(np_dtype), prm, steps, np_dtype)
    assert np.array_equal(s, ref)


def test_prime_grid_of_a_million_points_vs_oracle():
    # n = 1000003 (prime) heat FP64 at 1000 steps, the automatic tiling
    n = 1000003
    p = inputs.heat_large(n=n, steps=1000)
    plan = Plan(n, "heat", torch.float64, p.dt, p.dx, p.alpha)
    info = plan.info()
    assert info["tile_width"] == 1024
    us = _dev(p.u0, torch.float64)
    plan.run(us, p.steps)
    s = _host(us)
    ref = oracle.heat(p.u0, p.alpha, p.dt, p.dx, p.steps)
    assert np.array_equal(s, ref)


def test_prime_ks_grid_vs_oracle():
    n = 65521  # largest prime below 2^16
    p = inputs.ks(n=n, steps=400)
    plan = Plan(n, "ks", torch.float64, p.dt, p.dx)
    us = _dev(p.u0, torch.float64)
    plan.run(us, p.steps)
    assert np.array_equal(_host(us), oracle.ks(p.u0, p.dt, p.dx, p.steps))


def test_uneven_composition_and_engine_rules():
    n = 4099
    prm = _params("heat", n)
    u0 = np.random.default_rng(3).standard_normal(n)
    plan = Plan(n, "heat", torch.float64, prm["dt"], prm["dx"], prm["alpha"], tile_width=1024)
    a, b = _dev(u0, torch.float64), _dev(u0, torch.float64)
    plan.run(a, 301)
    plan.run(a, 0)
    plan.run(a, 700)
    plan.run(b, 1001)
    assert np.array_equal(_host(a), _host(b))
    # uneven tiles run on the compacted engine only
    plan.set_engine("compact")
    plan.set_engine("auto")
    for e in ("wave", "lds"):
        with pytest.raises(Exception):
            plan.set_engine(e)
