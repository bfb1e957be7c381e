"""Read-before-write check: with SWEPT_DEBUG_POISON set when a plan is
created, its edge slots (and the adjoints' checkpoints and lambda slots) are
filled with quiet NaNs before each run.  A phase that read an entry no
earlier phase wrote would turn the result into NaN; every result below must
instead equal the naive run (and the oracle) bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1612_02495_amd import AdjointPlan, Batch, KsAdjointPlan, Plan, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture
def poison(monkeypatch):
    monkeypatch.setenv("SWEPT_DEBUG_POISON", "1")


# kind, n, w, steps_per_cycle (0 = full), steps, engine: trapezoid remainders,
# one-tile rings, runs shorter than one phase, every engine
CASES = [
    ("heat", 4096, 1024, 0, 1300, "compact"),
    ("heat", 2048, 1024, 0, 700, "compact"),
    ("heat", 4096, 512, 100, 333, "compact"),
    ("heat", 1024, 128, 0, 100, "wave"),
    ("heat", 2048, 256, 37, 301, "wave"),
    ("heat", 64, 16, 0, 45, "lds"),
    ("heat", 1000, 40, 7, 93, "lds"),
    ("ks", 4096, 1024, 0, 700, "compact"),
    ("ks", 2048, 512, 24, 150, "compact"),
    ("ks", 1024, 256, 0, 90, "wave"),
    ("ks", 256, 64, 8, 61, "lds"),
    ("heat_insulated", 2048, 1024, 0, 1100, "compact"),
    ("heat_insulated", 1536, 512, 100, 333, "compact"),
    # tiles of uneven width (no tile width divides n): the tiles holding the
    # ring's last half climb their triangle twice, one band per pass
    ("heat", 3001, 1024, 0, 2100, "compact"),
    ("heat", 1025, 512, 37, 700, "compact"),
    ("heat", 99, 1024, 0, 170, "compact"),
    ("ks", 3001, 1024, 0, 300, "compact"),
    ("ks", 1001, 512, 5, 170, "compact"),
    ("ks", 77, 1024, 0, 60, "compact"),
]


@pytest.mark.parametrize("kind,n,w,spc,steps,engine", CASES)
def test_poisoned_slots_swept_equals_naive(poison, kind, n, w, spc, steps, engine):
    print(f"poison {kind} n={n} w={w} spc={spc} steps={steps} {engine}", flush=True)
    rng = np.random.default_rng(n + steps)
    if kind == "ks":
        p = inputs.ks(n=n, steps=steps)
        u0, dt, dx, alpha = p.u0, p.dt, p.dx, 0.0
    else:
        u0 = rng.standard_normal(n)
        dx = 1.0 / n
        dt = 0.3 * dx * dx
        alpha = 1.0
    plan = Plan(n, kind, torch.float64, dt, dx, alpha, tile_width=w, steps_per_cycle=spc, engine=engine)
    us = torch.tensor(u0, device="cuda")
    un = us.clone()
    plan.run(us, steps)
    plan.run(us, 0)
    plan.naive(un, steps)
    torch.cuda.synchronize()
    s = us.cpu().numpy()
    assert np.all(np.isfinite(s)), "a phase read a slot entry no earlier phase wrote"
    assert np.array_equal(s, un.cpu().numpy())


@pytest.mark.parametrize("engine", ["auto", "compact", "wave"])
@pytest.mark.parametrize("kind", ["heat", "ks"])
def test_poisoned_batch_equals_naive(poison, kind, engine):
    sizes = np.array([32, 48, 272, 1040, 2064, 5008, 16400, 20000], dtype=np.int64)
    rng = np.random.default_rng(17)
    steps = 97
    if kind == "heat":
        dx = 1.0 / sizes
        dt = rng.uniform(0.05, 0.45, size=sizes.size) * dx * dx
        alpha = np.ones(sizes.size)
    else:
        dx = np.full(sizes.size, 0.5)
        dt = np.full(sizes.size, 0.005)
        alpha = np.zeros(sizes.size)
    u0 = [rng.standard_normal(int(m)) for m in sizes]
    b = Batch(sizes, kind, torch.float64, dt, dx, alpha, steps).set_engine(engine)
    u = torch.tensor(np.concatenate(u0), device="cuda")
    b.run(u)
    torch.cuda.synchronize()
    for i, part in enumerate(b.split(u)):
        got = part.cpu().numpy()
        assert np.all(np.isfinite(got)), f"grid {i}: a phase read an unwritten slot entry"
        plan = Plan(int(sizes[i]), kind, torch.float64, dt[i], dx[i], alpha[i], tile_width=16)
        v = torch.tensor(u0[i], device="cuda")
        plan.naive(v, steps)
        torch.cuda.synchronize()
        assert np.array_equal(got, v.cpu().numpy()), f"grid {i} (n={sizes[i]})"


@pytest.mark.parametrize("engine", ["auto", "compact"])
@pytest.mark.parametrize("kind", ["heat", "ks"])
def test_poisoned_batch_any_sizes(poison, kind, engine):
    # sizes off the 16-point lane lattice: ragged last lanes of the whole-grid
    # kernels, uneven swept tiles of every width residue
    sizes = np.array([33, 47, 263, 1025, 2049, 5003, 16385, 20001, 30011], dtype=np.int64)
    rng = np.random.default_rng(19)
    steps = 83
    if kind == "heat":
        dx = 1.0 / sizes
        dt = rng.uniform(0.05, 0.45, size=sizes.size) * dx * dx
        alpha = np.ones(sizes.size)
    else:
        dx = np.full(sizes.size, 0.5)
        dt = np.full(sizes.size, 0.005)
        alpha = np.zeros(sizes.size)
    u0 = [rng.standard_normal(int(m)) for m in sizes]
    b = Batch(sizes, kind, torch.float64, dt, dx, alpha, steps).set_engine(engine)
    u = torch.tensor(np.concatenate(u0), device="cuda")
    b.run(u)
    torch.cuda.synchronize()
    for i, part in enumerate(b.split(u)):
        got = part.cpu().numpy()
        assert np.all(np.isfinite(got)), f"grid {i}: a phase read an unwritten slot entry"
        plan = Plan(int(sizes[i]), kind, torch.float64, dt[i], dx[i], alpha[i])
        v = torch.tensor(u0[i], device="cuda")
        plan.naive(v, steps)
        torch.cuda.synchronize()
        assert np.array_equal(got, v.cpu().numpy()), f"grid {i} (n={sizes[i]})"


def test_poisoned_heat_adjoint(poison):
    n, steps, batch = 192, 101, 2
    rng = np.random.default_rng(3)
    dx = 1.0 / n
    dt = dx * dx
    alpha = rng.uniform(0.05, 0.45, size=batch)
    u0 = rng.standard_normal((batch, n))
    y = rng.standard_normal((batch, n))
    plan = AdjointPlan(batch, n, dt, dx, steps)
    du0 = torch.tensor(u0, device="cuda")
    uT = torch.empty_like(du0)
    plan.forward(du0, torch.tensor(alpha, device="cuda"), uT)
    g = torch.empty_like(du0)
    ga = torch.empty(batch, dtype=torch.float64, device="cuda")
    plan.adjoint((uT - torch.tensor(y, device="cuda")).contiguous(), g, ga)
    torch.cuda.synchronize()
    for b in range(batch):
        _, gref, garef = oracle.heat_adjoint(u0[b], y[b], alpha[b], dt, dx, steps)
        assert np.array_equal(g[b].cpu().numpy(), gref)
        assert abs(ga[b].item() - garef) <= 1e-12 * abs(garef)


def test_poisoned_ks_adjoint(poison):
    n, steps, batch = 256, 45, 2
    rng = np.random.default_rng(4)
    x = np.arange(n) * 0.5
    u0 = np.cos(x / 16.0) * (1.0 + np.sin(x / 16.0)) + 1e-3 * rng.standard_normal((batch, n))
    y = 0.1 * rng.standard_normal((batch, n))
    plan = KsAdjointPlan(batch, n, 0.005, 0.5, steps)
    du0 = torch.tensor(u0, device="cuda")
    uT = torch.empty_like(du0)
    plan.forward(du0, uT)
    g = torch.empty_like(du0)
    plan.adjoint((uT - torch.tensor(y, device="cuda")).contiguous(), g)
    torch.cuda.synchronize()
    for b in range(batch):
        _, gref = oracle.ks_adjoint(u0[b], y[b], 0.005, 0.5, steps)
        assert np.array_equal(g[b].cpu().numpy(), gref)
