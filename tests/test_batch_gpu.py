"""Batched kernels on the GPU: every grid of the batch equals its own naive
run (and the oracle) bit for bit with every engine -- RESIDENT (grids of up
to 16384 points whole in one workgroup's registers, beside compacted swept
tiles for the rest), compacted tiles for all, register-engine tiles for all,
and AUTO; graph replays equal eager runs."""
import numpy as np
import pytest

import oracle
from paper_1612_02495_amd import Batch, Plan, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _sizes(seed, m, lattice=False):
    rng = np.random.default_rng(seed)
    if lattice:
        # sizes on the register engine's lane lattice (multiples of 16):
        # uneven halves, one-tile rings, multi-tile rings, the 2^16 maximum
        base = [32, 48, 256, 272, 1008, 1024, 1040, 2064, 4096, 4112, 5008, 8192, 8208, 16384, 16400, 65536]
        extra = list(16 * rng.integers(2, 700, size=m - len(base)))
        return np.array(base + extra, dtype=np.int64)
    # any integer sizes.  Whole-grid kernels: every count M = 1..16 of points
    # in the last lane (n = 16 (c-1) + M), a last lane that is lane 0 of its
    # wave (1025, 2049, 4097, 8193: M = 1; 1031: M = 7), the edges of the
    # size classes (1024 / 1025, 4096 / 4097, 8192 / 8193, 16384) and
    # primes.  Swept tiles: the first sizes beyond (16385, 16411 prime),
    # odd tile widths and every width mod 4 (KS), one-tile rings of odd
    # size under the compacted engine, and the largest prime below 2^16.
    base = [32, 33, 34, 35, 36, 37, 38, 39, 40, 41, 42, 43, 44, 45, 46, 47, 257, 263, 1023, 1025, 1031, 2049,
            4095, 4097, 4099, 8191, 8193, 16383, 16384, 16385, 16411, 20001, 33331, 65521]
    extra = list(np.rint(2.0 ** rng.uniform(5.0, 16.0, size=max(0, m - len(base)))).astype(np.int64))
    return np.array(base + extra, dtype=np.int64)


def _batch_case(kind, dtype, steps, seed=0, m=40, lattice=False):
    n = _sizes(seed, m, lattice)
    rng = np.random.default_rng(seed + 100)
    if kind == "heat":
        dx = 1.0 / n
        dt = rng.uniform(0.05, 0.45, size=n.size) * dx * dx
        alpha = np.ones(n.size)
    else:
        dx = np.full(n.size, 0.5)
        dt = np.full(n.size, 0.005)
        alpha = np.zeros(n.size)
    u0 = [rng.standard_normal(int(k)) for k in n]
    return n, dt, dx, alpha, u0


@pytest.mark.parametrize("engine", ["auto", "resident", "compact", "wave"])
@pytest.mark.parametrize("kind,dtype,steps", [("heat", torch.float64, 300), ("heat", torch.float32, 129),
                                              ("ks", torch.float64, 61), ("ks", torch.float32, 40)])
def test_batch_equals_per_grid_naive_and_oracle(kind, dtype, steps, engine):
    print(f"batch {engine} {kind} {dtype} steps={steps}", flush=True)
    # the register engine's halves are whole lanes: sizes on its lattice
    n, dt, dx, alpha, u0 = _batch_case(kind, dtype, steps, m=48, lattice=engine == "wave")
    b = Batch(n, kind, dtype, dt, dx, alpha, steps).set_engine(engine)
    u = torch.tensor(np.concatenate(u0), dtype=dtype, device="cuda")
    b.run(u, use_graph=True)
    torch.cuda.synchronize()
    parts = [t.cpu().numpy() for t in b.split(u)]
    np_dtype = np.float64 if dtype == torch.float64 else np.float32
    for i in range(n.size):
        plan = Plan(int(n[i]), kind, dtype, dt[i], dx[i], alpha[i])
        v = torch.tensor(u0[i], dtype=dtype, device="cuda")
        plan.naive(v, steps)
        torch.cuda.synchronize()
        assert np.array_equal(parts[i], v.cpu().numpy()), f"grid {i} (n={n[i]}) differs from naive"
        if n[i] <= 4096:
            ref = (oracle.heat(u0[i].astype(np_dtype), alpha[i], dt[i], dx[i], steps, dtype=np_dtype)
                   if kind == "heat" else oracle.ks(u0[i].astype(np_dtype), dt[i], dx[i], steps, dtype=np_dtype))
            assert np.array_equal(parts[i], ref), f"grid {i} (n={n[i]}) differs from the oracle"


@pytest.mark.parametrize("engine", ["auto", "resident", "compact", "wave"])
def test_batch_graph_replays_match_eager(engine):
    n, dt, dx, alpha, u0 = _batch_case("heat", torch.float64, 200, seed=5, m=40, lattice=engine == "wave")
    b = Batch(n, "heat", torch.float64, dt, dx, alpha, 200).set_engine(engine)
    state = torch.tensor(np.concatenate(u0), dtype=torch.float64, device="cuda")
    g = torch.empty_like(state)
    e = torch.empty_like(state)
    for rep in range(3):
        e.copy_(state)
        b.run(e, use_graph=False)  # eager reference on its own buffer
        torch.cuda.synchronize()
        g.copy_(state)
        b.run(g, use_graph=True)   # replay of the graph bound to g
        torch.cuda.synchronize()
        assert torch.equal(g, e), f"replay {rep} differs from eager"
        state = e.clone() * 0.5 + 1.0  # eager work between replays
        torch.cuda.synchronize()


def test_batch_full_workload_sampled():
    probs = inputs.heat_batch(nprob=4096, steps=5000)
    n = np.array([p.n for p in probs])
    dt = np.array([p.dt for p in probs])
    dx = np.array([p.dx for p in probs])
    b = Batch(n, "heat", torch.float64, dt, dx, np.ones(n.size), 5000)
    u0 = np.concatenate([p.u0 for p in probs])
    u = torch.tensor(u0, device="cuda")
    b.run(u)
    torch.cuda.synchronize()
    host = u.cpu().numpy()
    parts = [host[o:o + m] for o, m in zip(b.offsets, n)]
    # property at every size: the ring sum is conserved (heat FTCS, periodic)
    for i, p in enumerate(probs):
        assert abs(parts[i].sum() - p.u0.sum()) <= 1e-9 * max(1.0, np.abs(p.u0).sum())
    # sampled grids, smallest and largest included: bit for bit against naive
    order = np.argsort(n)
    pick = list(order[:3]) + list(order[-3:]) + list(np.random.default_rng(1).choice(n.size, 6, replace=False))
    for i in pick:
        plan = Plan(int(n[i]), "heat", torch.float64, dt[i], dx[i], 1.0)
        v = torch.tensor(probs[i].u0, device="cuda")
        plan.naive(v, 5000)
        torch.cuda.synchronize()
        assert np.array_equal(parts[i], v.cpu().numpy()), f"grid {i} (n={n[i]})"


@pytest.mark.parametrize("kind", ["heat", "ks"])
def test_batch_engines_agree_and_switch(kind):
    # heat: the compacted tiling has 8 points per lane and the register one
    # 16, so every switch rebuilds the grid descriptors and edge slots
    n, dt, dx, alpha, u0 = _batch_case(kind, torch.float64, 33, seed=9, m=20, lattice=True)
    b = Batch(n, kind, torch.float64, dt, dx, alpha, 33)
    x = torch.tensor(np.concatenate(u0), device="cuda")
    y = x.clone()
    b.run(x)                      # default (AUTO), graph
    b.set_engine("wave").run(y)   # register engine for every grid: the graph is re-captured
    torch.cuda.synchronize()
    assert torch.equal(x, y)
    b.set_engine("compact").run(y, use_graph=False)
    b.set_engine("resident").run(x, use_graph=False)
    torch.cuda.synchronize()
    assert torch.equal(x, y)
    with pytest.raises(Exception):
        b.set_engine("lds")


def test_wave_engine_refuses_sizes_off_its_lattice():
    n, dt, dx, alpha, u0 = _batch_case("heat", torch.float64, 10, m=40)
    b = Batch(n, "heat", torch.float64, dt, dx, alpha, 10)
    with pytest.raises(Exception):
        b.set_engine("wave")
    # the plan keeps its engine and still runs
    u = torch.tensor(np.concatenate(u0), device="cuda")
    b.run(u)
    torch.cuda.synchronize()
    plan = Plan(int(n[1]), "heat", torch.float64, dt[1], dx[1], 1.0)
    v = torch.tensor(u0[1], device="cuda")
    plan.naive(v, 10)
    torch.cuda.synchronize()
    assert np.array_equal(b.split(u)[1].cpu().numpy(), v.cpu().numpy())


@pytest.mark.parametrize("kind", ["heat", "ks"])
def test_batch_full_size_law_sampled_vs_oracle(kind):
    # the workload's own size law, round(2^U(8,16)), at a short horizon: every
    # grid equals its naive run, sampled grids up to 4096 points the oracle
    probs = (inputs.heat_batch(nprob=512, steps=97) if kind == "heat" else inputs.ks_batch(nprob=512, steps=41))
    steps = probs[0].steps
    n = np.array([p.n for p in probs])
    assert np.any(n % 16 != 0)
    b = Batch(n, kind, torch.float64, [p.dt for p in probs], [p.dx for p in probs],
              [p.alpha for p in probs], steps)
    u = torch.tensor(np.concatenate([p.u0 for p in probs]), device="cuda")
    b.run(u)
    torch.cuda.synchronize()
    parts = [t.cpu().numpy() for t in b.split(u)]
    checked = 0
    for i, p in enumerate(probs):
        plan = Plan(p.n, kind, torch.float64, p.dt, p.dx, p.alpha)
        v = torch.tensor(p.u0, device="cuda")
        plan.naive(v, steps)
        torch.cuda.synchronize()
        assert np.array_equal(parts[i], v.cpu().numpy()), f"grid {i} (n={p.n})"
        plan.close()
        if p.n <= 4096 and i % 8 == 0:
            ref = (oracle.heat(p.u0, p.alpha, p.dt, p.dx, steps) if kind == "heat"
                   else oracle.ks(p.u0, p.dt, p.dx, steps))
            assert np.array_equal(parts[i], ref), f"grid {i} (n={p.n}) vs oracle"
            checked += 1
    assert checked > 10
