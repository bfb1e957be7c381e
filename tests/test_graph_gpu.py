"""swept_run and naive_run captured into a HIP graph (through torch's graph
capture on a side stream) replay the eager results bit for bit: every launch
goes to the caller's stream and the runs record no memset nodes.  The graph is
replayed several times, with eager runs of the same plan and host
synchronisations in between, and each replay is checked."""
import numpy as np
import pytest

from paper_1612_02495_amd import Plan, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    # kind, n, tile width, steps (trapezoid remainders; odd heat step counts
    # end the naive ping-pong with a device copy)
    ("heat", 2 ** 16, 1024, 1301),
    ("heat", 4096, 128, 333),
    ("ks", 2 ** 15, 1024, 517),
    ("heat_insulated", 2 ** 14, 512, 777),
]


@pytest.mark.parametrize("kind,n,w,steps", CASES)
def test_graph_replays_match_eager(kind, n, w, steps):
    print(f"graph {kind} n={n} w={w} steps={steps}", flush=True)
    if kind == "ks":
        p = inputs.ks(n=n, steps=steps)
        dt, dx, alpha = p.dt, p.dx, 0.0
        u0 = p.u0
    else:
        rng = np.random.default_rng(n + steps)
        u0 = rng.standard_normal(n)
        dx = 1.0 / n
        dt = 0.25 * dx * dx
        alpha = 1.0
    plan = Plan(n, kind, torch.float64, dt, dx, alpha, tile_width=w)
    ref_s = torch.tensor(u0, device="cuda")
    ref_n = ref_s.clone()
    plan.run(ref_s, steps)
    plan.naive(ref_n, steps)
    torch.cuda.synchronize()

    src = torch.tensor(u0, device="cuda")
    xs = src.clone()
    xn = src.clone()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=side):
        plan.run(xs, steps)
        plan.naive(xn, steps)
    other = src.clone()
    for rep in range(3):
        xs.copy_(src)
        xn.copy_(src)
        torch.cuda.synchronize()
        g.replay()
        plan.run(other, 37)  # eager work of the same plan between replays
        torch.cuda.synchronize()
        assert torch.equal(xs, ref_s), f"swept replay {rep}"
        assert torch.equal(xn, ref_n), f"naive replay {rep}"
    plan.close()
