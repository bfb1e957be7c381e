"""The benchmark workloads at their full size and horizon, in the launch
configuration the benchmark times (tile width, phase height and engine chosen
by the autotuner): the swept run equals the naive run of the same GPU bit for
bit (the swept rule does not change the scheme, Sec. 2), and heat keeps its
ring sum (Sec. 4.1: periodic FTCS conserves sum u; KS conserves it as well).

The oracle cannot run these horizons in test time; the naive kernel is pinned
to it element by element at 2^20 points elsewhere (test_parity_gpu.py,
test_insulated_gpu.py), and these runs extend that pin to the full horizons
through the bit-exact swept == naive invariant.
"""
import numpy as np
import pytest

from paper_1612_02495_amd import Plan, inputs, swept_autotune

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

WORKLOADS = {
    # name: (kind, dtype, problem)
    "heat": ("heat", torch.float64, lambda: inputs.heat_large(n=2 ** 20, steps=100000)),
    "heat_f32": ("heat", torch.float32, lambda: inputs.heat_large(n=2 ** 20, steps=100000)),
    "heat_rod": ("heat_insulated", torch.float64, lambda: inputs.heat_rod(n=2 ** 20, steps=100000)),
    "ks": ("ks", torch.float64, lambda: inputs.ks(n=2 ** 20, steps=20000)),
}


@pytest.mark.parametrize("name", sorted(WORKLOADS))
def test_bench_workload_full_horizon_swept_equals_naive(name):
    kind, dtype, make = WORKLOADS[name]
    p = make()
    dname = "f64" if dtype == torch.float64 else "f32"
    tuned = swept_autotune(p.n, kind, dname, p.dt, p.dx, p.alpha)
    print(f"{name}: n={p.n} steps={p.steps} tuned w={tuned['tile_width']} spc={tuned['steps_per_cycle']} "
          f"engine={tuned['engine']}", flush=True)
    plan = Plan(p.n, kind, dtype, p.dt, p.dx, p.alpha, tile_width=tuned["tile_width"],
                steps_per_cycle=tuned["steps_per_cycle"], engine=tuned["engine"])
    us = torch.tensor(p.u0, dtype=dtype, device="cuda")
    un = us.clone()
    plan.run(us, p.steps)
    plan.naive(un, p.steps)
    torch.cuda.synchronize()
    s, nv = us.cpu().numpy(), un.cpu().numpy()
    assert np.all(np.isfinite(s))
    assert np.array_equal(s, nv), f"max |swept - naive| = {np.max(np.abs(s.astype(np.float64) - nv))}"
    if kind == "heat" and dtype == torch.float64:
        # sum u is conserved by periodic FTCS up to rounding: T n eps max|u| bounds the drift
        u0 = p.u0
        bound = p.steps * p.n * np.finfo(np.float64).eps * np.abs(u0).max()
        assert abs(s.sum() - u0.sum()) <= bound
    plan.close()


def test_ks_full_horizon_vs_oracle_at_2p16():
    # KS at N = 2^16 over the workload's full 2*10^4 steps (t = 100, chaotic),
    # autotuned configuration, against the FP64 oracle element by element.
    # The oracle's all-cores leg gives the single-thread bits (pinned on the
    # CPU) and finishes in seconds.
    import oracle
    p = inputs.ks(n=2 ** 16, steps=20000)
    tuned = swept_autotune(p.n, "ks", "f64", p.dt, p.dx, p.alpha)
    plan = Plan(p.n, "ks", torch.float64, p.dt, p.dx, tile_width=tuned["tile_width"],
                steps_per_cycle=tuned["steps_per_cycle"], engine=tuned["engine"])
    us = torch.tensor(p.u0, device="cuda")
    plan.run(us, p.steps)
    torch.cuda.synchronize()
    ref, _ = oracle.ks_mt(p.u0, p.dt, p.dx, p.steps)
    got = us.cpu().numpy()
    assert np.array_equal(got, ref), f"rel max-norm {np.max(np.abs(got - ref)) / np.max(np.abs(ref))}"
    plan.close()


def test_ks_largest_grid_vs_oracle():
    # the top of the KS size range, N = 2^22, at 1000 steps
    import oracle
    p = inputs.ks(n=2 ** 22, steps=1000)
    plan = Plan(p.n, "ks", torch.float64, p.dt, p.dx, tile_width=1024)
    us = torch.tensor(p.u0, device="cuda")
    plan.run(us, p.steps)
    torch.cuda.synchronize()
    ref, _ = oracle.ks_mt(p.u0, p.dt, p.dx, p.steps)
    assert np.array_equal(us.cpu().numpy(), ref)
    plan.close()
