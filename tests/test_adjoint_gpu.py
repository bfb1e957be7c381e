"""Swept adjoint on the GPU against the FP64 CPU reverse sweep, against
steps applications of the forward stencil (bit for bit), and against central
finite differences of the forward run."""
import math

import numpy as np
import pytest

import oracle
from paper_1612_02495_amd import AdjointPlan, Plan, inputs, swept_heat

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


# n = 576 is 9 tiles: the 8-tile waves of the checkpointing forward end in a
# wave holding one tile; n = 2112 (33 tiles) and 2560 (40 tiles) give the
# chained reverse launch (chains of 16 tiles) two full chains and a last
# chain of 1 and of 8 tiles, with chains of odd and even length
@pytest.mark.parametrize("n,steps", [(64, 5), (64, 32), (128, 45), (256, 96), (192, 101), (512, 333), (576, 70),
                                     (2112, 130), (2560, 97)])
def test_adjoint_matches_cpu_reverse_sweep(n, steps):
    rng = np.random.default_rng(n * 1000 + steps)
    batch = 3
    dx = 1.0 / n
    dt = dx * dx
    alpha = rng.uniform(0.05, 0.45, size=batch)
    u0 = rng.standard_normal((batch, n))
    y = rng.standard_normal((batch, n))
    plan = AdjointPlan(batch, n, dt, dx, steps)
    du0 = torch.tensor(u0, device="cuda")
    dal = torch.tensor(alpha, device="cuda")
    uT = torch.empty_like(du0)
    plan.forward(du0, dal, uT)
    g_uT = uT - torch.tensor(y, device="cuda")
    g_u0 = torch.empty_like(du0)
    g_a = torch.empty_like(dal)
    plan.adjoint(g_uT.contiguous(), g_u0, g_a)
    torch.cuda.synchronize()
    uT_h, g_h, ga_h, guT_h = uT.cpu().numpy(), g_u0.cpu().numpy(), g_a.cpu().numpy(), g_uT.cpu().numpy()
    for b in range(batch):
        ref_uT = oracle.heat(u0[b], alpha[b], dt, dx, steps)
        assert np.array_equal(uT_h[b], ref_uT)
        J, g, ga = oracle.heat_adjoint(u0[b], y[b], alpha[b], dt, dx, steps)
        assert np.array_equal(g_h[b], g), f"grid {b}: max |dJ/du0 diff| {np.max(np.abs(g_h[b] - g))}"
        assert abs(ga_h[b] - ga) <= 1e-12 * abs(ga), (ga_h[b], ga)
        # dJ/du0 = A^steps g_uT: the forward naive kernel on g_uT, bit for bit
        p = Plan(n, "heat", torch.float64, dt, dx, alpha[b], tile_width=64)
        v = torch.tensor(guT_h[b], device="cuda")
        p.naive(v, steps)
        torch.cuda.synchronize()
        assert np.array_equal(v.cpu().numpy(), g_h[b])


def test_autograd_function_and_gradcheck():
    n, steps, batch = 64, 40, 2
    dx = 1.0 / n
    dt = dx * dx
    rng = np.random.default_rng(5)
    u0 = torch.tensor(rng.standard_normal((batch, n)), device="cuda", requires_grad=True)
    alpha = torch.tensor(rng.uniform(0.1, 0.4, size=batch), device="cuda", requires_grad=True)
    y = torch.tensor(rng.standard_normal((batch, n)), device="cuda")
    uT = swept_heat(u0, alpha, steps, dt, dx)
    J = 0.5 * ((uT - y) ** 2).sum()
    J.backward()
    for b in range(batch):
        Jb, g, ga = oracle.heat_adjoint(u0[b].detach().cpu().numpy(), y[b].cpu().numpy(),
                                        alpha[b].item(), dt, dx, steps)
        assert np.array_equal(u0.grad[b].cpu().numpy(), g)
        assert abs(alpha.grad[b].item() - ga) <= 1e-12 * abs(ga)
    f = lambda a, b: swept_heat(a, b, steps, dt, dx)
    assert torch.autograd.gradcheck(f, (u0.detach().requires_grad_(), alpha.detach().requires_grad_()),
                                    eps=1e-6, atol=1e-7, rtol=1e-6)


def test_adjoint_full_size_central_differences():
    # N = 2^18, T = 10^4 heat grids of the adjoint workload (two of its 64 grids)
    u0s, alpha, u0t, alpha_t, dt, dx, steps = inputs.heat_adjoint(batch=2)
    n = u0s.shape[1]
    # target from a perturbed forward run
    y = np.empty_like(u0t)
    for b in range(2):
        p = Plan(n, "heat", torch.float64, dt, dx, alpha_t[b], tile_width=1024)
        v = torch.tensor(u0t[b], device="cuda")
        p.run(v, steps)
        torch.cuda.synchronize()
        y[b] = v.cpu().numpy()
    plan = AdjointPlan(2, n, dt, dx, steps)
    du0 = torch.tensor(u0s, device="cuda")
    dal = torch.tensor(alpha, device="cuda")
    uT = torch.empty_like(du0)
    plan.forward(du0, dal, uT)
    dy = torch.tensor(y, device="cuda")
    g_u0 = torch.empty_like(du0)
    g_a = torch.empty_like(dal)
    plan.adjoint((uT - dy).contiguous(), g_u0, g_a)
    torch.cuda.synchronize()

    def J(b, u, a):
        p = Plan(n, "heat", torch.float64, dt, dx, a, tile_width=1024)
        v = torch.tensor(u, device="cuda")
        p.run(v, steps)
        torch.cuda.synchronize()
        return 0.5 * math.fsum(((v.cpu().numpy() - y[b]) ** 2).tolist())

    h = 1e-6   # step on alpha
    hu = 1e-2  # J is exactly quadratic in u0: a central difference has no truncation error,
    # and a larger step keeps the round-off of J (about 1e-11) far below the 1e-6 bar
    rng = np.random.default_rng(9)
    for b in range(2):
        fd = (J(b, u0s[b], alpha[b] + h) - J(b, u0s[b], alpha[b] - h)) / (2 * h)
        ga = g_a[b].item()
        print(f"grid {b}: dJ/dalpha swept {ga:.12e} central FD {fd:.12e} rel {abs(fd - ga) / abs(ga):.2e}")
        assert abs(fd - ga) <= 1e-6 * abs(ga), (b, fd, ga)
        # eight random unit directions per grid
        g = g_u0[b].cpu().numpy()
        for k in range(8):
            d = rng.standard_normal(n)
            d /= np.linalg.norm(d)
            fdu = (J(b, u0s[b] + hu * d, alpha[b]) - J(b, u0s[b] - hu * d, alpha[b])) / (2 * hu)
            gd = float(np.dot(g, d))
            print(f"grid {b} direction {k}: dJ/du0 . d swept {gd:.12e} central FD {fdu:.12e}")
            assert abs(fdu - gd) <= 1e-6 * max(abs(gd), 1e-12), (b, k, fdu, gd)


def test_autograd_plans_are_reused_and_never_shared():
    # two forwards awaiting their backwards hold two plans (no shared
    # checkpoints); after a backward the plan goes back to the pool and the
    # next forward of the same configuration takes it instead of allocating
    from paper_1612_02495_amd import swept as sw
    sw.release_cached_plans()
    n, steps, batch = 128, 70, 2
    dx = 1.0 / n
    dt = dx * dx
    rng = np.random.default_rng(11)
    a = torch.tensor(rng.uniform(0.1, 0.4, size=batch), device="cuda", requires_grad=True)
    ys = [torch.tensor(rng.standard_normal((batch, n)), device="cuda") for _ in range(2)]
    xs = [torch.tensor(rng.standard_normal((batch, n)), device="cuda", requires_grad=True) for _ in range(2)]
    Js = [0.5 * ((swept_heat(x, a, steps, dt, dx) - y) ** 2).sum() for x, y in zip(xs, ys)]
    assert not sw._FREE_PLANS or not any(sw._FREE_PLANS.values())
    for J in Js:
        J.backward()
    for x, y in zip(xs, ys):
        for b in range(batch):
            _, g, _ = oracle.heat_adjoint(x[b].detach().cpu().numpy(), y[b].cpu().numpy(), a[b].item(), dt, dx, steps)
            assert np.array_equal(x.grad[b].cpu().numpy(), g)
    pooled = [p for free in sw._FREE_PLANS.values() for p in free]
    assert len(pooled) == 1
    x = torch.tensor(rng.standard_normal((batch, n)), device="cuda", requires_grad=True)
    J = 0.5 * ((swept_heat(x, a.detach(), steps, dt, dx) - ys[0]) ** 2).sum()
    assert not any(sw._FREE_PLANS.values())  # the pooled plan was taken
    J.backward()
    assert [p for free in sw._FREE_PLANS.values() for p in free] == pooled
    # a second backward of a graph whose plan has since run another forward
    # recomputes its checkpoints (retain_graph): the same gradient
    x1 = torch.tensor(rng.standard_normal((batch, n)), device="cuda", requires_grad=True)
    J1 = 0.5 * ((swept_heat(x1, a.detach(), steps, dt, dx) - ys[0]) ** 2).sum()
    J1.backward(retain_graph=True)
    g_first = x1.grad.clone()
    x2 = torch.tensor(rng.standard_normal((batch, n)), device="cuda", requires_grad=True)
    J2 = 0.5 * ((swept_heat(x2, a.detach(), steps, dt, dx) - ys[1]) ** 2).sum()  # reuses J1's plan
    x1.grad = None
    J1.backward()
    assert torch.equal(x1.grad, g_first)
    J2.backward()
    sw.release_cached_plans()


# K = steps // 32 full phases; the first kept phase is K mod Q: 5, 1, 1, 0, 0
# (Q = 1), 0 and 5 in turn, the last two with segments of 4 and 6 phases
@pytest.mark.parametrize("segment,steps", [(0, 32 * 40 + 7), (3, 32 * 10), (5, 32 * 11 + 31), (2, 64), (7, 40),
                                           (4, 32 * 12 + 5), (6, 32 * 17)])
def test_two_level_checkpointing_gives_the_same_bits(segment, steps):
    # keeping every segment-th phase's edge state and recomputing the others
    # during the reverse sweep gives the gradients of the plan that keeps all
    # (bit for bit, dJ/dalpha included), and those equal the oracle's
    n, batch = 256, 2
    dx = 1.0 / n
    dt = dx * dx
    rng = np.random.default_rng(segment * 1000 + steps)
    alpha = rng.uniform(0.1, 0.4, size=batch)
    u0 = rng.standard_normal((batch, n))
    y = rng.standard_normal((batch, n))
    outs = []
    for seg in (1, segment):
        plan = AdjointPlan(batch, n, dt, dx, steps, segment=seg)
        du0 = torch.tensor(u0, device="cuda")
        uT = torch.empty_like(du0)
        plan.forward(du0, torch.tensor(alpha, device="cuda"), uT)
        g = torch.empty_like(du0)
        ga = torch.empty(batch, dtype=torch.float64, device="cuda")
        plan.adjoint((uT - torch.tensor(y, device="cuda")).contiguous(), g, ga)
        torch.cuda.synchronize()
        outs.append((uT.cpu().numpy(), g.cpu().numpy(), ga.cpu().numpy(), plan.info["checkpoint_bytes"]))
        plan.close()
    (u1, g1, a1, b1), (u2, g2, a2, b2) = outs
    assert np.array_equal(u1, u2) and np.array_equal(g1, g2) and np.array_equal(a1, a2)
    K = steps // 32
    if K > 2 and segment != 1:
        assert b2 < b1
    for b in range(batch):
        _, gref, garef = oracle.heat_adjoint(u0[b], y[b], alpha[b], dt, dx, steps)
        assert np.array_equal(g2[b], gref)
        assert abs(a2[b] - garef) <= 1e-12 * abs(garef)


def test_two_level_checkpoint_memory_of_the_gradient_workload():
    # 64 grids of 2^18 points over 10^4 steps: 312 phases; segments of 18
    # keep 17 + 17 sets instead of 312 (plan creation only, no run)
    from paper_1612_02495_amd.swept import swept_adjoint_create_segmented, swept_adjoint_destroy, swept_adjoint_info
    u0s, alpha, u0t, alpha_t, dt, dx, steps = inputs.heat_adjoint(batch=1)
    n = u0s.shape[1]
    h = swept_adjoint_create_segmented(64, n, "f64", dt, dx, steps, 0)
    info = swept_adjoint_info(h)
    swept_adjoint_destroy(h)
    per_set = 64 * 2 * (n // 64) * 66 * 8
    assert info["checkpoint_bytes"] == 34 * per_set
    assert info["checkpoint_bytes"] <= 10e9
