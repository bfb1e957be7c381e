"""Runs are asynchronous on the caller's stream and plans hold no shared
state: independent plans (and a batch) run at once on separate streams give
the bits of the same runs made one after another."""
import numpy as np
import pytest

from paper_1612_02495_amd import Batch, Plan, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _cases():
    h = inputs.heat_large(n=2 ** 16, steps=3000)
    k = inputs.ks(n=2 ** 16, steps=800)
    r = inputs.heat_rod(n=2 ** 14, steps=2000)
    return [(Plan(h.n, "heat", torch.float64, h.dt, h.dx, h.alpha, tile_width=1024), h.u0, h.steps),
            (Plan(k.n, "ks", torch.float64, k.dt, k.dx, tile_width=512), k.u0, k.steps),
            (Plan(r.n, "heat_insulated", torch.float64, r.dt, r.dx, r.alpha, tile_width=512), r.u0, r.steps)]


def test_plans_on_separate_streams_match_sequential():
    cases = _cases()
    seq = []
    for plan, u0, steps in cases:
        u = torch.tensor(u0, device="cuda")
        plan.run(u, steps)
        torch.cuda.synchronize()
        seq.append(u.cpu().numpy())
    streams = [torch.cuda.Stream() for _ in cases]
    outs = [torch.tensor(u0, device="cuda") for _, u0, _ in cases]
    torch.cuda.synchronize()
    for rep in range(2):  # the second pass reuses every plan's workspace while the others run
        for (plan, u0, steps), st, u in zip(cases, streams, outs):
            with torch.cuda.stream(st):
                u.copy_(torch.tensor(u0, device="cuda"))
                plan.run(u, steps, stream=st)
        torch.cuda.synchronize()
        for i, u in enumerate(outs):
            assert np.array_equal(u.cpu().numpy(), seq[i]), f"plan {i}, pass {rep}"


def test_batch_beside_plans_on_separate_streams():
    probs = inputs.ks_batch(nprob=64, steps=300)
    n = np.array([p.n for p in probs])
    b = Batch(n, "ks", torch.float64, [p.dt for p in probs], [p.dx for p in probs], [p.alpha for p in probs], 300)
    u0 = np.concatenate([p.u0 for p in probs])
    ref = torch.tensor(u0, device="cuda")
    b.run(ref)
    (plan, pu0, steps), = _cases()[:1]
    pref = torch.tensor(pu0, device="cuda")
    plan.run(pref, steps)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    x = torch.tensor(u0, device="cuda")
    y = torch.tensor(pu0, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        b.run(x, stream=s1)      # graph launch with its forked side branch
    with torch.cuda.stream(s2):
        plan.run(y, steps, stream=s2)
    torch.cuda.synchronize()
    assert torch.equal(x, ref)
    assert torch.equal(y, pref)
