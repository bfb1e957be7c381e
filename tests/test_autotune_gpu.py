"""Autotuner on the GPU: it times real candidates, the winner drives a plan
created with tile_width = 0, and the tuned plan still matches naive bit for bit."""
import json

import numpy as np
import pytest

import paper_1612_02495_amd as P
from paper_1612_02495_amd import Plan

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,n", [("heat", 2 ** 14), ("ks", 2 ** 13)])
def test_autotune_picks_a_timed_candidate_and_plans_use_it(kind, n, tmp_path, monkeypatch):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("SWEPT_AUTOTUNE_CACHE", str(cache))
    P.swept_autotune_forget()
    dx, dt, alpha = (1.0 / n, 0.25 / n / n, 1.0) if kind == "heat" else (0.5, 0.005, 0.0)
    res = P.swept_autotune(n, kind, "f64", dt, dx, alpha, steps=256 if kind == "heat" else 64)
    cands = res["candidates"]
    assert len(cands) >= 4
    # every engine with a kernel for some candidate width is timed (n = 2^13,
    # 2^14 admit w = 512 and 1024, which the compacted engine covers)
    assert {c["engine"] for c in cands} == {"compact", "wave", "lds"}
    best = min(cands, key=lambda c: c["ns_per_cell_update"])
    assert (best["tile_width"], best["steps_per_cycle"], best["engine"]) == \
        (res["tile_width"], res["steps_per_cycle"], res["engine"])
    doc = json.loads(cache.read_text())
    assert any(e["n"] == n and e["tile_width"] == res["tile_width"] for e in doc["entries"])
    P.swept_autotune_forget()  # the plan below must find it in the file
    plan = Plan(n, kind, torch.float64, dt, dx, alpha)
    info = plan.info()
    assert info["tile_width"] == res["tile_width"] and info["steps_per_cycle"] == res["steps_per_cycle"]
    rng = np.random.default_rng(3)
    u0 = rng.standard_normal(n)
    a = torch.tensor(u0, device="cuda")
    b = torch.tensor(u0, device="cuda")
    plan.run(a, 300)
    plan.naive(b, 300)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    P.swept_autotune_forget()
