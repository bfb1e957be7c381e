#!/usr/bin/env python3
"""Benchmark: swept vs naive cell-updates per second on one MI355X.

Default workload: periodic heat FTCS, N = 2^20 points, FP64, Fo = 1/4,
u0 = 8 seeded Fourier modes, one bench step = one swept_run advancing the grid
by 10^5 timesteps (inputs resident in HBM before the timed region).

Prints one JSON line with the swept throughput (`value`), the naive kernel's
throughput on the same workload, the roofline of the dominant kernel (the
diamond phase) and the CPU oracle's throughput on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload heat|heat_f32|heat_rod|ks|batch|batch_ks|adjoint|ks_adjoint]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-updates/sec, swept vs naive on 1 GPU (FP64 heat/KS); adjoint grad time"

# Algorithmic cost per cell update of one tier (IEEE adds/subtracts/multiplies
# in stencil.h; negation is a free source modifier):
#   heat: Fo*(r + l) + c*o                        -> 4
#   KS:   rhs 18 + (u + h*rhs) 2, per sub-step    -> 20  (two sub-steps per step)
FLOPS_PER_TIER_UPDATE = {"heat": 4, "heat_insulated": 4, "ks": 20}
TIERS_PER_STEP = {"heat": 1, "heat_insulated": 1, "ks": 2}
# Plain-ALU peak for add/mul-only code (no FMA: the bit-exact operation order
# has none; packed FP32 is disabled): 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2.4e9 / 1e12

WORKLOADS = {
    "heat": dict(kind="heat", dtype="f64", n=2 ** 20, horizon=100000, tile=0,
                 desc="heat FTCS periodic, N=2^20, FP64, Fo=1/4, 8-mode u0, 1e5 steps per run"),
    "heat_f32": dict(kind="heat", dtype="f32", n=2 ** 20, horizon=100000, tile=0,
                     desc="heat FTCS periodic, N=2^20, FP32, Fo=1/4, 8-mode u0, 1e5 steps per run"),
    "heat_rod": dict(kind="heat_insulated", dtype="f64", n=2 ** 20, horizon=100000, tile=0,
                     desc="heat FTCS on a rod with insulated ends (Sec. 4.1), N=2^20 nodes, FP64, Fo=1/4, "
                          "temperature gradient plus 8 cosine modes, 1e5 steps per run"),
    "ks": dict(kind="ks", dtype="f64", n=2 ** 20, horizon=20000, tile=0,
               desc="Kuramoto-Sivashinsky RK2 periodic, N=2^20, FP64, dx=0.5, dt=0.005, 2e4 steps per run"),
    "batch": dict(kind="heat", dtype="f64", n=0, horizon=5000, tile=0, batch=4096,
                  desc="4096 independent periodic heat FTCS grids, N log-uniform in [2^8,2^16] "
                       "(multiples of 16), Fo ~ U(0.05,0.45), FP64, 5000 steps, one persistent "
                       "kernel per graph launch"),
    "batch_ks": dict(kind="ks", dtype="f64", n=0, horizon=5000, tile=0, batch=4096,
                     desc="4096 independent periodic KS grids, N log-uniform in [2^8,2^16] "
                          "(multiples of 16), dx=0.5, dt=0.005, FP64, 5000 steps, one persistent "
                          "kernel per graph launch"),
    "adjoint": dict(kind="heat", dtype="f64", n=2 ** 18, horizon=10000, tile=64, adjoint=64,
                    desc="gradient of J = 1/2 ||u_T - y||^2 w.r.t. u0 and alpha for 64 periodic heat "
                         "FTCS grids, N=2^18, FP64, 1e4 steps: checkpointed swept forward + swept "
                         "adjoint (one bench step = forward + reverse)"),
    "ks_adjoint": dict(kind="ks", dtype="f64", n=2 ** 20, horizon=20000, tile=64, adjoint=1,
                       desc="gradient of J = 1/2 ||u_T - y||^2 w.r.t. u0 for one periodic Kuramoto-"
                            "Sivashinsky grid, N=2^20, FP64, dx=0.5, dt=0.005, 2e4 RK2 steps: checkpointed "
                            "swept forward + swept adjoint (one bench step = forward + reverse)"),
}


def run_adjoint(args, wl):
    """Adjoint workload: one bench step = swept_forward_ckpt + swept_adjoint_run."""
    import numpy as np
    import torch

    from paper_1612_02495_amd import AdjointPlan, inputs
    B = args.batch or wl["adjoint"]
    T = wl["horizon"]
    u0, alpha, u0t, alpha_t, dt, dx, _ = inputs.heat_adjoint(batch=B, n=wl["n"], steps=T)
    n = u0.shape[1]
    plan = AdjointPlan(B, n, dt, dx, T)
    du0 = torch.tensor(u0, device="cuda")
    dal = torch.tensor(alpha, device="cuda")
    # the target: a forward run from the perturbed initial states and alphas
    y = torch.empty_like(du0)
    plan.forward(torch.tensor(u0t, device="cuda"), torch.tensor(alpha_t, device="cuda"), y)
    uT = torch.empty_like(du0)
    g_u0 = torch.empty_like(du0)
    g_a = torch.empty_like(dal)

    def step():
        plan.forward(du0, dal, uT)
        g = uT - y
        plan.adjoint(g, g_u0, g_a)

    for _ in range(args.warmup):
        step()
    t = _time_runs(step, args.steps, torch)
    t_fwd = _time_runs(lambda: plan.forward(du0, dal, uT), args.steps, torch)
    updates = B * n * T * args.steps

    # Dominant kernel: the fused reverse region launch (recompute, lambda walk,
    # dJ/dalpha terms).  Its time per launch is the difference of two reverse
    # sweeps whose horizons differ by D full phases (same remainder), timed
    # with events on the launch stream.  Algorithmic flops per launch: every
    # tile's region holds w h = 2048 cell-updates, each recomputed (4 flops),
    # walked by lambda (4 flops) and paired with its Laplacian term
    # ((ul + ur) - 2 u: 3 flops, times lambda and accumulated: 2).
    roof = None
    if not args.no_dominant:
        h = plan.info["steps_per_cycle"]
        r = plan.info["leading_classic_steps"]
        k_lo, k_hi = 8, 40
        times = {}
        for kk in (k_lo, k_hi):
            pk = AdjointPlan(B, n, dt, dx, kk * h + r)
            uk = torch.empty_like(du0)
            pk.forward(du0, dal, uk)
            gk = uk - y
            pk.adjoint(gk, g_u0, g_a)  # warm-up
            times[kk] = _time_runs(lambda: pk.adjoint(gk, g_u0, g_a), 3, torch) / 3
            pk.close()
            del uk, gk
        t_launch = (times[k_hi] - times[k_lo]) / (k_hi - k_lo)
        w = plan.info["tile_width"]
        flops = B * (n // w) * w * h * (4 + 4 + 5)
        achieved = flops / t_launch / 1e12
        roof = {"bound": "alu", "kernel": "fused reverse region launch (recompute + lambda + dJ/dalpha)",
                "achieved": achieved, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / ALU_PEAK_TFLOPS,
                "traffic": None, "launch_ms": 1e3 * t_launch, "flops_per_launch": flops}
    cpu = None
    if not args.no_cpu_baseline:
        import time as _time
        import oracle
        cs = args.cpu_steps or 4000
        t0 = _time.perf_counter()
        oracle.heat_adjoint(u0[0], u0t[0], alpha[0], dt, dx, cs)
        el = _time.perf_counter() - t0
        cpu = {"value": n * cs / el, "unit": "cell-updates/s of gradient (forward + reverse)", "cores": 1,
               "kind": "oracle", "sample": f"one of the {B} grids, {cs} of the {T} steps, single-thread C "
                                           f"checkpointed reverse sweep, {el:.1f} s",
               "host_cpu": host_cpu_model()}
    return {
        "metric": METRIC, "value": updates / t, "unit": "cell-updates/s of gradient (forward + reverse)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded; see paper_1612_02495_amd/inputs.py)",
        "config": {"workload": wl["desc"], "batch": B, "n": n, "timesteps": T,
                   "adjoint_grad_ms": 1e3 * t / args.steps, "forward_ckpt_ms": 1e3 * t_fwd / args.steps,
                   "checkpoint_bytes": plan.info["checkpoint_bytes"],
                   "tile_width": plan.info["tile_width"], "steps_per_cycle": plan.info["steps_per_cycle"],
                   "leading_classic_steps": plan.info["leading_classic_steps"], "parallelism": "single GPU"},
        "roofline": roof, "naive": None, "speedup_vs_naive": None, "cpu_baseline": cpu,
    }


def run_ks_adjoint(args, wl):
    """KS adjoint workload: one bench step = swept_ks_forward_ckpt + swept_ks_adjoint_run."""
    import torch

    from paper_1612_02495_amd import KsAdjointPlan, inputs
    B = args.batch or wl["adjoint"]
    T = wl["horizon"]
    u0, u0t, dt, dx, _ = inputs.ks_adjoint(batch=B, n=wl["n"], steps=T)
    n = u0.shape[1]
    plan = KsAdjointPlan(B, n, dt, dx, T)
    du0 = torch.tensor(u0, device="cuda")
    # the target: a forward run from the perturbed initial states
    y = torch.empty_like(du0)
    plan.forward(torch.tensor(u0t, device="cuda"), y)
    uT = torch.empty_like(du0)
    g_u0 = torch.empty_like(du0)

    def step():
        plan.forward(du0, uT)
        plan.adjoint((uT - y).contiguous(), g_u0)

    for _ in range(args.warmup):
        step()
    t = _time_runs(step, args.steps, torch)
    t_fwd = _time_runs(lambda: plan.forward(du0, uT), args.steps, torch)
    updates = B * n * T * args.steps

    # Dominant kernel: the fused reverse region launch.  Its time per launch is
    # the difference of two reverse sweeps whose horizons differ by D full
    # phases (same remainder), timed with events on the launch stream.
    # Algorithmic flops per launch: every tile's region holds w h = 1024
    # sub-step updates, each recomputed (20 flops) and walked back by the
    # adjoint: Jf^T w costs 13 (2 for the nonlinear weight, 2 for the two
    # neighbour weights, 5 products and 4 sums), plus 1 (dt mu, odd tiers) or 3
    # ((lambda'' + mu) + dt/2 Jf^T mu, even tiers): 35 per update on average.
    roof = None
    if not args.no_dominant:
        h = plan.info["steps_per_cycle"]
        r = plan.info["leading_classic_steps"]
        k_lo, k_hi = 8, 40
        times = {}
        for kk in (k_lo, k_hi):
            pk = KsAdjointPlan(B, n, dt, dx, kk * h + r)
            uk = torch.empty_like(du0)
            pk.forward(du0, uk)
            gk = (uk - y).contiguous()
            pk.adjoint(gk, g_u0)  # warm-up
            times[kk] = _time_runs(lambda: pk.adjoint(gk, g_u0), 3, torch) / 3
            pk.close()
            del uk, gk
        t_launch = (times[k_hi] - times[k_lo]) / (k_hi - k_lo)
        w = plan.info["tile_width"]
        tiers = 2 * h
        flops = B * (n // w) * w * tiers * (20 + 15)
        achieved = flops / t_launch / 1e12
        roof = {"bound": "alu", "kernel": "fused reverse region launch (recompute + adjoint walk)",
                "achieved": achieved, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / ALU_PEAK_TFLOPS,
                "traffic": None, "launch_ms": 1e3 * t_launch, "flops_per_launch": flops}
    cpu = None
    if not args.no_cpu_baseline:
        import time as _time
        import oracle
        cs = args.cpu_steps or 400
        t0 = _time.perf_counter()
        oracle.ks_adjoint(u0[0], u0t[0], dt, dx, cs)
        el = _time.perf_counter() - t0
        cpu = {"value": n * cs / el, "unit": "cell-updates/s of gradient (forward + reverse)", "cores": 1,
               "kind": "oracle", "sample": f"grid 0 of {B}, {cs} of the {T} steps, single-thread C "
                                           f"checkpointed reverse sweep, {el:.1f} s",
               "host_cpu": host_cpu_model()}
    return {
        "metric": METRIC, "value": updates / t, "unit": "cell-updates/s of gradient (forward + reverse)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded; see paper_1612_02495_amd/inputs.py)",
        "config": {"workload": wl["desc"], "batch": B, "n": n, "timesteps": T,
                   "adjoint_grad_ms": 1e3 * t / args.steps, "forward_ckpt_ms": 1e3 * t_fwd / args.steps,
                   "checkpoint_bytes": plan.info["checkpoint_bytes"],
                   "tile_width": plan.info["tile_width"], "steps_per_cycle": plan.info["steps_per_cycle"],
                   "leading_classic_steps": plan.info["leading_classic_steps"], "parallelism": "single GPU"},
        "roofline": roof, "naive": None, "speedup_vs_naive": None, "cpu_baseline": cpu,
    }


def run_batch(args, wl):
    """Batched workload: one bench step = one graph launch of the persistent kernel."""
    import numpy as np
    import torch

    from paper_1612_02495_amd import Batch, inputs
    T = wl["horizon"]
    probs = (inputs.heat_batch(nprob=wl["batch"], steps=T) if wl["kind"] == "heat"
             else inputs.ks_batch(nprob=wl["batch"], steps=T))
    n = np.array([p.n for p in probs])
    b = Batch(n, wl["kind"], wl["dtype"], [p.dt for p in probs], [p.dx for p in probs],
              [p.alpha for p in probs], T)
    engine = args.engine  # AUTO: small grids whole in the resident kernels, the rest compacted swept tiles
    b.set_engine(engine)
    u = torch.tensor(np.concatenate([p.u0 for p in probs]), device="cuda")
    for _ in range(args.warmup):
        b.run(u)
    t = _time_runs(lambda: b.run(u), args.steps, torch)
    updates = int(n.sum()) * T * args.steps
    tiers = TIERS_PER_STEP[wl["kind"]]
    flops = FLOPS_PER_TIER_UPDATE[wl["kind"]] * int(n.sum()) * T * tiers
    achieved = flops / (t / args.steps) / 1e12
    cpu = None
    if not args.no_cpu_baseline:
        import time as _time
        import oracle
        budget = min(T, args.cpu_steps or (5000 if wl["kind"] == "heat" else 1000))
        big = max(probs, key=lambda p: p.n)
        t0 = _time.perf_counter()
        for p in probs[:64]:
            if wl["kind"] == "heat":
                oracle.heat(p.u0, p.alpha, p.dt, p.dx, budget)
            else:
                oracle.ks(p.u0, p.dt, p.dx, budget)
        el = _time.perf_counter() - t0
        cells = sum(p.n for p in probs[:64]) * budget
        cpu = {"value": cells / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
               "sample": f"first 64 of the {len(probs)} grids, {budget} of the {T} steps each "
                         f"(largest grid in batch n={big.n}), single-thread C oracle, {el:.1f} s",
               "host_cpu": host_cpu_model()}
    return {
        "metric": METRIC, "value": updates / t, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": wl["dtype"],
        "data": "synthetic (seeded; see paper_1612_02495_amd/inputs.py)",
        "config": {"workload": wl["desc"], "grids": int(n.size), "total_points": int(n.sum()),
                   "timesteps_per_run": T, "kind": wl["kind"], "engine": engine, "persistent_grid": b.grid,
                   "edge_slot_bytes": b.workspace_bytes, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": "batched persistent swept kernel (whole launch)",
                     "achieved": achieved, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / ALU_PEAK_TFLOPS, "traffic": None,
                     "launch_ms": 1e3 * t / args.steps, "flops_per_launch": flops},
        "naive": None, "speedup_vs_naive": None, "cpu_baseline": cpu,
    }


CSRC = "paper_1612_02495_amd/csrc/"
# Per engine: the sources that define its diamond kernel; per (kind, dtype,
# engine): the committed rocprofv3 counter summary of the N=2^20 w=1024 workload.
KERNEL_SOURCES = {
    "wave": [CSRC + "phase_wave.hip", CSRC + "stencil.h", CSRC + "internal.h"],
    "compact": [CSRC + "phase_compact.hip", CSRC + "compact_tile.h", CSRC + "wave_tile.h", CSRC + "stencil.h",
                CSRC + "internal.h"],
}
TRAFFIC_SUMMARY = {
    ("heat", "f64", "wave"): "profiles/phase_wave_heat_f64_n2p20_w1024_pmc.md",
    ("heat", "f64", "compact"): "profiles/phase_compact_heat_f64_n2p20_w1024_pmc.md",
    ("heat", "f32", "compact"): "profiles/phase_compact_heat_f32_n2p20_w1024_pmc.md",
    ("heat_insulated", "f64", "compact"): "profiles/phase_compact_heat_insulated_f64_n2p20_w1024_pmc.md",
    ("ks", "f64", "compact"): "profiles/phase_compact_ks_f64_n2p20_w1024_pmc.md",
}


def _traffic_from_profile(wl, tile, engine):
    """Calibrated HBM bytes per diamond launch from the committed rocprofv3
    counter summary -- only if it covers this workload and the kernel source
    has not changed since the counters were taken; otherwise None."""
    import hashlib
    if engine == "auto":  # the library's AUTO choice for these widths
        engine = "compact" if tile in (512, 1024) else "wave"
    key = (wl["kind"], wl["dtype"], engine)
    if not (wl["n"] == 2 ** 20 and tile == 1024 and key in TRAFFIC_SUMMARY):
        return None
    path = os.path.join(ROOT, TRAFFIC_SUMMARY[key])
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", "|", "`")):
            k, _, v = line.partition(":")
            fields[k.strip()] = v.strip()
    src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in KERNEL_SOURCES[engine])
    if fields.get("source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _problem(wl):
    from paper_1612_02495_amd import inputs
    if wl["kind"] == "heat":
        return inputs.heat_large(n=wl["n"], steps=wl["horizon"])
    if wl["kind"] == "heat_insulated":
        return inputs.heat_rod(n=wl["n"], steps=wl["horizon"])
    return inputs.ks(n=wl["n"], steps=wl["horizon"])


def _time_runs(fn, reps, torch):
    """Median-free total: events bracket `reps` calls on the current stream."""
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        fn()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / 1e3  # seconds


def _naive_graph_rate(plan, v, steps, reps, torch):
    """Seconds per timestep of the naive run replayed from a captured graph of
    `steps` timesteps (one kernel node per step or sub-step), which takes the
    host's launch cost out of the naive kernel's time."""
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=side):
        plan.naive(v, steps)
    g.replay()
    t = _time_runs(g.replay, reps, torch)
    del g
    return t / (reps * steps)


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(wl, budget_steps):
    import numpy as np

    import oracle
    p = _problem(wl)
    t0 = time.perf_counter()
    if wl["kind"] == "heat":
        oracle.heat(p.u0, p.alpha, p.dt, p.dx, budget_steps,
                    dtype=np.float64 if wl["dtype"] == "f64" else np.float32)
    elif wl["kind"] == "heat_insulated":
        oracle.heat_insulated(p.u0, p.alpha, p.dt, p.dx, budget_steps,
                              dtype=np.float64 if wl["dtype"] == "f64" else np.float32)
    else:
        oracle.ks(p.u0, p.dt, p.dx, budget_steps, dtype=np.float64 if wl["dtype"] == "f64" else np.float32)
    el = time.perf_counter() - t0
    return {"value": p.n * budget_steps / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{wl['kind']} N={p.n} {wl['dtype']}, {budget_steps} of the {wl['horizon']} steps, "
                      f"single-thread C oracle, {el:.1f} s",
            "host_cpu": host_cpu_model()}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed bench steps (swept runs)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="heat", choices=sorted(WORKLOADS))
    ap.add_argument("--engine", default="auto", choices=["auto", "lds", "wave", "compact", "resident"],
                    help="phase engine; 'resident' is for the batched workloads only")
    ap.add_argument("--tile", type=int, default=0,
                    help="tile width (0 = run the autotuner and use its choice)")
    ap.add_argument("--horizon", type=int, default=0, help="timesteps per run (0 = workload default)")
    ap.add_argument("--naive-steps", type=int, default=0, help="timed naive runs (0 = same as --steps)")
    ap.add_argument("--no-naive", action="store_true")
    ap.add_argument("--no-naive-graph", action="store_true",
                    help="skip the graph-replayed naive timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=0, help="oracle timesteps in the CPU sample")
    ap.add_argument("--no-dominant", action="store_true",
                    help="skip the per-launch timing of the diamond kernel (short profiler passes)")
    ap.add_argument("--batch", type=int, default=0, help="grids in the adjoint workloads (0 = 64 heat, 1 KS)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of MIB mebibytes (counter calibration)")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the swept path here is a single-GPU build "
              "(multi-GPU sharding is a design note only); run with --gpus 1.", file=sys.stderr)
        return 2

    import torch

    from paper_1612_02495_amd import Plan

    wl = dict(WORKLOADS[args.workload])
    if args.horizon:
        wl["horizon"] = args.horizon
    if wl.get("batch"):
        print(json.dumps(run_batch(args, wl)))
        return 0
    if wl.get("adjoint"):
        print(json.dumps(run_ks_adjoint(args, wl) if wl["kind"] == "ks" else run_adjoint(args, wl)))
        return 0
    tile = args.tile or wl["tile"]
    p = _problem(wl)
    tdtype = torch.float64 if wl["dtype"] == "f64" else torch.float32
    tuned = None
    if tile == 0:
        # untimed plan setup: search tile width, phase height and engine on the real kernels
        from paper_1612_02495_amd import swept_autotune
        tuned = swept_autotune(p.n, wl["kind"], wl["dtype"], p.dt, p.dx, p.alpha)
        plan = Plan(p.n, wl["kind"], tdtype, p.dt, p.dx, p.alpha, tile_width=tuned["tile_width"],
                    steps_per_cycle=tuned["steps_per_cycle"], engine=tuned["engine"])
        args.engine = tuned["engine"]
    else:
        plan = Plan(p.n, wl["kind"], tdtype, p.dt, p.dx, p.alpha, tile_width=tile, engine=args.engine)
    info = plan.info()
    T = wl["horizon"]
    u = torch.tensor(p.u0, dtype=tdtype, device="cuda")

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        plan.run(u, T)
    t_swept = _time_runs(lambda: plan.run(u, T), args.steps, torch)
    updates = p.n * T * args.steps
    value = updates / t_swept

    # Dominant kernel (diamond phase): difference of two runs that differ only
    # in their number of full diamonds, timed with events on the launch stream.
    spc = info["steps_per_cycle"]
    tiers = spc * TIERS_PER_STEP[wl["kind"]]
    flops = FLOPS_PER_TIER_UPDATE[wl["kind"]] * p.n * tiers
    t_diamond = None
    achieved = None
    if not args.no_dominant:
        d_lo, d_hi = 1, 21

        def run_d(d):
            return lambda: plan.run(u, spc * (d + 1))
        samples = []
        for _ in range(3):
            a = _time_runs(run_d(d_lo), 2, torch) / 2
            b = _time_runs(run_d(d_hi), 2, torch) / 2
            samples.append((b - a) / (d_hi - d_lo))
        t_diamond = statistics.median(samples)
        achieved = flops / t_diamond / 1e12

    naive = None
    if not args.no_naive:
        k_naive = args.naive_steps or args.steps
        v = torch.tensor(p.u0, dtype=tdtype, device="cuda")
        plan.naive(v, min(T, 100))
        t_naive = _time_runs(lambda: plan.naive(v, T), k_naive, torch)
        bytes_per_update = (40 if wl["kind"] == "ks" else 16) // (1 if wl["dtype"] == "f64" else 2)
        naive = {"value": p.n * T * k_naive / t_naive, "ms_per_step": 1e3 * t_naive / k_naive,
                 "ms_per_timestep": 1e3 * t_naive / (k_naive * T),
                 "hbm_bound": {"bytes_per_cell_update": bytes_per_update,
                               "achieved_GBps": bytes_per_update * p.n * T * k_naive / t_naive / 1e9,
                               "peak_GBps": 8000.0}}
        if not args.no_naive_graph:
            g_steps = min(T, 1000)
            per_step = _naive_graph_rate(plan, v, g_steps, 5, torch)
            naive["graph"] = {"value": p.n / per_step, "ms_per_timestep": 1e3 * per_step,
                              "achieved_GBps": bytes_per_update * p.n / per_step / 1e9,
                              "captured_timesteps": g_steps}

    cpu = None
    if not args.no_cpu_baseline:
        budget = args.cpu_steps or (300 if wl["kind"] == "ks" else 4000)
        cpu = cpu_baseline(wl, budget)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_swept / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": wl["dtype"],
        "data": "synthetic (seeded; see paper_1612_02495_amd/inputs.py)",
        "config": {"workload": wl["desc"], "n": p.n, "timesteps_per_run": T, "kind": wl["kind"],
                   "tile_width": info["tile_width"], "steps_per_cycle": spc, "engine": args.engine,
                   "parallelism": "single GPU",
                   "autotune": None if tuned is None else sorted(
                       ({"w": c["tile_width"], "spc": c["steps_per_cycle"], "engine": c["engine"],
                         "ns_per_update": round(c["ns_per_cell_update"], 6)} for c in tuned["candidates"]),
                       key=lambda c: c["ns_per_update"])},
        "roofline": {"bound": "alu", "kernel": "swept diamond phase", "achieved": achieved,
                     "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": (achieved / ALU_PEAK_TFLOPS) if achieved else None,
                     "traffic": _traffic_from_profile(wl, info["tile_width"], args.engine),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
                     "launch_ms": (1e3 * t_diamond) if t_diamond else None,
                     "flops_per_launch": flops},
        "naive": naive,
        "speedup_vs_naive": (value / naive["value"]) if naive else None,
        "speedup_vs_naive_graph": (value / naive["graph"]["value"]) if naive and "graph" in naive else None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
