#!/usr/bin/env python3
"""Benchmark: swept vs naive cell-updates per second on one MI355X.

Default workload: periodic heat FTCS, N = 2^20 points, FP64, Fo = 1/4,
u0 = 8 seeded Fourier modes, one bench step = one swept_run advancing the grid
by 10^5 timesteps (inputs resident in HBM before the timed region).  The same
run then measures the rest of the metric as nested records under
"workloads": KS at N = 2^20 over 2*10^4 steps, the batched heat and KS
workloads (4096 grids each) and the heat and KS gradient times.

Every record carries the roofline of its dominant kernel (achieved FLOP/s
against MI355X's published vector peak for its dtype, and against the
vector issue rate times the kernel's flops per floating-point instruction,
what its operation order can reach) and the CPU oracle's throughput on a
bounded sample, single-threaded and on all host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload heat|heat_f32|heat_rod|ks|batch|batch_ks|adjoint|ks_adjoint|sweep]
                    [--no-nested]
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

# Algorithmic cost per cell update of one tier, the operations of the
# discretisation as written in Sec. 4.1 (heat: Fo (r + l) + (1 - 2 Fo) o;
# KS: the 5-point right-hand side, 18, and the RK2 stage u + h f, 2), and the
# floating-point instructions that carry it in stencil.h's order (a fused
# multiply-add is one instruction; negation is a free source modifier):
#   heat: fma(Fo, r + l, c*o)                                   -> 4 flops in 3 instructions
#   KS:   u - h g, h g from S1, S2, the flux and two fmas       -> 20 in 11  (two sub-steps per step)
FLOPS_PER_TIER_UPDATE = {"heat": 4, "heat_insulated": 4, "ks": 20}
FP_INSTR_PER_TIER_UPDATE = {"heat": 3, "heat_insulated": 3, "ks": 11}
TIERS_PER_STEP = {"heat": 1, "heat_insulated": 1, "ks": 2}
# MI355X's published dense vector peaks (an FMA counts as two operations).
PUBLISHED_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
# Vector instruction issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one
# lane-instruction per lane per clock (packed FP32 is disabled).  A kernel
# whose operation order carries f flops in i instructions can reach at most
# this rate times f / i.
ALU_ISSUE_TERA = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBPS = 8000.0

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
                  desc="4096 independent periodic heat FTCS grids, N = round(2^U(8,16)), Fo ~ U(0.05,0.45), "
                       "FP64, 5000 steps, one graph launch"),
    "batch_ks": dict(kind="ks", dtype="f64", n=0, horizon=5000, tile=0, batch=4096,
                     desc="4096 independent periodic KS grids, N = round(2^U(8,16)), dx=0.5, dt=0.005, FP64, "
                          "5000 steps, one graph launch"),
    "adjoint": dict(kind="heat", dtype="f64", n=2 ** 18, horizon=10000, tile=64, adjoint=64,
                    desc="gradient of J = 1/2 ||u_T - y||^2 w.r.t. u0 and alpha for 64 periodic heat "
                         "FTCS grids, N=2^18, FP64, 1e4 steps: checkpointed swept forward + swept "
                         "adjoint (one bench step = forward + reverse)"),
    "ks_adjoint": dict(kind="ks", dtype="f64", n=2 ** 20, horizon=20000, tile=64, adjoint=1,
                       desc="gradient of J = 1/2 ||u_T - y||^2 w.r.t. u0 for one periodic Kuramoto-"
                            "Sivashinsky grid, N=2^20, FP64, dx=0.5, dt=0.005, 2e4 RK2 steps: checkpointed "
                            "swept forward + swept adjoint (one bench step = forward + reverse)"),
}
# measured beside the default heat line, in this order
NESTED = ["ks", "batch", "batch_ks", "adjoint", "ks_adjoint"]
DATA = "synthetic (seeded; see paper_1612_02495_amd/inputs.py)"


def roofline(kernel, flops, t_launch, dtype, traffic=None, fp_instr=None):
    """ALU roofline of one kernel launch: algorithmic flops / launch time.
    fp_instr: the floating-point instructions (lane-instructions) that carry
    those flops in the kernel's operation order; sets the issue-rate ceiling."""
    achieved = flops / t_launch / 1e12
    peak = PUBLISHED_PEAK_TFLOPS[dtype]
    issue = ALU_ISSUE_TERA * flops / (fp_instr if fp_instr else flops)
    return {"bound": "alu", "kernel": kernel, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "launch_ms": 1e3 * t_launch, "flops_per_launch": flops,
            "issue_peak": issue, "frac_of_issue_peak": achieved / issue,
            "issue_peak_note": "one floating-point lane-instruction per lane per clock at 2.4 GHz, times "
                               "this kernel's flops per instruction (an FMA carries two)"}


def host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": affinity,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def host_cpu_model():
    return host_info()["cpu_model"]


def _timed(fn):
    t0 = time.perf_counter()
    out = fn()
    return time.perf_counter() - t0, out


def cpu_legs(single, multi=None, unit="cell-updates/s"):
    """The CPU oracle timed on a bounded sample: `single` = (callable, updates,
    description) on one thread; `multi` = (callable returning the thread count,
    updates, description) on all host cores, or None."""
    fn, upd, desc = single
    el, _ = _timed(fn)
    st = {"value": upd / el, "unit": unit, "cores": 1, "sample": f"{desc}, {el:.1f} s"}
    out = {"value": st["value"], "unit": unit, "cores": 1, "kind": "oracle", "sample": st["sample"],
           "single_thread": st, "host": host_info()}
    if multi is not None:
        fn, upd, desc = multi
        el, threads = _timed(fn)
        out.update({"value": upd / el, "cores": threads,
                    "sample": f"{desc}, {threads} threads (OpenMP over each step's points; same bits as one "
                              f"thread), {el:.1f} s"})
    return out


def _time_runs(fn, reps, torch):
    """Seconds for `reps` calls, bracketed by events on the current stream."""
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        fn()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / 1e3


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


CSRC = "paper_1612_02495_amd/csrc/"
# Per engine: the sources that define its diamond kernel; per (kind, dtype,
# engine): the committed rocprofv3 counter summary of the N=2^20 w=1024 workload.
KERNEL_SOURCES = {
    "wave": [CSRC + "phase_wave.hip", CSRC + "wave_tile.h", CSRC + "stencil.h", CSRC + "internal.h"],
    "compact": [CSRC + "phase_compact.hip", CSRC + "compact_tile.h", CSRC + "wave_tile.h", CSRC + "stencil.h",
                CSRC + "internal.h", CSRC + "poison.h"],
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


def _problem(kind, n, horizon):
    from paper_1612_02495_amd import inputs
    if kind == "heat":
        return inputs.heat_large(n=n, steps=horizon)
    if kind == "heat_insulated":
        return inputs.heat_rod(n=n, steps=horizon)
    return inputs.ks(n=n, steps=horizon)


def single_cpu_baseline(wl, p, args):
    """Oracle on the workload's own grid: a few of its steps on one thread and
    more on all host cores (heat and KS in FP64; the others single-thread)."""
    import numpy as np

    import oracle
    kind, dtype = wl["kind"], wl["dtype"]
    st_steps = args.cpu_steps or (100 if kind == "ks" else 2000)
    np_dtype = np.float64 if dtype == "f64" else np.float32
    if kind == "heat":
        single = (lambda: oracle.heat(p.u0, p.alpha, p.dt, p.dx, st_steps, dtype=np_dtype), p.n * st_steps,
                  f"heat N={p.n} {dtype}, {st_steps} of the {wl['horizon']} steps, single-thread C oracle")
    elif kind == "heat_insulated":
        single = (lambda: oracle.heat_insulated(p.u0, p.alpha, p.dt, p.dx, st_steps, dtype=np_dtype),
                  p.n * st_steps, f"insulated rod N={p.n} {dtype}, {st_steps} of the {wl['horizon']} steps, "
                                  f"single-thread C oracle")
    else:
        single = (lambda: oracle.ks(p.u0, p.dt, p.dx, st_steps, dtype=np_dtype), p.n * st_steps,
                  f"KS N={p.n} {dtype}, {st_steps} of the {wl['horizon']} steps, single-thread C oracle")
    multi = None
    if dtype == "f64" and kind in ("heat", "ks"):
        mt_steps = 8 * st_steps
        if kind == "heat":
            multi = (lambda: oracle.heat_mt(p.u0, p.alpha, p.dt, p.dx, mt_steps)[1], p.n * mt_steps,
                     f"heat N={p.n} f64, {mt_steps} of the {wl['horizon']} steps, C oracle")
        else:
            multi = (lambda: oracle.ks_mt(p.u0, p.dt, p.dx, mt_steps)[1], p.n * mt_steps,
                     f"KS N={p.n} f64, {mt_steps} of the {wl['horizon']} steps, C oracle")
    return cpu_legs(single, multi)


def run_single(args, wl, tile=0, engine="auto", want_naive=True, want_cpu=True):
    """One grid: one bench step = one swept_run over the workload's horizon."""
    import torch

    from paper_1612_02495_amd import Plan, swept_autotune
    p = _problem(wl["kind"], wl["n"], wl["horizon"])
    tdtype = torch.float64 if wl["dtype"] == "f64" else torch.float32
    tuned = None
    if tile == 0:
        # untimed plan setup: search tile width, phase height and engine on the real kernels
        tuned = swept_autotune(p.n, wl["kind"], wl["dtype"], p.dt, p.dx, p.alpha)
        plan = Plan(p.n, wl["kind"], tdtype, p.dt, p.dx, p.alpha, tile_width=tuned["tile_width"],
                    steps_per_cycle=tuned["steps_per_cycle"], engine=tuned["engine"])
        engine = tuned["engine"]
    else:
        plan = Plan(p.n, wl["kind"], tdtype, p.dt, p.dx, p.alpha, tile_width=tile, engine=engine)
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
    value = p.n * T * args.steps / t_swept

    # Dominant kernel (diamond phase): difference of two runs that differ only
    # in their number of full diamonds, timed with events on the launch stream.
    spc = info["steps_per_cycle"]
    tiers = spc * TIERS_PER_STEP[wl["kind"]]
    flops = FLOPS_PER_TIER_UPDATE[wl["kind"]] * p.n * tiers
    instr = FP_INSTR_PER_TIER_UPDATE[wl["kind"]] * p.n * tiers
    roof = None
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
        roof = roofline("swept diamond phase", flops, t_diamond, wl["dtype"],
                        _traffic_from_profile(wl, info["tile_width"], engine), fp_instr=instr)
        # a full run's phases: one up, the diamonds, one down
        roof["diamonds_per_run"] = -(-T * TIERS_PER_STEP[wl["kind"]] // tiers) - 1

    naive = None
    if want_naive and not args.no_naive:
        k_naive = args.naive_steps or args.steps
        v = torch.tensor(p.u0, dtype=tdtype, device="cuda")
        plan.naive(v, min(T, 100))
        t_naive = _time_runs(lambda: plan.naive(v, T), k_naive, torch)
        bytes_per_update = (40 if wl["kind"] == "ks" else 16) // (1 if wl["dtype"] == "f64" else 2)
        naive = {"value": p.n * T * k_naive / t_naive, "ms_per_step": 1e3 * t_naive / k_naive,
                 "ms_per_timestep": 1e3 * t_naive / (k_naive * T),
                 "hbm_bound": {"bytes_per_cell_update": bytes_per_update,
                               "achieved_GBps": bytes_per_update * p.n * T * k_naive / t_naive / 1e9,
                               "peak_GBps": HBM_PEAK_GBPS}}
        if not args.no_naive_graph:
            g_steps = min(T, 1000)
            per_step = _naive_graph_rate(plan, v, g_steps, 5, torch)
            naive["graph"] = {"value": p.n / per_step, "ms_per_timestep": 1e3 * per_step,
                              "achieved_GBps": bytes_per_update * p.n / per_step / 1e9,
                              "captured_timesteps": g_steps}
        del v

    cpu = single_cpu_baseline(wl, p, args) if want_cpu and not args.no_cpu_baseline else None
    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t_swept / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": wl["dtype"], "data": DATA,
        "config": {"workload": wl["desc"], "n": p.n, "timesteps_per_run": T, "kind": wl["kind"],
                   "tile_width": info["tile_width"], "steps_per_cycle": spc, "engine": engine,
                   "parallelism": "single GPU",
                   "autotune": None if tuned is None else sorted(
                       ({"w": c["tile_width"], "spc": c["steps_per_cycle"], "engine": c["engine"],
                         "ns_per_update": round(c["ns_per_cell_update"], 6)} for c in tuned["candidates"]),
                       key=lambda c: c["ns_per_update"])},
        "roofline": roof,
        "naive": naive,
        "speedup_vs_naive": (value / naive["value"]) if naive else None,
        "speedup_vs_naive_graph": (value / naive["graph"]["value"]) if naive and "graph" in naive else None,
        "cpu_baseline": cpu,
    }
    plan.close()
    del u
    return out


def run_batch(args, wl):
    """Batched workload: one bench step = one graph launch (the whole batch)."""
    import numpy as np
    import torch

    import oracle
    from paper_1612_02495_amd import Batch, inputs
    T = wl["horizon"]
    probs = (inputs.heat_batch(nprob=wl["batch"], steps=T) if wl["kind"] == "heat"
             else inputs.ks_batch(nprob=wl["batch"], steps=T))
    n = np.array([p.n for p in probs])
    b = Batch(n, wl["kind"], wl["dtype"], [p.dt for p in probs], [p.dx for p in probs],
              [p.alpha for p in probs], T)
    engine = args.engine if args.engine in ("auto", "resident", "compact", "wave") else "auto"
    b.set_engine(engine)
    u = torch.tensor(np.concatenate([p.u0 for p in probs]), device="cuda")
    for _ in range(args.warmup):
        b.run(u)
    t = _time_runs(lambda: b.run(u), args.steps, torch)
    updates = int(n.sum()) * T * args.steps
    flops = FLOPS_PER_TIER_UPDATE[wl["kind"]] * int(n.sum()) * T * TIERS_PER_STEP[wl["kind"]]
    instr = FP_INSTR_PER_TIER_UPDATE[wl["kind"]] * int(n.sum()) * T * TIERS_PER_STEP[wl["kind"]]
    cpu = None
    if not args.no_cpu_baseline:
        budget = min(T, args.cpu_steps or (2000 if wl["kind"] == "heat" else 200))
        sample = probs[:32]
        cells = sum(p.n for p in sample) * budget
        if wl["kind"] == "heat":
            single = (lambda: [oracle.heat(p.u0, p.alpha, p.dt, p.dx, budget) for p in sample], cells,
                      f"first 32 of the {len(probs)} grids, {budget} of the {T} steps each, single-thread C oracle")
        else:
            single = (lambda: [oracle.ks(p.u0, p.dt, p.dx, budget) for p in sample], cells,
                      f"first 32 of the {len(probs)} grids, {budget} of the {T} steps each, single-thread C oracle")
        cpu = cpu_legs(single)
    out = {
        "metric": METRIC, "value": updates / t, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": wl["dtype"], "data": DATA,
        "config": {"workload": wl["desc"], "grids": int(n.size), "total_points": int(n.sum()),
                   "sizes_off_16_lattice": int(np.sum(n % 16 != 0)), "timesteps_per_run": T,
                   "kind": wl["kind"], "engine": engine, "persistent_grid": b.grid,
                   "edge_slot_bytes": b.workspace_bytes, "parallelism": "single GPU"},
        "roofline": roofline("batched run (whole graph launch)", flops, t / args.steps, wl["dtype"],
                             fp_instr=instr),
        "naive": None, "speedup_vs_naive": None, "cpu_baseline": cpu,
    }
    b.close()
    del u
    return out


def _reverse_launch_time(make_plan, forward, adjoint, h, r, torch):
    """Seconds per fused reverse launch: the difference of two reverse sweeps
    whose horizons differ by 32 full phases (same remainder)."""
    k_lo, k_hi = 8, 40
    times = {}
    for kk in (k_lo, k_hi):
        pk = make_plan(kk * h + r)
        state = forward(pk)
        adjoint(pk, state)  # warm-up
        times[kk] = _time_runs(lambda: adjoint(pk, state), 3, torch) / 3
        pk.close()
        del state
    return (times[k_hi] - times[k_lo]) / (k_hi - k_lo)


def run_adjoint(args, wl):
    """Heat gradient: one bench step = swept_forward_ckpt + swept_adjoint_run."""
    import torch

    import oracle
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
    # dJ/dalpha terms).  Algorithmic flops per launch: every tile's region
    # holds w h cell-updates, each recomputed (4 flops in 3 instructions),
    # walked by lambda (4 in 3) and paired with its Laplacian term (the
    # recompute's neighbour sum minus 2 u: 2 in one fused multiply-add; times
    # lambda and accumulated: 2 in one): 12 flops in 8 instructions.
    roof = None
    if not args.no_dominant:
        h = plan.info["steps_per_cycle"]
        r = plan.info["leading_classic_steps"]

        def fwd(pk):
            uk = torch.empty_like(du0)
            pk.forward(du0, dal, uk)
            return uk - y
        t_launch = _reverse_launch_time(lambda steps: AdjointPlan(B, n, dt, dx, steps), fwd,
                                        lambda pk, gk: pk.adjoint(gk, g_u0, g_a), h, r, torch)
        w = plan.info["tile_width"]
        flops = B * (n // w) * w * h * (4 + 4 + 4)
        roof = roofline("fused reverse region launch (recompute + lambda + dJ/dalpha)", flops, t_launch, "f64",
                        fp_instr=B * (n // w) * w * h * (3 + 3 + 2))
    # the same gradient with two-level checkpointing (about sqrt(K) phases per
    # segment: every segment-th phase's edge state kept, the rest recomputed)
    two = None
    if not args.no_two_level:
        p2 = AdjointPlan(B, n, dt, dx, T, segment=0)

        def step2():
            p2.forward(du0, dal, uT)
            p2.adjoint(uT - y, g_u0, g_a)
        step2()
        t2 = _time_runs(step2, args.steps, torch)
        two = {"adjoint_grad_ms": 1e3 * t2 / args.steps, "checkpoint_bytes": p2.info["checkpoint_bytes"],
               "time_vs_all_phases_kept": t2 / t}
        p2.close()
    cpu = None
    if not args.no_cpu_baseline:
        cs = args.cpu_steps or 1500
        cpu = cpu_legs((lambda: oracle.heat_adjoint(u0[0], u0t[0], alpha[0], dt, dx, cs), n * cs,
                        f"one of the {B} grids, {cs} of the {T} steps, single-thread C checkpointed reverse sweep"),
                       unit="cell-updates/s of gradient (forward + reverse)")
    out = {
        "metric": METRIC, "value": updates / t, "unit": "cell-updates/s of gradient (forward + reverse)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": DATA,
        "config": {"workload": wl["desc"], "batch": B, "n": n, "timesteps": T,
                   "adjoint_grad_ms": 1e3 * t / args.steps, "forward_ckpt_ms": 1e3 * t_fwd / args.steps,
                   "checkpoint_bytes": plan.info["checkpoint_bytes"],
                   "tile_width": plan.info["tile_width"], "steps_per_cycle": plan.info["steps_per_cycle"],
                   "leading_classic_steps": plan.info["leading_classic_steps"], "parallelism": "single GPU",
                   "two_level_checkpointing": two},
        "roofline": roof, "naive": None, "speedup_vs_naive": None, "cpu_baseline": cpu,
    }
    plan.close()
    del du0, y, uT, g_u0
    return out


def run_ks_adjoint(args, wl):
    """KS gradient: one bench step = swept_ks_forward_ckpt + swept_ks_adjoint_run."""
    import torch

    import oracle
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

    # Dominant kernel: the fused reverse region launch.  Algorithmic flops per
    # launch: every tile's region holds w h sub-step updates, each recomputed
    # (20 flops in 11 instructions) and walked back by the adjoint: Jf^T w
    # costs 12 in 8 (1 for the nonlinear weight v/(2 dx), 2 for the two
    # neighbour weights, 5 products and 4 sums in one multiply and 4 fused
    # multiply-adds), plus 1 in 1 (dt mu, odd tiers) or 3 in 2 ((lambda'' +
    # mu) + dt/2 Jf^T mu, even tiers): 34 flops in 20.5 instructions per
    # update on average.
    roof = None
    if not args.no_dominant:
        h = plan.info["steps_per_cycle"]
        r = plan.info["leading_classic_steps"]

        def fwd(pk):
            uk = torch.empty_like(du0)
            pk.forward(du0, uk)
            return (uk - y).contiguous()
        t_launch = _reverse_launch_time(lambda steps: KsAdjointPlan(B, n, dt, dx, steps), fwd,
                                        lambda pk, gk: pk.adjoint(gk, g_u0), h, r, torch)
        w = plan.info["tile_width"]
        flops = B * (n // w) * w * 2 * h * (20 + 14)
        roof = roofline("fused reverse region launch (recompute + adjoint walk)", flops, t_launch, "f64",
                        fp_instr=B * (n // w) * w * h * (2 * 11 + 2 * 8 + 1 + 2))
    cpu = None
    if not args.no_cpu_baseline:
        cs = args.cpu_steps or 100
        cpu = cpu_legs((lambda: oracle.ks_adjoint(u0[0], u0t[0], dt, dx, cs), n * cs,
                        f"grid 0 of {B}, {cs} of the {T} steps, single-thread C checkpointed reverse sweep"),
                       unit="cell-updates/s of gradient (forward + reverse)")
    out = {
        "metric": METRIC, "value": updates / t, "unit": "cell-updates/s of gradient (forward + reverse)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": DATA,
        "config": {"workload": wl["desc"], "batch": B, "n": n, "timesteps": T,
                   "adjoint_grad_ms": 1e3 * t / args.steps, "forward_ckpt_ms": 1e3 * t_fwd / args.steps,
                   "checkpoint_bytes": plan.info["checkpoint_bytes"],
                   "tile_width": plan.info["tile_width"], "steps_per_cycle": plan.info["steps_per_cycle"],
                   "leading_classic_steps": plan.info["leading_classic_steps"], "parallelism": "single GPU"},
        "roofline": roof, "naive": None, "speedup_vs_naive": None, "cpu_baseline": cpu,
    }
    plan.close()
    del du0, y, uT, g_u0
    return out


def run_workload(args, name):
    wl = dict(WORKLOADS[name])
    if args.horizon:
        wl["horizon"] = args.horizon
    if wl.get("batch"):
        return run_batch(args, wl)
    if wl.get("adjoint"):
        return run_ks_adjoint(args, wl) if wl["kind"] == "ks" else run_adjoint(args, wl)
    return run_single(args, wl, tile=args.tile or wl["tile"], engine=args.engine)


def nested_record(rec):
    """The fields of a workload's line that a nested record keeps."""
    keep = ("value", "unit", "steps", "warmup", "ms_per_step", "dtype", "config", "roofline", "naive",
            "speedup_vs_naive", "speedup_vs_naive_graph", "cpu_baseline")
    out = {k: rec[k] for k in keep if k in rec}
    cfg = dict(out.get("config") or {})
    cfg.pop("autotune", None)
    out["config"] = cfg
    return out


SWEEP_N = [2 ** k for k in range(11, 23)]
SWEEP_HORIZON = {"heat": 20000, "ks": 4000}


def run_sweep(args):
    """The paper's size sweep (Sec. 5): time per timestep of the swept and the
    naive run against N, heat and KS in FP64, autotuned per N."""
    import torch
    from paper_1612_02495_amd import Plan, swept_autotune
    rows = []
    for kind in ("heat", "ks"):
        T = args.horizon or SWEEP_HORIZON[kind]
        for n in SWEEP_N:
            print(f"sweep {kind} N={n}", file=sys.stderr, flush=True)
            p = _problem(kind, n, T)
            tuned = swept_autotune(p.n, kind, "f64", p.dt, p.dx, p.alpha)
            plan = Plan(p.n, kind, torch.float64, p.dt, p.dx, p.alpha, tile_width=tuned["tile_width"],
                        steps_per_cycle=tuned["steps_per_cycle"], engine=tuned["engine"])
            u = torch.tensor(p.u0, device="cuda")
            plan.run(u, T)
            t_s = _time_runs(lambda: plan.run(u, T), args.steps, torch) / args.steps
            v = torch.tensor(p.u0, device="cuda")
            plan.naive(v, min(T, 100))
            t_n = _time_runs(lambda: plan.naive(v, T), args.steps, torch) / args.steps
            g_steps = min(T, 1000)
            t_g = _naive_graph_rate(plan, v, g_steps, 3, torch) * T
            rows.append({"kind": kind, "n": n, "timesteps": T, "tile_width": tuned["tile_width"],
                         "steps_per_cycle": tuned["steps_per_cycle"], "engine": tuned["engine"],
                         "swept_us_per_timestep": 1e6 * t_s / T, "naive_us_per_timestep": 1e6 * t_n / T,
                         "naive_graph_us_per_timestep": 1e6 * t_g / T,
                         "swept_cell_updates_per_s": n * T / t_s, "naive_cell_updates_per_s": n * T / t_n,
                         "speedup_vs_naive": t_n / t_s, "speedup_vs_naive_graph": t_g / t_s})
            plan.close()
            del u, v
    return {"metric": "swept vs naive time per timestep against N (Sec. 5 sweep), FP64 heat and KS, one GPU",
            "unit": "see rows", "n_gpus": 1, "steps": args.steps, "dtype": "f64", "data": DATA,
            "paper_context": "the paper reports about 6x (small N) falling to about 2x (N = 2^20) for its "
                             "shared-memory swept kernels against its classic kernels on a Tesla K40c (Sec. 5); "
                             "context only",
            "rows": rows}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed bench steps (runs)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="heat", choices=sorted(WORKLOADS) + ["sweep"])
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
                    help="skip the per-launch timing of the dominant kernel (short profiler passes)")
    ap.add_argument("--no-nested", action="store_true",
                    help="measure the chosen workload only (no nested KS, batch and gradient records)")
    ap.add_argument("--batch", type=int, default=0, help="grids in the adjoint workloads (0 = 64 heat, 1 KS)")
    ap.add_argument("--no-two-level", action="store_true",
                    help="skip the two-level checkpointing timing of the heat gradient")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of MIB mebibytes (counter calibration)")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the swept path here is a single-GPU build "
              "(multi-GPU sharding is a design note only); run with --gpus 1.", file=sys.stderr)
        return 2

    import torch

    if args.workload == "sweep":
        print(json.dumps(run_sweep(args)))
        return 0
    print(f"workload {args.workload}", file=sys.stderr, flush=True)
    out = run_workload(args, args.workload)
    if args.workload == "heat" and not args.no_nested and not args.horizon and not args.tile:
        nested = {}
        sub = argparse.Namespace(**vars(args))
        sub.engine = "auto"
        sub.copy_calibration = 0
        for name in NESTED:
            print(f"workload {name}", file=sys.stderr, flush=True)
            nested[name] = nested_record(run_workload(sub, name))
            torch.cuda.empty_cache()
        out["workloads"] = nested
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
