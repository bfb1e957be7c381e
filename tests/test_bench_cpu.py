"""Host-side checks of bench.py: it measures one GPU and refuses more, its
roofline fraction is taken against MI355X's published vector peak for the
dtype (with the instruction issue rate as a second figure), the traffic figure is
read from the committed counter summary only while the kernel sources match
it, the CPU baseline reports its thread counts and host, and the flop counts
per update are the stencils' operation counts."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_issue_rate_is_fp64_lane_instructions():
    # 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz, one instruction per lane per cycle
    assert bench.ALU_ISSUE_TERA == pytest.approx(256 * 4 * 16 * 2.4e9 / 1e12)
    assert bench.ALU_ISSUE_TERA == pytest.approx(78.6 / 2, rel=1e-3)


def test_flops_per_update():
    # heat: Fo (r + l) + c o is 4 operations, carried by fma(Fo, r + l, c*o)
    # in 3 instructions; a KS sub-step is the 5-point right-hand side (18
    # operations, the two squares included) plus the stage update (2), carried
    # in 11 instructions (two pair sums, the flux difference and product, three
    # multiply-adds of the numerators, one product and two multiply-adds with
    # the step-scaled coefficients, the final subtraction)
    assert bench.FLOPS_PER_TIER_UPDATE["heat"] == 4
    assert bench.FLOPS_PER_TIER_UPDATE["heat_insulated"] == 4
    assert bench.FLOPS_PER_TIER_UPDATE["ks"] == 20
    assert bench.FP_INSTR_PER_TIER_UPDATE == {"heat": 3, "heat_insulated": 3, "ks": 11}


def test_traffic_read_only_for_matching_sources(tmp_path, monkeypatch):
    wl = {"kind": "heat", "dtype": "f64", "n": 2 ** 20}
    t = bench._traffic_from_profile(wl, 1024, "compact")
    assert t is not None and 3.0e7 < t < 4.0e7  # both 1026-value slots of 1024 tiles, read and written
    # other sizes, widths or precisions have no committed counters
    assert bench._traffic_from_profile({"kind": "heat", "dtype": "f64", "n": 2 ** 21}, 1024, "compact") is None
    assert bench._traffic_from_profile({"kind": "ks", "dtype": "f32", "n": 2 ** 20}, 1024, "compact") is None
    assert bench._traffic_from_profile(wl, 512, "compact") is None
    # a changed kernel source voids the figure
    src = os.path.join(ROOT, bench.KERNEL_SOURCES["compact"][0])
    real = open(src, "rb").read()
    fake_root = tmp_path
    for f in bench.KERNEL_SOURCES["compact"]:
        dst = fake_root / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        dst.write_bytes(open(os.path.join(ROOT, f), "rb").read())
    (fake_root / bench.KERNEL_SOURCES["compact"][0]).write_bytes(real + b"\n// changed\n")
    prof = fake_root / bench.TRAFFIC_SUMMARY[("heat", "f64", "compact")]
    prof.parent.mkdir(parents=True, exist_ok=True)
    prof.write_bytes(open(os.path.join(ROOT, bench.TRAFFIC_SUMMARY[("heat", "f64", "compact")]), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(fake_root))
    assert bench._traffic_from_profile(wl, 1024, "compact") is None
    assert hashlib.sha256(real).hexdigest()  # the real tree is untouched


def test_roofline_uses_the_published_peak_and_the_issue_rate():
    r = bench.roofline("k", flops=4.0e9, t_launch=1e-4, dtype="f64")
    assert r["achieved"] == pytest.approx(40.0)
    assert r["peak"] == 78.6 and r["frac"] == pytest.approx(40.0 / 78.6)
    assert r["issue_peak"] == pytest.approx(39.3216) and r["frac_of_issue_peak"] == pytest.approx(40.0 / 39.3216)
    # four flops in three instructions raise the issue ceiling by 4/3
    r = bench.roofline("k", flops=4.0e9, t_launch=1e-4, dtype="f64", fp_instr=3.0e9)
    assert r["issue_peak"] == pytest.approx(39.3216 * 4 / 3) and r["frac"] == pytest.approx(40.0 / 78.6)
    assert r["unit"] == "TFLOP/s" and r["bound"] == "alu" and r["launch_ms"] == pytest.approx(0.1)
    assert bench.roofline("k", 1.0, 1.0, "f32")["peak"] == 157.3


def test_cpu_legs_report_threads_and_host():
    out = bench.cpu_legs((lambda: None, 100, "one"), (lambda: 7, 800, "all"))
    assert out["kind"] == "oracle" and out["cores"] == 7 and out["single_thread"]["cores"] == 1
    assert "7 threads" in out["sample"]
    host = out["host"]
    assert set(host) >= {"cpu_model", "nproc", "affinity_cpus", "omp_num_threads"}
    single_only = bench.cpu_legs((lambda: None, 100, "one"))
    assert single_only["cores"] == 1 and single_only["value"] == single_only["single_thread"]["value"]


def test_default_run_nests_the_rest_of_the_metric():
    assert bench.NESTED == ["ks", "batch", "batch_ks", "adjoint", "ks_adjoint"]
    rec = {"value": 1.0, "unit": "u", "ms_per_step": 2.0, "roofline": {}, "cpu_baseline": {}, "metric": "m",
           "config": {"workload": "w", "autotune": [1, 2]}}
    nr = bench.nested_record(rec)
    assert "metric" not in nr and "autotune" not in nr["config"] and nr["ms_per_step"] == 2.0
