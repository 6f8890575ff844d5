"""bench.py's host-side contract (no GPU): one GPU only, the shape of the CPU-baseline record,
and the committed counter summary that fills `roofline.traffic` and `valu_fp64` only while
the kernel sources hash to the profiled build."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

from paper_2108_06476_amd import inputs  # noqa: E402


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})])
def test_more_than_one_gpu_exits_with_a_message(argv, env):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv,
                       capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, **env))
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_cpu_baseline_record():
    cfg = inputs.scaled(inputs.workload("tgv_32"), cells=(2, 2, 2))
    rec = bench.cpu_baseline(cfg, 0.05)
    assert rec["kind"] == "oracle" and rec["unit"] == "DOF-RHS/s"
    assert rec["cores"] >= 1 and rec["value"] > 0 and "RK steps" in rec["sample"]
    one = bench.cpu_baseline_1core(cfg, 0.05)
    assert one["cores"] == 1 and one["value"] > 0


def test_stored_counters_are_gated_by_the_source_hash(monkeypatch):
    path = os.path.join(ROOT, "profiles", "k_stage_tgv32_fp64_pmc.json")
    rec = json.load(open(path))
    for key in ("source_sha256", "traffic_bytes_per_launch", "algorithmic_bytes_per_launch",
                "fp64_flops_per_launch", "calibration", "commands"):
        assert key in rec, key
    assert all(c.startswith("rocprofv3 ") for c in rec["commands"])
    assert rec["traffic_bytes_per_launch"] >= 0.9 * rec["algorithmic_bytes_per_launch"]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: rec["source_sha256"])
    assert bench.stored_traffic("k_stage_tgv32_fp64") == rec["traffic_bytes_per_launch"]
    assert bench.stored_pmc("k_stage_tgv32_fp64")["fp64_flops_per_launch"] > 0
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.stored_traffic("k_stage_tgv32_fp64") is None
    assert bench.stored_pmc("k_stage_tgv32_fp64") is None


def test_valu_object_from_the_stored_counters():
    """FP64 rate and vector-issue rate of the stage kernel from the committed counters: the
    arithmetic by hand, and None without a summary."""
    rec = json.load(open(os.path.join(ROOT, "profiles", "k_stage_tgv32_fp64_pmc.json")))
    avg_ms = 0.075
    v = bench.valu_object(rec, avg_ms)
    flops = rec["fp64_flops_per_launch"]
    assert abs(v["achieved"] - flops / 75e-6 / 1e12) < 0.01
    assert v["peak"] == 78.6 and abs(v["frac"] - v["achieved"] / 78.6) < 1e-3
    insts = rec["counters_per_launch"]["SQ_INSTS_VALU"]
    # 1024 SIMDs x 2.4 GHz / 4 clocks per 64-lane instruction
    assert v["issue"]["peak"] == 614.4
    assert abs(v["issue"]["frac"] - insts / 75e-6 / 614.4e9) < 1e-3
    # the counters hold 64 lanes per instruction: SQ_INSTS_VALU / SQ_WAVES is the per-wave count
    assert abs(insts / rec["counters_per_launch"]["SQ_WAVES"] - rec["valu_insts_per_wave"]) < 0.1
    assert bench.valu_object(None, avg_ms) is None
