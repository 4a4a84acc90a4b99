"""bench.py's one-line JSON on a small workload (GPU): every field of the line, the roofline entry
of the FP64 Jacobian apply, the error between the two V-cycle precisions and the oracle's CPU
baseline with the replica's errors against the oracle."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.gpu
def test_bench_line_small3d():
    cmd = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--workload", "small3d", "--steps", "2",
           "--warmup", "1", "--apply-reps", "3", "--cpu-sample", "8"]
    print("bench:", " ".join(cmd[2:]), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["unit"] == "DoFs/s" and d["higher_is_better"] is True and d["scaling"] == "weak"
    assert d["dtype"] == "f64" and d["data"] == "synthetic" and d["vs_baseline"] is None
    assert d["config"]["workload"] == "small3d"
    assert d["value"] > 0 and d["ms_per_step"] > 0
    # value: DoFs/s of the FP64 Jacobian apply; ms_per_step: the Newton step in the workload's precision
    assert d["value"] == pytest.approx(d["apply_dofs_per_s_fp64"], rel=1e-12)
    assert d["value"] == pytest.approx(d["config"]["dofs"] / d["roofline"]["apply_call_s"], rel=1e-9)
    base = d["newton_s_fp64"] if d["config"]["vcycle"] == "f64" else d["newton_s_fp32_vcycle"]
    assert d["ms_per_step"] == pytest.approx(1e3 * base, rel=1e-12)
    assert d["rel_residual_fp64"] <= 1e-8 and d["rel_residual_fp32"] <= 1e-8
    # both precisions solve the same step to 1e-8: their updates agree far below 1
    assert 0 <= d["dU_fp32_vs_fp64_rel"] < 1e-5
    assert 0 < d["config"]["active_fraction"] < 1
    roof = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in roof
    assert roof["bound"] in ("hbm", "alu")
    # frac and achieved are rounded separately (5 and 2-4 decimals)
    assert roof["frac"] == pytest.approx(roof["achieved"] / roof["peak"], rel=1e-3, abs=1e-5)
    assert 0 < roof["frac"] < 1
    # small3d is a 3D Q1 mesh: its Jacobian apply is bound by FP64 VALU
    assert roof["kernel"] == d["kernels"]["jacobian"]["kernel"] and roof["bound"] == "alu"
    assert roof["hbm_frac"] == pytest.approx(roof["bytes_per_launch"] / roof["kernel_s_mean"] / 8e12, rel=1e-3, abs=1e-5)
    # 3D Q1: 2,496 flop against 26.25 B per DoF, so at the FP64 peak the apply moves bytes at
    # (bytes / 8 TB/s) / (flops / 78.6 TF/s) of the HBM peak; the measured fraction stays below it
    ceil = d["apply_hbm_frac_ceiling_fp64"]
    assert 0 < ceil < 1 and d["apply_hbm_frac_fp64"] <= ceil
    assert ceil == pytest.approx((roof["bytes_per_launch"] / 8e12) / (roof["flop_per_launch"] / 78.6e12), rel=1e-3)
    cpu = d["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["unit"] == "DoFs/s" and cpu["cores"] == 1 and cpu["value"] > 0
    assert "8^3" in cpu["sample"]
    for tag in ("fp64_vcycle", "fp32_vcycle"):
        rv = cpu["replica_vs_oracle"][tag]
        if rv["n_active"] == rv["oracle_n_active"]:
            assert rv["dU_rel_err_vs_oracle"] < 1e-5 and rv["oracle_rel_residual_of_gpu_dU"] < 1.1e-8
