"""bench.py's one-line JSON on a small workload (GPU): every field of the line, the roofline entry
of the dominant counted kernel and the oracle's CPU baseline."""
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
    assert d["value"] == pytest.approx(d["config"]["dofs"] / (d["ms_per_step"] * 1e-3), rel=1e-9)
    roof = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in roof
    assert roof["bound"] in ("hbm", "alu")
    # frac and achieved are rounded separately (5 and 2-4 decimals)
    assert roof["frac"] == pytest.approx(roof["achieved"] / roof["peak"], rel=1e-3, abs=1e-5)
    assert 0 < roof["frac"] < 1
    counted = [v for v in d["kernels"].values() if "frac" in v]
    assert roof["s_per_step"] == max(v["s_per_step"] for v in counted)
    cpu = d["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["unit"] == "DoFs/s" and cpu["cores"] == 1 and cpu["value"] > 0
    assert "8^3" in cpu["sample"]
