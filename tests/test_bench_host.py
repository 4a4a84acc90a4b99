"""Host logic of bench.py (CPU): the --gpus guard, kernel names against the HIP sources, and the
lookup of committed traffic records."""
import glob
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_1902_08112_amd.profiling import sources_sha  # noqa: E402


def _template_arity():
    """Number of template parameters of every __global__ kernel in the HIP sources."""
    arity = {}
    for path in glob.glob(os.path.join(ROOT, "paper_1902_08112_amd", "csrc", "*.hip")):
        src = open(path).read()
        for m in re.finditer(r"template\s*<([^>]*)>\s*__global__"
                             r"(?:\s+__launch_bounds__\([^)]*\)|\s+__attribute__\(\((?:[^()]|\([^()]*\))*\)\))*"
                             r"\s+void\s+(k_\w+)\s*\(", src):
            arity[m.group(2)] = len([p for p in m.group(1).split(",") if p.strip()])
    return arity


def test_multi_gpu_request_exits():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("dim,degree,split", [(2, 1, False), (3, 1, False), (3, 2, False), (2, 2, False),
                                              (2, 1, True), (3, 1, True), (3, 2, True), (2, 2, True)])
@pytest.mark.parametrize("mode", [0, 1])
def test_kernel_names_match_sources(dim, degree, split, mode):
    arity = _template_arity()
    for variant in range(5):
        for fused in (False, True):
            name = bench.kernel_name(dim, degree, variant, split, mode, fused)
            m = re.fullmatch(r"(k_\w+)<([^<>]*)>", name)
            assert m, name
            stem, args = m.group(1), [t.strip() for t in m.group(2).split(",")]
            assert stem in arity, name
            assert len(args) == arity[stem], name
            assert str(mode) in args, name
            if stem in ("k_q1s", "k_q1_split", "k_cell_generic"):
                assert args[0] == str(dim), name
            if stem == "k_cell_generic":
                assert args[1] == str(degree) and args[-1] == ("true" if split else "false"), name
            if stem == "k_q1_3d":
                assert args[-1] == ("true" if fused else "false"), name


def test_split_names_pick_the_split_kernels():
    assert bench.kernel_name(3, 1, 0, True, 1).startswith("k_q1s<3, double, 1, 2>")
    assert bench.kernel_name(3, 1, 2, True, 0) == "k_q1s<3, double, 0, 1>"
    assert bench.kernel_name(3, 2, 0, True, 0) == "k_cell_generic<3, 2, double, 0, true>"
    assert bench.kernel_name(3, 2, 0, False, 1) == "k_q2_3d<double, 1>"


def test_committed_traffic_records_are_well_formed():
    paths = glob.glob(os.path.join(ROOT, "profiles", "*_traffic.json"))
    assert paths
    for p in paths:
        rec = json.load(open(p))
        for k in ("kernel", "hbm_bytes_per_launch", "sources", "sources_sha", "command"):
            assert k in rec, (p, k)
        assert rec["hbm_bytes_per_launch"] > 0
        for src in rec["sources"]:
            assert os.path.exists(os.path.join(ROOT, src)), (p, src)


def test_traffic_lookup_checks_kernel_and_sources(tmp_path, monkeypatch):
    srcs = ["paper_1902_08112_amd/csrc/cell_q1.hip", "paper_1902_08112_amd/csrc/q1_math.h"]
    (tmp_path / "profiles").mkdir()
    rec = {"kernel": "k_q1_3d<double, 1, 8, 8, false>", "hbm_bytes_per_launch": 1.5e7,
           "sources": srcs, "sources_sha": sources_sha(srcs), "command": "-"}
    path = tmp_path / "profiles" / "w_block_traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("w", rec["kernel"], "block") == 1.5e7
    assert bench.measured_traffic("w", "k_q1_3d<double, 1, 16, 4, false>", "block") is None
    assert bench.measured_traffic("w", rec["kernel"], "apply") is None
    assert bench.measured_traffic("other", rec["kernel"], "block") is None
    # a record taken from other sources (here: a different hash) no longer counts
    path.write_text(json.dumps(dict(rec, sources_sha="0" * 16)))
    assert bench.measured_traffic("w", rec["kernel"], "block") is None
