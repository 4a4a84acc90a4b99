"""Benchmark: seconds per Newton/active-set step and Jacobian-apply throughput on one MI355X.

Workload (default): 3D unit cube, 64^3 Q1 hexahedra (274,625 nodes, 1,098,500
DoFs), pressurized penny crack of radius 0.2, eps = 2h, seeded uniform(-1e-3,
1e-3) displacement, 5-level GMG.  A step is one whole Newton step of the
library (residual, active set, level data, diagonals, eigenvalue estimates,
FGMRES with the V-cycle to a 1e-8 true relative residual, update), starting
each time from the same iterate U_k (the reset copy is inside the timed loop).

value = fine-level DoFs per second of Newton steps in the workload's own
V-cycle precision; the other precision's step time and the speedup are
reported beside it.  Inside the timed FP64 Newton steps the library brackets
every 8th launch of the two finest-level FP64 cell kernels, the Jacobian G~
and the smoother's block operator B~, with HIP events on the launch stream
(pf_set_kernel_timing); "kernels" reports both (launches per step, mean launch
duration, achieved = algorithmic flops or bytes per launch / mean duration),
and the roofline entry is the one with the larger time per step among those
with an algorithmic count (B~ is counted on Q1 levels, where it reads stored
per-point coefficients or the split's eigen-records, and on 3D Q2).  traffic = HBM bytes per launch from the
committed rocprofv3 FETCH_SIZE / WRITE_SIZE summaries of this command
(profiles/<workload>_apply_traffic.json for G~, _block_traffic.json for B~),
while the kernel's sources are unchanged.  After the timed region a plain
device copy of one fine-level vector runs (the counters' calibration).
With --tuning-cache the autotuner's choices are read from (or written to) a
file, so that profiled runs use the choices of an unprofiled one.
cpu_baseline: the FP64 oracle's Newton step on a 32^3 sample of the same
workload (same crack, material and eps), one core.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu] [--tuning-cache F]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Jacobian-apply DoFs/s + %HBM peak; s/Newton step, FP32 vs FP64 GMG at 1e-8"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# algorithmic work of one Jacobian apply (per cell flops, per DoF bytes in FP64)
FLOP_PER_CELL = {(2, 1): 656.0, (3, 1): 2496.0, (3, 2): 12312.0, (2, 2): 2124.0}
BYTES_PER_DOF_F64 = {2: 8 * 3 + (8 + 1) / 3.0, 3: 8 * 3 + (8 + 1) / 4.0}
# Miehe split, Q1 apply from stored per-point records: flops per cell (the unsplit count plus the
# tangent C - (1 - g) C^+ in the eigenbasis and sigma^+ : e(du), E_s^+ from the eigenvalues) and the
# record bytes per cell (tr e, eigenvalues, eigenvectors: 8 values x 8 points 3D, 5 x 4 2D, FP64)
SPLIT_FLOP_PER_CELL = {2: 656.0 + 4 * 76.0, 3: 2496.0 + 8 * 240.0}
SPLIT_REC_BYTES_PER_CELL = {2: 5 * 4 * 8.0, 3: 8 * 8 * 8.0}
# block operator B~ (the smoother's operator), same counting rule over the fields B~ touches; its
# per-point coefficients are stored at the linearization.  Q1 reads c_phi JxW per Gauss point:
# forward (d+1)(I+Gr) + I, backward (d+1)(I+Gr), 36 flops per 3D and 21 per 2D point; x, y at d+1
# values, phi~ and the mask per node plus 2^d FP64 coefficients per cell.  3D Q2 reads g(phi~) JxW
# and c_phi: forward and backward (d+1)(I+Gr), 48 flops per point (the Jacobian's 96 less the phi-u
# coupling and the linearization-point terms); x, y at d+1 values and the mask per node plus 54
# FP64 coefficients per cell.
BLOCK_FLOP_PER_CELL = {(2, 1): 396.0, (3, 1): 1512.0, (3, 2): 7776.0}
BLOCK_BYTES_PER_NODE_F64 = {(2, 1): 8 * 6 + 8 + 1.0, (3, 1): 8 * 8 + 8 + 1.0, (3, 2): 8 * 8 + 1.0}
BLOCK_COEF_BYTES_PER_CELL = {(2, 1): 4 * 8.0, (3, 1): 8 * 8.0, (3, 2): 54 * 8.0}
# B~ of the Miehe split (3D Q1) from the per-point eigen-records: the unsplit block count plus the
# tangent's eigenbasis rotations in the displacement rows (190 flops per point; the phase-field
# rows take E_s^+ from the eigenvalues); x, y, phi~ and the mask per node plus the 512 B record
SPLIT_BLOCK_FLOP_PER_CELL = {3: 1512.0 + 8 * 190.0}
# every KT_EVERY-th launch of each fine-level FP64 cell kernel is bracketed with HIP events in the
# timed FP64 steps (a bracket delays the stream by a few microseconds)
KT_EVERY = 8
# a Chebyshev step fused into a marching-tile B~ apply (per DoF: r -= t, d' = c1 d + c2 r / diag,
# x += d'; bytes: r read and written, diag, x read and written, d' written)
CHEB_FLOP_PER_DOF = 7.0
CHEB_BYTES_PER_DOF_F64 = 6 * 8.0


# kernel of the finest-level FP64 Jacobian (mode 0) or block (mode 1) apply for a tuning variant,
# as rocprofv3 names it
def kernel_name(dim, degree, variant, split=False, mode=0, fused=False):
    fused = "true" if fused else "false"
    if split and degree == 1:
        return f"k_q1s<{dim}, double, {mode}, {1 if variant == 2 else 2}>"
    if degree == 2:
        if dim == 3 and not split:
            return f"k_q2_3d<double, {mode}>"
        return f"k_cell_generic<{dim}, 2, double, {mode}, {'true' if split else 'false'}>"
    if dim == 2:
        return {0: f"k_q1_2d<double, {mode}>", 2: f"k_q1_2d_atomic<double, {mode}>",
                4: f"k_q1_split<2, double, {mode}>"}.get(variant, f"k_q1_2d<double, {mode}>")
    return {0: f"k_q1_3d<double, {mode}, 8, 8, {fused}>", 1: f"k_q1_3d<double, {mode}, 16, 4, {fused}>",
            2: f"k_q1_3d_atomic<double, {mode}>", 3: f"k_q1_3d_brick<double, {mode}>",
            4: f"k_q1_split<3, double, {mode}>", 5: f"k_q1_3d_slab<double, {mode}, {fused}>"}.get(variant, "?")


def measured_traffic(workload, kname, role="apply"):
    """HBM bytes per launch of a kernel (role "apply": the Jacobian, "block": B~) from the
    committed rocprofv3 --pmc summary (FETCH_SIZE + WRITE_SIZE scaled by a plain copy), or None
    if there is none for this kernel or its sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{workload}_{role}_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        from paper_1902_08112_amd.profiling import sources_sha
        rec = json.load(open(path))
        if rec.get("kernel") != kname or rec.get("sources_sha") != sources_sha(rec.get("sources", [])):
            return None
        return rec["hbm_bytes_per_launch"]
    except Exception:
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg5_3d_q1_lshape_256")
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tuning-cache", default=None,
                    help="JSON file of autotuner choices: read if it holds this mesh, else written")
    ap.add_argument("--cpu-sample", type=int, default=32)
    return ap.parse_args()


def cpu_baseline(spec, n_sample):
    """The oracle's Newton step on the n_sample^d replica of the workload (the same recipe with eps
    at the same multiple of h; one core), and the library's FP64- and FP32-V-cycle steps from the
    same iterate compared with it: the error of each result against the FP64 oracle solve."""
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    try:
        from threadpoolctl import threadpool_limits
        ctx = threadpool_limits(1)
    except Exception:  # pragma: no cover
        ctx = None
    import numpy as np
    import torch

    import workloads as W
    from oracle import mg, model, newton
    from paper_1902_08112_amd import pff
    s = W.scaled(spec, n_sample, min(spec["n_levels"], 3))
    mat = model.Material(**s["material"])
    U, Uold, phit = W.make_state(s)
    t0 = time.perf_counter()
    H = mg.Hierarchy(s["dim"], s["degree"], s["n_cells"], s["extent"], s["domain"], s["n_levels"], s["faces"], mat,
                     extra_u_bits=W.extra_constraint_bits(s))
    ref = newton.newton_step(H, U, Uold, phit)
    dt = time.perf_counter() - t0
    if ctx is not None:
        ctx.__exit__(None, None, None)
    nd = int((~H.fine.hole_node).sum()) * (s["dim"] + 1)   # DoFs of the domain
    S = pff.solver_from_spec(s)
    bits = W.extra_constraint_bits(s)
    if bits is not None:
        S.set_constraints(torch.from_numpy(bits).cuda())
    errs = {}
    for prec, tag in ((pff.PF_F64, "fp64_vcycle"), (pff.PF_F32, "fp32_vcycle")):
        S.set_vcycle_precision(prec)
        Ud = torch.from_numpy(U).cuda()
        _, rep = S.newton_step(Ud, torch.from_numpy(Uold).cuda(), torch.from_numpy(phit).cuda())
        dU = Ud.cpu().numpy() - U
        errs[tag] = {"dU_rel_err_vs_oracle": float(np.linalg.norm(dU - ref["dU"]) / np.linalg.norm(ref["dU"])),
                     "oracle_rel_residual_of_gpu_dU": float(np.linalg.norm(ref["Rt"] - ref["Gt"] @ dU)
                                                            / np.linalg.norm(ref["Rt"])),
                     "gmres_iters": rep.gmres_iters, "n_active": rep.n_active, "oracle_n_active": ref["n_active"]}
    S.close()
    return {"value": nd / dt, "unit": "DoFs/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle Newton step (assembly, FGMRES+V-cycle to 1e-8) on the {n_sample}^{s['dim']} "
                      f"replica of the workload ({nd} DoFs, {s['n_levels']} levels, "
                      f"eps = same multiple of h), {dt:.1f} s, {ref['info']['iters']} FGMRES iterations, "
                      f"|A_k| = {ref['n_active']}; 1 of os.cpu_count()={os.cpu_count()} cores",
            "replica_vs_oracle": errs}


def run_batch(a):
    """The 64-instance 2D family (16^2..256^2 Q1, 4 levels each) in one batched Newton step."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1902_08112_amd import pff

    torch.cuda.set_device(0)
    specs = W.batched_instances(seed=4, count=64)
    states = [W.make_state(s) for s in specs]
    o = pff.pf_default_options()
    o.vcycle_precision = pff.PF_F32
    BS = pff.BatchSolver(specs, o)
    U0 = BS.pack([st[0] for st in states])
    Uold = BS.pack([st[1] for st in states])
    phit = BS.pack([st[2] for st in states], nodes=True)
    U = torch.empty_like(U0)
    n_dofs = sum(BS.dof_off[-1][b + 1] - BS.dof_off[-1][b] for b in range(BS.n))
    n_cells = sum(int(np.prod(s["n_cells"])) for s in specs)

    def steps(k, prec):
        BS.set_vcycle_precision(prec)
        reps = None
        for _ in range(k):
            U.copy_(U0)
            _, reps = BS.newton_step(U, Uold, phit)
        return reps

    # one step sets the linearization; the autotuner then picks the cell-loop shape per level
    # (or the choices of an earlier run are read back from the tuning cache)
    steps(1, pff.PF_F32)
    tuning = None
    if not a.no_tune:
        cache = {}
        if a.tuning_cache and os.path.exists(a.tuning_cache):
            with open(a.tuning_cache) as f:
                cache = json.load(f)
        if "batch64_2d_q1" in cache:
            for lv in cache["batch64_2d_q1"]:
                for ch in lv["choices"]:
                    BS.set_tuning(lv["level"], pff.PF_F64 if ch["prec"] == "f64" else pff.PF_F32,
                                  0 if ch["mode"] == "jacobian" else 1, ch["shape"], ch["zc"])
            tuning = BS.tuning()
        else:
            tuning = BS.autotune(reps=10)
            if a.tuning_cache:
                cache["batch64_2d_q1"] = tuning
                with open(a.tuning_cache, "w") as f:
                    json.dump(cache, f)
    res = {}
    for prec in (pff.PF_F32, pff.PF_F64):
        steps(max(1, a.warmup), prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = steps(a.steps, prec)
        torch.cuda.synchronize()
        res[prec] = ((time.perf_counter() - t0) / a.steps, reps)
    t32, reps32 = res[pff.PF_F32]
    t64, _ = res[pff.PF_F64]
    # the same 64 instances one by one (one context each), FP32 V-cycle
    seq = 0.0
    for b, s in enumerate(specs):
        S = pff.solver_from_spec(s)
        u0, uo, pt = (torch.from_numpy(x).cuda() for x in states[b])
        u = u0.clone()
        S.newton_step(u, uo, pt)
        u.copy_(u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.newton_step(u, uo, pt)
        torch.cuda.synchronize()
        seq += time.perf_counter() - t0
        S.close()
    # batched FP64 apply on the finest level of every instance (2D Q1: HBM-bound)
    BS.set_vcycle_precision(pff.PF_F32)
    x = BS.pack([np.random.default_rng(b).uniform(-1, 1, st[0].size) for b, st in enumerate(states)])
    for _ in range(5):
        BS.jacobian_apply(-1, x)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(a.apply_reps):
        BS.jacobian_apply(-1, x)
    e1.record(stream)
    torch.cuda.synchronize()
    t_apply = e0.elapsed_time(e1) / 1e3 / a.apply_reps
    bytes_ = BYTES_PER_DOF_F64[2] * n_dofs
    ach = bytes_ / t_apply / 1e9
    # the fine level's shape as tuned: its work-item kernel, and that kernel's traffic record
    shape = None if tuning is None else tuning[-1]["choices"][0]["shape"]
    kname = None if shape is None or shape < 0 else f"k_b_items<2, double, 0, {shape}>"
    traffic = None if kname is None else measured_traffic("batch64_2d_q1", kname, "apply")
    out = {
        "metric": METRIC, "value": n_dofs / t32, "unit": "DoFs/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * t32, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batch64_2d_q1", "instances": len(specs), "dofs": n_dofs, "n_levels": 4,
                   "vcycle": "f32", "gmres_rtol": 1e-8},
        "newton_s_fp32_vcycle": t32, "newton_s_fp64": t64, "fp32_vcycle_speedup": t64 / t32,
        "one_by_one_s": seq, "batched_speedup": seq / t32,
        "gmres_iters_min_max": [min(r["gmres_iters"] for r in reps32), max(r["gmres_iters"] for r in reps32)],
        "roofline": {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": traffic,
                     "kernel": kname, "role": "batched FP64 Jacobian apply, finest levels of all instances",
                     "bytes_per_launch": bytes_, "flop_per_launch": FLOP_PER_CELL[(2, 1)] * n_cells,
                     "traffic_over_algorithmic": None if traffic is None else round(traffic / bytes_, 4),
                     "apply_s": t_apply},
        "cpu_baseline": None,
        "tuning_fine_level": None if tuning is None else tuning[-1]["choices"],
    }
    BS.close()
    if not a.no_cpu:
        small = [s for s in specs if s["n_cells"][0] <= 24]
        t0 = time.perf_counter()
        nd = 0
        from oracle import mg, model, newton
        for s in small:
            mat = model.Material(**s["material"])
            u, uo, pt = W.make_state(s)
            H = mg.Hierarchy(s["dim"], s["degree"], s["n_cells"], s["extent"], s["domain"], s["n_levels"],
                             s["faces"], mat)
            newton.newton_step(H, u, uo, pt)
            nd += H.fine.n_dofs
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": nd / dt, "unit": "DoFs/s", "cores": 1, "kind": "oracle",
                               "sample": f"oracle Newton steps of the {len(small)} instances with <= 24^2 cells "
                                         f"({nd} DoFs) run one after another, {dt:.1f} s"}
    print(json.dumps(out), flush=True)


def state_counts(S, s, n_active):
    """Domain DoFs, phi-nodes and the active fraction |A_k| / #phi of a workload."""
    n_nodes = int(S.levels[-1].n_domain_nodes)
    return n_nodes * (s["dim"] + 1), n_nodes, n_active / n_nodes


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {a.gpus}); the multi-GPU path is a design, "
              f"not part of this build.", file=sys.stderr)
        sys.exit(2)
    if a.workload == "batch64":
        return run_batch(a)
    import numpy as np
    import torch

    import workloads as W
    from paper_1902_08112_amd import pff

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    s = W.config(a.workload)
    U0, Uold, phit = W.make_state(s)
    S = pff.solver_from_spec(s)
    bits = W.extra_constraint_bits(s)
    if bits is not None:
        S.set_constraints(torch.from_numpy(bits).cuda())
    n_vec = S.n_dofs()                   # stored lattice vector length (hole nodes included)
    dU0 = torch.from_numpy(U0).cuda()
    dUold = torch.from_numpy(Uold).cuda()
    dphit = torch.from_numpy(phit).cuda()
    U = torch.empty_like(dU0)
    print(f"bench: {a.workload}, {n_vec} stored DoFs, set-up done", file=sys.stderr, flush=True)

    def run_steps(k, prec, solver=None):
        solver = solver or S
        solver.set_vcycle_precision(prec)
        reps = []
        for _ in range(k):
            U.copy_(dU0)
            st, rep = solver.newton_step(U, dUold, dphit)
            reps.append(rep.as_dict())
        return reps

    def timed(k, prec):
        # both precisions run with the same brackets: every KT_EVERY-th finest-level FP64 launch
        # of G~ (the FGMRES operator, FP64 in both) is timed with HIP events on its stream
        S.set_kernel_timing(pff.PF_KTIME_JACOBIAN, every=KT_EVERY)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = run_steps(k, prec)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / k
        S.set_kernel_timing(False)
        kt = S.kernel_timing(pff.PF_KTIME_JACOBIAN, launches=True)
        dU = U - dU0                     # the update of the last step
        return dt, reps, kt, dU

    base_prec = pff.PF_F32 if s.get("vcycle") == "f32" else pff.PF_F64
    other_prec = pff.PF_F64 if base_prec == pff.PF_F32 else pff.PF_F32
    # one step sets the linearization point; the autotuner then picks the cell-loop shape per level
    run_steps(1, base_prec)
    tuning = S.autotune(reps=10, cache_path=a.tuning_cache) if not a.no_tune else None
    run_steps(a.warmup, base_prec)
    t_base, reps, kt_base, dU_base = timed(a.steps, base_prec)
    run_steps(a.warmup, other_prec)
    t_other, reps_o, kt_other, dU_other = timed(a.steps, other_prec)
    t64, t32 = (t_base, t_other) if base_prec == pff.PF_F64 else (t_other, t_base)
    r64, r32 = (reps, reps_o) if base_prec == pff.PF_F64 else (reps_o, reps)
    dU64, dU32 = (dU_base, dU_other) if base_prec == pff.PF_F64 else (dU_other, dU_base)
    # error of the FP32-V-cycle result against the all-FP64 solve of the same step
    dU_err = float(torch.linalg.norm(dU32 - dU64) / torch.linalg.norm(dU64))
    print(f"bench: Newton steps FP64 {1e3 * t64:.2f} ms, FP32 V-cycle {1e3 * t32:.2f} ms", file=sys.stderr,
          flush=True)

    # kernel records of every finest-level FP64 cell kernel (G~, B~, B~ with a fused Chebyshev
    # step) from extra FP64 steps outside the timed region
    n_kt = max(2, min(a.steps, 4))
    S.set_kernel_timing(pff.PF_KTIME_JACOBIAN | pff.PF_KTIME_BLOCK | pff.PF_KTIME_BLOCK_CHEB, every=KT_EVERY)
    run_steps(n_kt, pff.PF_F64)
    torch.cuda.synchronize()
    S.set_kernel_timing(False)
    kt = {op: S.kernel_timing(op, launches=True)
          for op in (pff.PF_KTIME_JACOBIAN, pff.PF_KTIME_BLOCK, pff.PF_KTIME_BLOCK_CHEB)}

    # the Jacobian apply on its own: the whole pf_jacobian_apply call on the finest level
    # (linearization of the last step), back to back on one stream, FP64 and FP32
    x = torch.from_numpy(np.random.default_rng(0).uniform(-1, 1, n_vec)).cuda()
    y = torch.empty_like(x)
    L = s["n_levels"] - 1
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def time_apply(xv, yv):
        for _ in range(5):
            S.jacobian_apply(L, xv, out=yv)
        ev0.record(stream)
        for _ in range(a.apply_reps):
            S.jacobian_apply(L, xv, out=yv)
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / 1e3 / a.apply_reps

    t_apply = time_apply(x, y)
    x32 = x.float()
    t_apply32 = time_apply(x32, torch.empty_like(x32))

    info = S.levels[L]
    n_cells = int(info.n_active_cells)
    n_dofs, n_phi, active_frac = state_counts(S, s, r64[-1]["n_active"])
    n_nodes = n_phi
    # the split's Q1 operators stream per-point records (counted below); with Q2 the split is
    # evaluated on the fly in the generic cell kernel, which has no algorithmic count here
    mat_split = s["material"].get("split", "none") == "miehe"
    split = mat_split and s["degree"] == 1

    def kernel_entry(rec, steps_seen, flops, bytes_, bound, kname, role, extra_bytes=0.0, t_fallback=None):
        """Roofline entry of one kernel: algorithmic flops or bytes per launch (the counting rule of
        the hot-path table: x, U, y at d+1 values, phi~ and a mask byte per node) / mean duration of
        its bracketed launches.  extra_bytes: bytes the kernel reads beyond that rule (coefficients
        stored at the linearization, the split's records), reported separately."""
        launches, k_count, k_mean, k_min, k_max = rec
        t_kernel = k_mean if k_count > 0 else t_fallback
        e = {"kernel": kname, "launches_per_step": launches / steps_seen, "launches_timed": k_count,
             "timed_every": KT_EVERY, "kernel_s_mean": t_kernel, "kernel_s_min": k_min, "kernel_s_max": k_max,
             "s_per_step": (launches / steps_seen) * (t_kernel or 0.0)}
        if flops is None or not t_kernel:
            return e
        ach_tf = flops / t_kernel / 1e12
        ach_gbs = bytes_ / t_kernel / 1e9
        if bound == "hbm":
            roof = {"bound": "hbm", "achieved": round(ach_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach_gbs / HBM_PEAK_GBS, 5)}
        else:
            roof = {"bound": "alu", "achieved": round(ach_tf, 4), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(ach_tf / FP64_PEAK_TFLOPS, 5)}
        traffic = measured_traffic(a.workload, kname, role)
        roof.update({"traffic": traffic}, **e)
        roof.update({"flop_per_launch": flops, "bytes_per_launch": bytes_,
                     "stored_bytes_per_launch": extra_bytes,
                     "traffic_over_algorithmic": None if traffic is None else round(traffic / bytes_, 4),
                     "tflops_achieved": round(ach_tf, 4), "tflops_frac": round(ach_tf / FP64_PEAK_TFLOPS, 5),
                     "hbm_achieved_GBs": round(ach_gbs, 2), "hbm_frac": round(ach_gbs / HBM_PEAK_GBS, 5)})
        return roof

    # the Jacobian G~: algorithmic flops (bytes) per launch / mean duration of the timed launches
    rule_bytes = BYTES_PER_DOF_F64[s["dim"]] * n_dofs
    if split:
        flops = SPLIT_FLOP_PER_CELL[s["dim"]] * n_cells
        extra = SPLIT_REC_BYTES_PER_CELL[s["dim"]] * n_cells
    elif mat_split:
        flops = extra = None
    else:
        flops = FLOP_PER_CELL[(s["dim"], s["degree"])] * n_cells
        extra = 0.0
    vj = pff.pf_get_tuning(S.ctx, L, pff.PF_F64, 0)[0]
    jname = kernel_name(s["dim"], s["degree"], vj, mat_split, 0)
    # the binding roof is the one with the longer time at peak (flop/B against the FP64 ridge of 9.8):
    # FP64 VALU for the 3D applies, HBM for 2D Q1 and for the split's record-streaming Q1 apply
    jbound = None if flops is None else (
        "alu" if flops / FP64_PEAK_TFLOPS / 1e12 >= (rule_bytes + extra) / HBM_PEAK_GBS / 1e9 else "hbm")
    jac = kernel_entry(kt_base, a.steps, flops, rule_bytes + (extra or 0.0), jbound, jname, "apply",
                       extra_bytes=extra or 0.0, t_fallback=t_apply)
    jac.update({"apply_call_s": t_apply, "apply_call_f32_s": t_apply32,
                "measured_in": "the timed Newton steps of the workload's V-cycle precision"})
    # the block operator B~ (unsplit on Q1 and 3D Q2; with the split on 3D Q1, from its records):
    # by the counting rule its bytes are those of an on-the-fly evaluation (it would read U to form
    # its phase-field coefficient), the stored coefficients it reads instead are reported apart
    vb = pff.pf_get_tuning(S.ctx, L, pff.PF_F64, 1)[0]
    key = (s["dim"], s["degree"])
    if split and s["dim"] in SPLIT_BLOCK_FLOP_PER_CELL:
        bflops = SPLIT_BLOCK_FLOP_PER_CELL[s["dim"]] * n_cells
        bextra = SPLIT_REC_BYTES_PER_CELL[s["dim"]] * n_cells
    elif key in BLOCK_FLOP_PER_CELL and not mat_split:
        bflops = BLOCK_FLOP_PER_CELL[key] * n_cells
        bextra = BLOCK_COEF_BYTES_PER_CELL[key] * n_cells
    else:
        bflops = bextra = None
    bbytes = None if bflops is None else rule_bytes + (bextra if split else 0.0)
    bextra_rep = 0.0 if bextra is None else bextra
    # flop/B is near the FP64 ridge (9.8): the binding roof is the larger of the two times
    bbound = None if bflops is None else (
        "alu" if bflops / FP64_PEAK_TFLOPS / 1e12 >= bbytes / HBM_PEAK_GBS / 1e9 else "hbm")
    blk = kernel_entry(kt[pff.PF_KTIME_BLOCK], n_kt, bflops, bbytes, bbound,
                       kernel_name(s["dim"], s["degree"], vb, mat_split, 1), "block", extra_bytes=bextra_rep)
    kernels = {"jacobian": jac, "block": blk}
    if kt[pff.PF_KTIME_BLOCK_CHEB][0] > 0 and bflops is not None:
        cflops = bflops + CHEB_FLOP_PER_DOF * n_dofs
        cbytes = bbytes + CHEB_BYTES_PER_DOF_F64 * n_dofs
        cbound = "alu" if cflops / FP64_PEAK_TFLOPS / 1e12 >= cbytes / HBM_PEAK_GBS / 1e9 else "hbm"
        kernels["block_cheb"] = kernel_entry(kt[pff.PF_KTIME_BLOCK_CHEB], n_kt, cflops, cbytes, cbound,
                                             kernel_name(s["dim"], s["degree"], vb, split, 1, fused=True),
                                             "block_cheb", extra_bytes=bextra_rep)
    # the roofline entry is the FP64 Jacobian apply that the metric names
    if "frac" in jac:
        roof = dict(jac, role="Jacobian G~ (FP64, finest level)")
    else:
        roof = dict(jac, role="Jacobian G~ (FP64, finest level)", bound=None, achieved=None, peak=None,
                    unit=None, frac=None, traffic=None,
                    note="no algorithmic count for the split evaluated on the fly (Q2)")
    # the PDAS loop to convergence (Algorithm 1 repeated until A_k = A_{k-1} and ||R~|| <= 1e-10)
    # from the same iterate, in the workload's V-cycle precision
    S.set_vcycle_precision(base_prec)
    U.copy_(dU0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, prep = S.pdas_solve(U, dUold, dphit, max_iter=50, tol_as=1e-10, raise_on_error=False)
    torch.cuda.synchronize()
    pdas_out = dict(prep.as_dict(), wall_s=time.perf_counter() - t0)
    # quantities of interest of the converged state (synchronizing calls, 10 each)
    t0 = time.perf_counter()
    for _ in range(10):
        ec, eb = S.energies(U)
    t_en = (time.perf_counter() - t0) / 10
    face = 2 * s["dim"] - 1
    t0 = time.perf_counter()
    for _ in range(10):
        load = S.boundary_traction(U, face)
    t_ld = (time.perf_counter() - t0) / 10
    quant = {"crack_energy": ec, "bulk_energy": eb, "energies_s": t_en, "face": face, "face_load": load,
             "face_load_s": t_ld}
    print("bench: PDAS loop and quantities done", file=sys.stderr, flush=True)
    # the alternative preconditioner P_diag = diag(MG(U~), MG(P~)) (Sec. 3.3): the same Newton
    # step from the same iterate in the workload's V-cycle precision, on its own tuned context
    S.close()
    Sd = pff.solver_from_spec(s, preconditioner=pff.PF_PREC_DIAG)
    if bits is not None:
        Sd.set_constraints(torch.from_numpy(bits).cuda())
    run_steps(1, base_prec, Sd)
    if not a.no_tune:
        Sd.autotune(reps=10, cache_path=a.tuning_cache)
    run_steps(a.warmup, base_prec, Sd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps_d = run_steps(a.steps, base_prec, Sd)
    torch.cuda.synchronize()
    t_diag = (time.perf_counter() - t0) / a.steps
    pdiag = {"newton_s": t_diag, "gmres_iters": reps_d[-1]["gmres_iters"],
             "converged": reps_d[-1]["converged"], "rel_residual": reps_d[-1]["rel_residual"],
             "p_full_newton_s": t_base, "p_full_gmres_iters": reps[-1]["gmres_iters"]}
    Sd.close()
    # plain device copy of a known size: the scale of the FETCH_SIZE / WRITE_SIZE counters
    # in rocprofv3 --pmc runs of this same command (not timed, not part of the result)
    src = torch.rand(n_vec, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    out = {
        "metric": METRIC,
        "value": n_dofs / t_apply,
        "unit": "DoFs/s",
        "value_of": "FP64 Jacobian apply G~ (pf_jacobian_apply, finest level, inputs resident in HBM)",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * t_base,
        "step_of": "one Newton/PDAS step (Algorithm 1) in the workload's V-cycle precision",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "dim": s["dim"], "degree": s["degree"], "n_cells": list(s["n_cells"]),
                   "n_levels": s["n_levels"], "dofs": n_dofs, "phi_nodes": n_phi,
                   "vcycle": "f64" if base_prec == pff.PF_F64 else "f32", "gmres_rtol": 1e-8,
                   "split": s["material"].get("split", "none"),
                   "active_target": s.get("active_target"), "active_fraction": round(active_frac, 5)},
        "apply_dofs_per_s_fp64": n_dofs / t_apply,
        "apply_dofs_per_s_fp32": n_dofs / t_apply32,
        "apply_hbm_frac_fp64": round(rule_bytes / t_apply / 1e9 / HBM_PEAK_GBS, 5),
        # the largest fraction of HBM peak the FP64 apply could reach with its flops at the FP64
        # VALU peak (1 where the bytes bind, below 1 where the flops do)
        "apply_hbm_frac_ceiling_fp64": None if not flops else round(
            ((rule_bytes + (extra or 0.0)) / HBM_PEAK_GBS / 1e9)
            / max((rule_bytes + (extra or 0.0)) / HBM_PEAK_GBS / 1e9, flops / FP64_PEAK_TFLOPS / 1e12), 5),
        "newton_s_fp64": t64,
        "newton_s_fp32_vcycle": t32,
        "fp32_vcycle_speedup": t64 / t32,
        "gmres_iters_fp64": r64[-1]["gmres_iters"],
        "gmres_iters_fp32": r32[-1]["gmres_iters"],
        "rel_residual_fp64": r64[-1]["rel_residual"],
        "rel_residual_fp32": r32[-1]["rel_residual"],
        "dU_fp32_vs_fp64_rel": dU_err,
        "n_active": r64[-1]["n_active"],
        "stage_s_fp64": {k: r64[-1][k] for k in ("t_residual_s", "t_setup_s", "t_solve_s")},
        "roofline": roof,
        "kernels": kernels,
        "cpu_baseline": None,
        "pdas_loop": pdas_out,
        "quantities": quant,
        "p_diag": pdiag,
        "tuning_fine_level": None if tuning is None else tuning["levels"][-1]["choices"],
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(s, a.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
