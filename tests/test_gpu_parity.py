"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle, element by element.

Tolerances: FP64 operators agree with the oracle to 1e-12 relative (normwise,
and per block); FP32 operators to 2e-6 relative (FP32 rounding of O(1e2)
terms); masks, injected data and active sets bit-exact (active sets outside
the rounding band |v| <= 1e-10 max|v|).
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import (EIG_DUMMY, block_rel_errs, dev, gpu_solver, host, inject_bounds, mask_to_dofs, oracle_hierarchy,
                        oracle_residual_of, rel_err)
from oracle import model

pytestmark = pytest.mark.gpu

APPLY_CASES = ["tiny2d", "tiny2d_q2", "tiny3d", "tiny3d_q2", "small2d", "small3d", "small3d_q2", "small_lshape",
               "cfg1_2d_q1_32"]


def setup_case(name, seed=1, active_frac=0.1):
    print(f"[case] {name} seed={seed}", flush=True)
    s = W.config(name)
    U, phit = W.random_linearization(s, seed)
    act = W.random_active(s, seed + 1, active_frac)
    H = oracle_hierarchy(s)
    H.set_linearization(U, phit, act, eig_bounds=[EIG_DUMMY] * s["n_levels"])
    S = gpu_solver(s)
    S.set_linearization(dev(U), dev(phit), dev(act))
    return s, U, phit, act, H, S


@pytest.mark.parametrize("name", APPLY_CASES)
def test_apply_f64_all_levels(name):
    s, U, phit, act, H, S = setup_case(name)
    torch = __import__("torch")
    for l in range(s["n_levels"]):
        n = H.levels[l].n_dofs
        x = np.random.default_rng(100 + l).uniform(-1, 1, n)
        ref = H.mg[l].G @ x
        y = host(S.jacobian_apply(l, dev(x)))
        torch.cuda.synchronize()
        e = rel_err(y, ref)
        be = block_rel_errs(y, ref, H.levels[l].n_nodes, s["dim"])
        print(f"  level {l}: rel {e:.2e} per block {be}", flush=True)
        assert e <= 1e-12 and max(be.values()) <= 1e-12
        # constrained rows are the identity
        c = H.mg[l].constrained
        assert np.array_equal(y[c], x[c])


@pytest.mark.parametrize("name", ["cfg1_2d_q1_32", "small3d", "small_lshape"])
def test_apply_every_kernel_variant(name):
    """Each Q1 cell-loop shape the autotuner can pick (atomic, split cells, LDS bricks with
    ragged edge bricks, 8x8 / 16x4 marching tiles and 16x16 LDS-staged slabs with full and ragged
    chunks) matches the oracle, in both operators and precisions."""
    from paper_1902_08112_amd import pff
    s, U, phit, act, H, S = setup_case(name, seed=29)
    torch = __import__("torch")
    variants = [(2, -1), (3, -1), (4, -1), (0, 8), (0, 3), (0, 1)] + (
        [(1, 8), (1, 5), (5, 16), (5, 3), (5, 1)] if s["dim"] == 3 else [])
    for l in range(s["n_levels"]):
        x = np.random.default_rng(300 + l).uniform(-1, 1, H.levels[l].n_dofs)
        refG, refB = H.mg[l].G @ x, H.mg[l].B @ x
        for v, zc in variants:
            for mode in (0, 1):
                pff.pf_set_tuning(S.ctx, l, pff.PF_F64, mode, v, zc)
                pff.pf_set_tuning(S.ctx, l, pff.PF_F32, mode, v, zc)
            y = host(S.jacobian_apply(l, dev(x)))
            yb = host(S.block_apply(l, dev(x)))
            y32 = host(S.jacobian_apply(l, dev(x).to(torch.float32))).astype(np.float64)
            yb32 = host(S.block_apply(l, dev(x).to(torch.float32))).astype(np.float64)
            e, eb, e32, eb32 = rel_err(y, refG), rel_err(yb, refB), rel_err(y32, refG), rel_err(yb32, refB)
            print(f"  level {l} variant {v} zc {zc}: {e:.1e} {eb:.1e} FP32 {e32:.1e} {eb32:.1e}", flush=True)
            assert e <= 1e-12 and eb <= 1e-12 and e32 <= 2e-6 and eb32 <= 2e-6


@pytest.mark.parametrize("name", ["small2d", "small3d", "small_lshape", "small3d_q2"])
def test_block_apply_follows_pressure(name):
    """B~ on Q1 and 3D Q2 levels reads its phase-field coefficient (which holds 2 p div u) from a
    per-level array written at the linearization; a pressure set afterwards reaches the next
    apply, in every shape and both precisions, as it reaches G~."""
    from paper_1902_08112_amd import pff
    s, U, phit, act, H, S = setup_case(name, seed=37)
    torch = __import__("torch")
    p2 = 100.0 * s["material"]["pressure"] + 0.1
    s2 = dict(s, material=dict(s["material"], pressure=p2))
    H2 = oracle_hierarchy(s2)
    H2.set_linearization(U, phit, act, eig_bounds=[EIG_DUMMY] * s["n_levels"])
    S.set_pressure(p2)
    variants = [(2, -1), (4, -1), (0, 4)] + ([(3, -1), (1, 4), (5, 4)] if s["dim"] == 3 else [])
    for l in range(s["n_levels"]):
        x = np.random.default_rng(400 + l).uniform(-1, 1, H.levels[l].n_dofs)
        refG, refB, oldB = H2.mg[l].G @ x, H2.mg[l].B @ x, H.mg[l].B @ x
        nd = s["dim"] * H.levels[l].n_nodes
        # the pressure moves B~ far beyond the FP64 bar on this state (a stale coefficient fails)
        assert rel_err(refB[nd:], oldB[nd:]) > 1e-8
        for v, zc in variants:
            for mode in (0, 1):
                pff.pf_set_tuning(S.ctx, l, pff.PF_F64, mode, v, zc)
                pff.pf_set_tuning(S.ctx, l, pff.PF_F32, mode, v, zc)
            yb = host(S.block_apply(l, dev(x)))
            yb32 = host(S.block_apply(l, dev(x).to(torch.float32))).astype(np.float64)
            y = host(S.jacobian_apply(l, dev(x)))
            e, eb, eb32 = rel_err(y, refG), rel_err(yb, refB), rel_err(yb32, refB)
            print(f"  level {l} variant {v} zc {zc}: G {e:.1e} B {eb:.1e} B FP32 {eb32:.1e}", flush=True)
            assert e <= 1e-12 and eb <= 1e-12 and eb32 <= 2e-6


def test_kernel_timing_records():
    """pf_set_kernel_timing brackets the finest-level FP64 launches of G~ and of B~ in a Newton
    step (all, or every k-th); the records count what they saw and what they timed, and bad
    arguments fail before anything is recorded."""
    from paper_1902_08112_amd import pff
    s = W.config("small3d")
    print("[case] kernel timing small3d", flush=True)
    U, Uold, phit = W.make_state(s)
    S = gpu_solver(s)
    S.set_vcycle_precision(pff.PF_F64)
    for every in (1, 3):
        S.set_kernel_timing(pff.PF_KTIME_JACOBIAN | pff.PF_KTIME_BLOCK, every=every)
        S.newton_step(dev(U), dev(Uold), dev(phit))
        S.set_kernel_timing(False)
        for op in (pff.PF_KTIME_JACOBIAN, pff.PF_KTIME_BLOCK):
            seen, n, mean, lo, hi = S.kernel_timing(op, launches=True)
            print(f"  every {every} op {op}: {seen} launches, {n} timed, mean {mean * 1e6:.1f} us", flush=True)
            assert seen > 0 and n == (seen + every - 1) // every
            assert 0.0 < lo <= mean <= hi
    # only the Jacobian record
    S.set_kernel_timing(pff.PF_KTIME_JACOBIAN)
    S.newton_step(dev(U), dev(Uold), dev(phit))
    S.set_kernel_timing(False)
    assert S.kernel_timing(pff.PF_KTIME_JACOBIAN)[0] > 0 and S.kernel_timing(pff.PF_KTIME_BLOCK)[0] == 0
    for bad in (dict(enable=8), dict(enable=-1), dict(enable=1, every=0)):
        with pytest.raises(pff.PffError):
            S.set_kernel_timing(**bad)


def test_autotune_report_and_cache(tmp_path):
    from paper_1902_08112_amd import pff
    s, U, phit, act, H, S = setup_case("small3d", seed=31)
    rep = S.autotune(reps=3, cache_path=str(tmp_path / "tune.json"))
    assert len(rep["levels"]) == s["n_levels"]
    for lv in rep["levels"]:
        for ch in lv["choices"]:
            assert ch["variant"] in (0, 1, 2, 3, 4, 5)
            times = [t for v, z, t in ch["us"] if t > 0]
            assert len(times) >= 4 and min(times) > 0
            if ch["mode"] == "block":
                # the fused-smoother choice is timed exactly on the marching-tile levels
                assert ch["fused"] in (0, 1)
                tiled = ch["variant"] in (0, 1, 5)
                assert (min(ch["step_us"]) > 0) == tiled
                assert ch["fused"] == 0 or ch["step_us"][1] < ch["step_us"][0]
    # cached choices are restored without timing
    S2 = gpu_solver(s)
    S2.set_linearization(dev(U), dev(phit), dev(act))
    rep2 = S2.autotune(reps=3, cache_path=str(tmp_path / "tune.json"))
    for a, b in zip(rep["levels"], rep2["levels"]):
        assert [c["variant"] for c in a["choices"]] == [c["variant"] for c in b["choices"]]
        assert [c.get("fused") for c in a["choices"]] == [c.get("fused") for c in b["choices"]]
    x = np.random.default_rng(5).uniform(-1, 1, H.fine.n_dofs)
    assert rel_err(host(S2.jacobian_apply(-1, dev(x))), H.mg[-1].G @ x) <= 1e-12


@pytest.mark.parametrize("name", APPLY_CASES)
def test_block_apply_f64(name):
    s, U, phit, act, H, S = setup_case(name, seed=3)
    l = s["n_levels"] - 1
    x = np.random.default_rng(7).uniform(-1, 1, H.levels[l].n_dofs)
    ref = H.mg[l].B @ x
    y = host(S.block_apply(l, dev(x)))
    assert rel_err(y, ref) <= 1e-12


@pytest.mark.parametrize("name", ["tiny3d", "small2d", "small3d_q2", "small_lshape"])
def test_apply_f32(name):
    s, U, phit, act, H, S = setup_case(name, seed=5)
    torch = __import__("torch")
    for l in range(s["n_levels"]):
        x = np.random.default_rng(200 + l).uniform(-1, 1, H.levels[l].n_dofs)
        ref = H.mg[l].G @ x
        y = host(S.jacobian_apply(l, dev(x).to(torch.float32))).astype(np.float64)
        e = rel_err(y, ref)
        print(f"  level {l}: FP32 rel {e:.2e}", flush=True)
        assert e <= 2e-6


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d_q2", "small3d", "small_lshape", "cfg1_2d_q1_32"])
def test_residual_f64(name):
    s, U, phit, act, H, S = setup_case(name, seed=11)
    fine = H.fine
    ref = -model.assemble_residual(fine, H.mat, U, phit)
    R = host(S.residual(dev(U), dev(phit)))
    assert rel_err(R, ref) <= 1e-12
    assert max(block_rel_errs(R, ref, fine.n_nodes, s["dim"]).values()) <= 1e-12


@pytest.mark.parametrize("name", ["tiny2d_q2", "tiny3d", "small3d_q2", "small_lshape"])
def test_diagonal_and_level_data(name):
    s, U, phit, act, H, S = setup_case(name, seed=13)
    d = s["dim"]
    for l in range(s["n_levels"]):
        diag = host(S.diagonal(l))
        ref = H.mg[l].D
        assert rel_err(diag, ref) <= 1e-12, l
        Ul, pl, mk = S.level_data(l)
        assert np.array_equal(host(Ul), H.mg[l].U)      # injection is a copy: bit-exact
        assert np.array_equal(host(pl), H.mg[l].phit)
        assert np.array_equal(mask_to_dofs(host(mk), d), H.mg[l].constrained)


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d_q2", "small_lshape"])
def test_lumped_mass(name):
    s, U, phit, act, H, S = setup_case(name)
    M = host(S.lumped_mass())
    assert rel_err(M, model.lumped_mass(H.fine)) <= 1e-14


@pytest.mark.parametrize("name", ["tiny2d_q2", "small3d", "small3d_q2"])
def test_transfers(name):
    from oracle import mg
    s, U, phit, act, H, S = setup_case(name)
    for l in range(1, s["n_levels"]):
        cf, ff = H.levels[l - 1], H.levels[l]
        P = mg.prolongation(cf, ff)
        xf = np.random.default_rng(l).uniform(-1, 1, ff.n_dofs)
        xc = np.random.default_rng(50 + l).uniform(-1, 1, cf.n_dofs)
        assert rel_err(host(S.transfer(l, 0, dev(xf))), P.T @ xf) <= 1e-14
        assert rel_err(host(S.transfer(l, 1, dev(xc))), P @ xc) <= 1e-14
        inj = mg.inject_nodal(cf, ff, xf, s["dim"] + 1)
        assert np.array_equal(host(S.transfer(l, 2, dev(xf))), inj)


@pytest.mark.parametrize("name", ["cfg1_2d_q1_32", "small3d_q2", "small_lshape"])
def test_active_set(name):
    from oracle import newton
    print(f"[case] active set {name}", flush=True)
    s = W.config(name)
    H = oracle_hierarchy(s)
    U, Uold, phit = W.make_state(s)
    act_ref, v_ref, R_ref = newton.active_set(H.fine, H.mat, U, Uold, phit)
    S = gpu_solver(s)
    R = S.residual(dev(U), dev(phit))
    act, v, n = S.active_set(R, dev(U), dev(Uold))
    v = host(v)
    act = host(act).astype(bool)
    assert rel_err(v, v_ref) <= 1e-11
    band = np.abs(v_ref) <= 1e-10 * np.abs(v_ref).max()
    assert np.array_equal(act[~band], act_ref[~band])
    print(f"  |A| = {n} (oracle {act_ref.sum()}), excluded ties {band.sum()}", flush=True)
    assert abs(n - act_ref.sum()) <= band.sum()


@pytest.mark.parametrize("name", ["small2d", "tiny3d_q2", "small_lshape"])
def test_eigenvalue_estimates(name):
    """The eigenvalue CG runs in each level's V-cycle precision: with FP64 V-cycles every level
    matches the oracle's CG-Lanczos (same SplitMix64 start vectors) to 1e-8; with FP32 V-cycles
    the coarsest level still does, and the FP32 CGs of the other levels to 1e-4 (FP32 vectors,
    FP64 dots and coefficients)."""
    from paper_1902_08112_amd import PF_F32, PF_F64
    s, U, phit, act, H, S = setup_case(name, seed=17)
    H.set_linearization(U, phit, act)       # oracle CG-Lanczos with the same SplitMix64 start vectors
    for prec in (PF_F64, PF_F32):
        S.set_vcycle_precision(prec)
        S.set_linearization(dev(U), dev(phit), dev(act))
        for l in range(s["n_levels"]):
            got = S.eig_bounds(l)
            e = H.mg[l].eig
            ref = [e["u"][0], e["u"][1], e["phi"][0], e["phi"][1]]
            tol = 1e-8 if (prec == PF_F64 or l == 0) else 1e-4
            print(f"  prec {prec} level {l}: gpu {np.round(got, 6)} oracle {np.round(ref, 6)}", flush=True)
            assert np.allclose(got, ref, rtol=tol)


@pytest.mark.parametrize("name", ["small2d", "tiny3d_q2", "small3d", "small_lshape"])
def test_vcycle_f64_matches_oracle(name):
    s, U, phit, act, H, S = setup_case(name, seed=19)
    H.set_linearization(U, phit, act)
    inject_bounds(S, H)
    r = np.random.default_rng(23).uniform(-1, 1, H.fine.n_dofs)
    z_ref = H.vcycle(r)
    from paper_1902_08112_amd import PF_F32, pff
    # every way of running the coarse Chebyshev solve computes the same polynomial: the dense matrix
    # formed at set-up (the default for small Q1 coarse levels), the single-workgroup kernel, and one
    # launch per step
    for mode in (pff.PF_COARSE_AUTO, pff.PF_COARSE_FUSED, pff.PF_COARSE_STEPS):
        S.set_coarse_mode(mode)
        z = host(S.vcycle(dev(r)))
        e = rel_err(z, z_ref)
        print(f"  coarse mode {mode}: vcycle rel {e:.2e}", flush=True)
        assert e <= 1e-11
    z32 = host(S.vcycle(dev(r), PF_F32))
    e32 = rel_err(z32, z_ref)
    print(f"  vcycle FP32 levels rel {e32:.2e}", flush=True)
    assert e32 <= 1e-4


@pytest.mark.parametrize("name", ["small3d", "small_lshape"])
def test_vcycle_fused_smoother_steps(name):
    """With the block operator on marching tiles on every level, the Chebyshev steps run inside
    the tile kernel: the V-cycle matches the oracle (FP64 1e-11, FP32 levels 1e-4), the unfused
    V-cycle to rounding, and a Newton step converges to the oracle's update."""
    from paper_1902_08112_amd import PF_F32, PF_F64, pff
    s, U, phit, act, H, S = setup_case(name, seed=43)
    for v, zc in [(0, 3), (1, 2), (5, 3)]:
        for l in range(s["n_levels"]):
            pff.pf_set_tuning(S.ctx, l, pff.PF_F64, 1, v, zc)
            pff.pf_set_tuning(S.ctx, l, pff.PF_F32, 1, v, zc)
        H.set_linearization(U, phit, act)
        inject_bounds(S, H)
        r = np.random.default_rng(47).uniform(-1, 1, H.fine.n_dofs)
        z_ref = H.vcycle(r)
        out = {}
        for fuse in (True, False):
            S.set_smoother_fusion(pff.PF_FUSE_ALWAYS if fuse else pff.PF_FUSE_OFF)
            S.set_kernel_timing(pff.PF_KTIME_BLOCK_CHEB)
            out[fuse] = (host(S.vcycle(dev(r))), host(S.vcycle(dev(r), PF_F32)))
            S.set_kernel_timing(False)
            seen = S.kernel_timing(pff.PF_KTIME_BLOCK_CHEB, launches=True)[0]
            print(f"  tiles {v},{zc} fused {fuse}: rel {rel_err(out[fuse][0], z_ref):.2e} FP32 "
                  f"{rel_err(out[fuse][1], z_ref):.2e}, fused launches {seen}", flush=True)
            assert (seen > 0) == fuse
            assert rel_err(out[fuse][0], z_ref) <= 1e-11 and rel_err(out[fuse][1], z_ref) <= 1e-4
        assert rel_err(out[True][0], out[False][0]) <= 1e-13
        assert rel_err(out[True][1], out[False][1]) <= 1e-6
    from oracle import newton
    U0, Uold, ph0 = W.make_state(s)
    H2 = oracle_hierarchy(s)
    ref = newton.newton_step(H2, U0, Uold, ph0)
    S2 = gpu_solver(s)
    S2.set_smoother_fusion(pff.PF_FUSE_ALWAYS)
    for l in range(s["n_levels"]):
        for prec in (pff.PF_F64, pff.PF_F32):
            pff.pf_set_tuning(S2.ctx, l, prec, 1, 0, 4)
    Ud = dev(U0)
    _, rep = S2.newton_step(Ud, dev(Uold), dev(ph0))
    e = rel_err(host(Ud) - U0, ref["dU"])
    print(f"  newton: its {rep.gmres_iters} (oracle {ref['info']['iters']}), rel {e:.1e}", flush=True)
    assert rep.converged and rep.n_active == ref["n_active"] and e <= 1e-5


@pytest.mark.parametrize("name", ["small2d", "small3d", "small3d_q2"])
def test_vcycle_graph_replay_matches_eager(name):
    """The captured V-cycle, replayed several times with eager work and synchronizations in between,
    gives the eager V-cycle's result every time (both precisions)."""
    from paper_1902_08112_amd import PF_F32, PF_F64
    s, U, phit, act, H, S = setup_case(name, seed=37)
    torch = __import__("torch")
    n = H.fine.n_dofs
    r = dev(np.random.default_rng(41).uniform(-1, 1, n))
    for prec in (PF_F64, PF_F32):
        # atomic scatter reorders sums: rounding-level differences of the working precision
        tol = 1e-12 if prec == PF_F64 else 2e-6
        S.set_graphs(False)
        z_eager = host(S.vcycle(r, prec))
        S.set_graphs(True)
        for rep in range(4):
            z = host(S.vcycle(r, prec))
            e = rel_err(z, z_eager)
            print(f"  prec {prec} replay {rep}: rel diff {e:.1e}", flush=True)
            assert e <= tol
            # eager work between replays
            S.jacobian_apply(-1, r)
            torch.cuda.synchronize()
    # a new linearization invalidates the capture: the replay follows the new data
    S.set_linearization(dev(U * 0.5), dev(phit), dev(act))
    S.set_graphs(False)
    z_eager2 = host(S.vcycle(r))
    S.set_graphs(True)
    assert rel_err(host(S.vcycle(r)), z_eager2) <= 1e-12
    # a pressure change re-captures, and B~'s stored coefficients follow it (refreshed before the
    # capture): replays and the eager V-cycle agree, and both differ from the old pressure's
    S.set_pressure(3.0 * s["material"]["pressure"] + 0.3)
    z_graph3 = [host(S.vcycle(r)) for _ in range(3)]
    S.set_graphs(False)
    z_eager3 = host(S.vcycle(r))
    for z in z_graph3:
        assert rel_err(z, z_eager3) <= 1e-12
    assert rel_err(z_eager3, z_eager2) > 1e-9


GRAPH_RELIN_CASES = [("small3d", None, 0), ("small3d", (0, 3), 1), ("small3d", (5, 3), 2), ("small_lshape", None, 1),
                     ("small3d_q2", None, 0), ("cfg1_2d_q1_32", None, 1)]


@pytest.mark.parametrize("name,tiles,coarse", GRAPH_RELIN_CASES)
def test_vcycle_graph_survives_relinearization(name, tiles, coarse):
    """One capture per precision serves every later linearization and every new eigenvalue bound
    (the kernels read level data and Chebyshev coefficients from device memory): a solver that
    replays its captured V-cycles and one that launches eagerly, given the same linearizations
    (new U, phi~ and active set each time) and injected bounds, agree after each, and the replay
    after the last one matches the oracle's V-cycle with the oracle's bounds.  A coarse solve whose
    operator sums cell contributions with atomics in no fixed order (the single-workgroup kernel of
    coarse mode 1, the Q2 coarse level) has its rounding-level differences amplified by the
    degree-20 Chebyshev polynomial: two eager launches, like a replay and an eager launch, then
    agree to about 1e-9 rather than 1e-12.  The dense coarse matrix of small Q1 levels (mode 0) is
    deterministic."""
    from paper_1902_08112_amd import PF_F32, PF_F64, pff
    s, U, phit, act, H, S = setup_case(name, seed=53)
    E = gpu_solver(s)
    for X in (S, E):
        X.set_coarse_mode(coarse)
        if tiles is not None:
            # marching tiles or slabs for B~ on every level, the smoother steps fused into them
            for l in range(s["n_levels"]):
                for prec in (PF_F64, PF_F32):
                    pff.pf_set_tuning(X.ctx, l, prec, 1, tiles[0], tiles[1])
            X.set_smoother_fusion(pff.PF_FUSE_ALWAYS)
    S.set_graphs(True)
    E.set_graphs(False)
    r = np.random.default_rng(59).uniform(-1, 1, H.fine.n_dofs)
    rd = dev(r)
    c0 = S.graph_captures()
    exact_coarse = coarse == 0 and s["degree"] == 1
    for k in range(4):
        Uk, phk = W.random_linearization(s, 70 + k)
        actk = W.random_active(s, 80 + k, 0.05 + 0.04 * k)
        for X in (S, E):
            X.set_linearization(dev(Uk), dev(phk), dev(actk))
        if k == 2:
            # bounds injected on the finest level (wider interval): device coefficients change
            b = E.eig_bounds(-1)
            wide = [b[0], 1.25 * b[1], b[2], 1.25 * b[3]]
            for X in (S, E):
                X.set_eig_bounds(-1, wide)
        if k == 3:
            H.set_linearization(Uk, phk, actk)
            inject_bounds(S, H)
            inject_bounds(E, H)
        for prec, tol in ((PF_F64, 1e-12 if exact_coarse else 5e-9), (PF_F32, 2e-6)):
            z_e = host(E.vcycle(rd, prec))
            print(f"  linearization {k} prec {prec}: two eager launches differ by "
                  f"{rel_err(host(E.vcycle(rd, prec)), z_e):.1e}", flush=True)
            for rep in range(2):
                z = host(S.vcycle(rd, prec))
                e = rel_err(z, z_e)
                print(f"  linearization {k} prec {prec} replay {rep}: rel diff to eager {e:.1e}", flush=True)
                assert e <= tol
    z_ref = H.vcycle(r)
    e = rel_err(host(S.vcycle(rd)), z_ref)
    print(f"  replay after the last linearization vs oracle: {e:.1e}; captures {S.graph_captures() - c0}",
          flush=True)
    assert e <= (1e-11 if exact_coarse else 5e-9)
    # the first V-cycle of each precision captured; every later linearization replayed
    assert S.graph_captures() - c0 == 2
    assert E.graph_captures() == 0


@pytest.mark.parametrize("name,prec", [("cfg1_2d_q1_32", "f64"), ("cfg1_2d_q1_32", "f32"), ("small3d", "f64"),
                                       ("small3d_q2", "f32"), ("small_lshape", "f32")])
def test_newton_step_matches_oracle(name, prec):
    from oracle import newton
    print(f"[case] newton {name} {prec}", flush=True)
    s = dict(W.config(name))
    s["vcycle"] = prec
    U, Uold, phit = W.make_state(s)
    H = oracle_hierarchy(s)
    ref = newton.newton_step(H, U, Uold, phit)
    S = gpu_solver(s)
    Ud = dev(U)
    st, rep = S.newton_step(Ud, dev(Uold), dev(phit))
    Un = host(Ud)
    dU = Un - U
    e = rel_err(dU, ref["dU"])
    print(f"  gmres {rep.gmres_iters} (oracle {ref['info']['iters']}), rel res {rep.rel_residual:.2e}, "
          f"|A| {rep.n_active} (oracle {ref['n_active']}), |dU - dU_oracle|/|dU_oracle| = {e:.2e}", flush=True)
    assert rep.converged and rep.rel_residual <= 1e-8
    # both solves reach 1e-8 of the same linear system: the solutions agree to ~cond * 1e-8
    assert e <= 1e-5
    # the oracle's own matrices confirm the library's residual claim
    assert rep.n_active == ref["n_active"]
    res = oracle_residual_of(ref, dU)
    print(f"  oracle residual of the GPU update {res:.2e}", flush=True)
    assert res <= 1.1e-8
    if prec == "f64":
        assert abs(rep.gmres_iters - ref["info"]["iters"]) <= 1
    d, nn = s["dim"], H.fine.n_nodes
    act = ref["active"]
    assert np.allclose(Un[d * nn:][act], Uold[d * nn:][act], atol=1e-12)
