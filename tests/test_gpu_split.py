"""The Miehe spectral split (Sec. 2.1) on the GPU vs the oracle's split.

Same bars as the unsplit operators: FP64 applies, block applies, residuals and diagonals
to 1e-12 relative on every level, FP32 applies to 2e-6, the FP64 V-cycle to 1e-11, the
FP32-level cycle to 1e-4, energies and face loads to 1e-12.  Newton steps solved to 1e-8
on both sides agree to 1e-5; the PDAS loop (tight solves) takes the same number of
corrections and ends at the same active set, |U - U_oracle| <= 1e-7 |U|.  Each case also
checks that the split changes the operator (the states are not all-tension or
all-compression, where the split and the unsplit forms coincide).
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import EIG_DUMMY, block_rel_errs, dev, gpu_solver, host, inject_bounds, oracle_hierarchy, rel_err
from oracle import model, pdas, quantities

pytestmark = pytest.mark.gpu

CASES = ["tiny2d_miehe", "tiny2d_q2_miehe", "tiny3d_miehe", "tiny3d_q2_miehe", "small3d_miehe",
         "small_lshape_miehe", "cfg1_2d_q1_32_miehe"]


def setup_case(name, seed=1, active_frac=0.1):
    print(f"[case] split {name} seed={seed}", flush=True)
    s = W.config(name)
    U, phit = W.random_linearization(s, seed)
    act = W.random_active(s, seed + 1, active_frac)
    H = oracle_hierarchy(s)
    H.set_linearization(U, phit, act, eig_bounds=[EIG_DUMMY] * s["n_levels"])
    S = gpu_solver(s)
    S.set_linearization(dev(U), dev(phit), dev(act))
    return s, U, phit, act, H, S


@pytest.mark.parametrize("name", CASES)
def test_split_apply_all_levels(name):
    s, U, phit, act, H, S = setup_case(name)
    torch = __import__("torch")
    plain = model.Material(**dict(s["material"], split="none"))
    for l in range(s["n_levels"]):
        lev = H.levels[l]
        x = np.random.default_rng(100 + l).uniform(-1, 1, lev.n_dofs)
        ref, refB = H.mg[l].G @ x, H.mg[l].B @ x
        y = host(S.jacobian_apply(l, dev(x)))
        yb = host(S.block_apply(l, dev(x)))
        y32 = host(S.jacobian_apply(l, dev(x).to(torch.float32))).astype(np.float64)
        e, eb, e32 = rel_err(y, ref), rel_err(yb, refB), rel_err(y32, ref)
        be = block_rel_errs(y, ref, lev.n_nodes, s["dim"])
        print(f"  level {l}: rel {e:.2e} block {eb:.2e} FP32 {e32:.2e} per block {be}", flush=True)
        assert e <= 1e-12 and eb <= 1e-12 and max(be.values()) <= 1e-12 and e32 <= 2e-6
        c = H.mg[l].constrained
        assert np.array_equal(y[c], x[c])
    # the split is active on this state
    G0 = model.constrain_matrix(model.assemble_jacobian(H.fine, plain, H.mg[-1].U, H.mg[-1].phit),
                                H.mg[-1].constrained)
    assert rel_err(G0 @ x, ref) > 1e-4


@pytest.mark.parametrize("name", ["small2d_miehe", "small3d_miehe", "small_lshape_miehe"])
def test_split_apply_every_shape(name):
    """Both Q1 shapes of the split apply from the stored eigen-records (one work item per cell,
    variant 2; displacement and phase-field rows in two wavefronts, variant 4), both operators,
    both precisions, every level."""
    from paper_1902_08112_amd import pff
    s, U, phit, act, H, S = setup_case(name, seed=29)
    torch = __import__("torch")
    for l in range(s["n_levels"]):
        x = np.random.default_rng(300 + l).uniform(-1, 1, H.levels[l].n_dofs)
        refG, refB = H.mg[l].G @ x, H.mg[l].B @ x
        for v in (2, 4):
            for mode in (0, 1):
                pff.pf_set_tuning(S.ctx, l, pff.PF_F64, mode, v, -1)
                pff.pf_set_tuning(S.ctx, l, pff.PF_F32, mode, v, -1)
            y = host(S.jacobian_apply(l, dev(x)))
            yb = host(S.block_apply(l, dev(x)))
            y32 = host(S.jacobian_apply(l, dev(x).to(torch.float32))).astype(np.float64)
            yb32 = host(S.block_apply(l, dev(x).to(torch.float32))).astype(np.float64)
            e, eb, e32, eb32 = rel_err(y, refG), rel_err(yb, refB), rel_err(y32, refG), rel_err(yb32, refB)
            print(f"  level {l} shape {v}: {e:.1e} {eb:.1e} FP32 {e32:.1e} {eb32:.1e}", flush=True)
            assert e <= 1e-12 and eb <= 1e-12 and e32 <= 2e-6 and eb32 <= 2e-6


@pytest.mark.parametrize("name", ["small2d_miehe", "small3d_miehe"])
def test_split_broken_tension_rows(name):
    """Every point fully broken (phi~ = 0) and in tension (all principal strains and tr e positive):
    there C^+ = C and sigma^+ = sigma, so the split operator equals the unsplit one, whose
    displacement rows are kappa C, ten orders below an undamaged row (Sec. 2.1).  The reference is
    the unsplit oracle's assembled Jacobian, which forms g C directly.  Written as
    C - (1 - g) C^+, the displacement tangent there would be a difference of two O(|C|) terms that
    FP32 rounding swamps; the record-streaming kernels form it as one spectral sum with weights
    g F + (1 - F), so both record shapes, both operators and both precisions meet the usual bars
    on the unconstrained displacement rows alone (the constrained rows return x and would hide
    them).  The split oracle itself, which forms C - (1 - g) C^+ in FP64, is printed for
    comparison: its cancellation leaves about 1e-6 on these rows."""
    from paper_1902_08112_amd import pff
    torch = __import__("torch")
    s = W.config(name)
    d = s["dim"]
    print(f"[case] split broken tension {name}", flush=True)
    _, X = W.lattice(s)
    nn = X.shape[0]
    rng = np.random.default_rng(5)
    U = np.zeros((d + 1) * nn)
    for c in range(d):
        # principal strains about 1e-3 (1, 1.1, 1.2); the perturbation keeps them positive and distinct
        U[c * nn:(c + 1) * nn] = 1e-3 * (1 + 0.1 * c) * X[:, c] + 1e-7 * rng.uniform(-1, 1, nn)
    U[d * nn:] = rng.uniform(0, 1, nn)
    phit = np.zeros(nn)
    act = np.zeros(nn, dtype=np.uint8)
    H = oracle_hierarchy(s)
    H.set_linearization(U, phit, act, eig_bounds=[EIG_DUMMY] * s["n_levels"])
    plain = model.Material(**dict(s["material"], split="none"))
    mg_f = H.mg[-1]
    G0 = model.constrain_matrix(model.assemble_jacobian(H.fine, plain, mg_f.U, mg_f.phit), mg_f.constrained)
    S = gpu_solver(s)
    S.set_linearization(dev(U), dev(phit), dev(act))
    L = s["n_levels"] - 1
    x = np.random.default_rng(7).uniform(-1, 1, H.fine.n_dofs)
    ref = G0 @ x
    rows = np.flatnonzero(~mg_f.constrained[:d * nn])
    e_or = rel_err((mg_f.G @ x)[rows], ref[rows])
    print(f"  {rows.size} free displacement rows, |G x| there {np.linalg.norm(ref[rows]):.1e}; split oracle "
          f"(C - (1 - g) C^+ in FP64) vs unsplit oracle there: {e_or:.1e}", flush=True)
    for v in (2, 4):
        for mode in (0, 1):
            pff.pf_set_tuning(S.ctx, L, pff.PF_F64, mode, v, -1)
            pff.pf_set_tuning(S.ctx, L, pff.PF_F32, mode, v, -1)
        for op, tag in ((S.jacobian_apply, "G"), (S.block_apply, "B")):
            y = host(op(L, dev(x)))
            y32 = host(op(L, dev(x).to(torch.float32))).astype(np.float64)
            e, e32 = rel_err(y[rows], ref[rows]), rel_err(y32[rows], ref[rows])
            print(f"  shape {v} {tag}: displacement rows FP64 {e:.1e} FP32 {e32:.1e}", flush=True)
            assert e <= 1e-12 and e32 <= 2e-6
            if tag == "G":
                assert rel_err(y, ref) <= 1e-12


@pytest.mark.parametrize("name", ["tiny2d_miehe", "tiny3d_q2_miehe", "small3d_miehe", "small_lshape_miehe"])
def test_split_residual_and_diagonal(name):
    s, U, phit, act, H, S = setup_case(name, seed=11)
    fine = H.fine
    ref = -model.assemble_residual(fine, H.mat, U, phit)
    R = host(S.residual(dev(U), dev(phit)))
    e = rel_err(R, ref)
    print(f"  residual rel {e:.2e}", flush=True)
    assert e <= 1e-12 and max(block_rel_errs(R, ref, fine.n_nodes, s["dim"]).values()) <= 1e-12
    for l in range(s["n_levels"]):
        ed = rel_err(host(S.diagonal(l)), H.mg[l].D)
        print(f"  level {l}: diagonal rel {ed:.2e}", flush=True)
        assert ed <= 1e-12


@pytest.mark.parametrize("name", ["small2d_miehe", "tiny3d_q2_miehe", "small3d_miehe", "small_lshape_miehe"])
def test_split_vcycle_matches_oracle(name):
    from paper_1902_08112_amd import PF_F32
    s, U, phit, act, H, S = setup_case(name, seed=19)
    H.set_linearization(U, phit, act)
    inject_bounds(S, H)
    r = np.random.default_rng(23).uniform(-1, 1, H.fine.n_dofs)
    z_ref = H.vcycle(r)
    e = rel_err(host(S.vcycle(dev(r))), z_ref)
    e32 = rel_err(host(S.vcycle(dev(r), PF_F32)), z_ref)
    print(f"  vcycle rel {e:.2e}, FP32 levels {e32:.2e}", flush=True)
    assert e <= 1e-11 and e32 <= 1e-4


@pytest.mark.parametrize("name,prec", [("cfg1_2d_q1_32_miehe", "f64"), ("small3d_miehe", "f32"),
                                       ("small_lshape_miehe", "f32"), ("tiny3d_q2_miehe", "f64")])
def test_split_newton_step_matches_oracle(name, prec):
    from oracle import newton
    print(f"[case] split newton {name} {prec}", flush=True)
    s = dict(W.config(name))
    s["vcycle"] = prec
    U, Uold, phit = W.make_state(s)
    H = oracle_hierarchy(s)
    ref = newton.newton_step(H, U, Uold, phit)
    S = gpu_solver(s)
    Ud = dev(U)
    _, rep = S.newton_step(Ud, dev(Uold), dev(phit))
    e = rel_err(host(Ud) - U, ref["dU"])
    print(f"  gmres {rep.gmres_iters} (oracle {ref['info']['iters']}), rel res {rep.rel_residual:.2e}, "
          f"|A| {rep.n_active} (oracle {ref['n_active']}), rel {e:.2e}", flush=True)
    assert rep.converged and rep.rel_residual <= 1e-8
    assert rep.n_active == ref["n_active"]
    assert e <= 1e-5


@pytest.mark.parametrize("name", ["small2d_miehe", "tiny3d_miehe"])
def test_split_pdas_loop_matches_oracle(name):
    from paper_1902_08112_amd import pff
    s = W.config(name)
    print(f"[case] split pdas loop {name}", flush=True)
    U0, Uold, phit = W.make_state(s)
    H = oracle_hierarchy(s)
    H.opts.gmres_rtol = 1e-12
    ref = pdas.pdas_solve(H, U0, Uold, phit, tol_as=1e-10, max_iter=30)
    S = gpu_solver(s, gmres_rtol=1e-12, vcycle_precision=pff.PF_F64)
    U = dev(U0)
    _, rep = S.pdas_solve(U, dev(Uold), dev(phit), max_iter=30, tol_as=1e-10)
    print(f"  oracle {ref['iterations']} corrections, GPU {rep.iterations} ({rep.gmres_iters_total} FGMRES its), "
          f"|R~| {rep.residual_norm:.1e}", flush=True)
    assert ref["converged"] and rep.converged == 1
    assert rep.iterations == ref["iterations"]
    assert rep.n_active == int(ref["active"].sum())
    assert rel_err(host(U), ref["U"]) <= 1e-7


@pytest.mark.parametrize("name", ["small2d_miehe", "tiny2d_q2_miehe", "small3d_miehe", "small_lshape_miehe"])
def test_split_quantities_match_oracle(name):
    s = W.config(name)
    print(f"[case] split quantities {name}", flush=True)
    mat = model.Material(**s["material"])
    H = oracle_hierarchy(s)
    S = gpu_solver(s)
    for U in (W.make_state(s)[0], W.random_linearization(s, 41)[0]):
        dU = dev(U)
        ec, eb = S.energies(dU)
        rc, rb = quantities.energies(H.fine, mat, U)
        print(f"  energies GPU ({ec:.12e}, {eb:.12e}) oracle ({rc:.12e}, {rb:.12e})", flush=True)
        assert abs(ec - rc) <= 1e-12 * abs(rc) and abs(eb - rb) <= 1e-12 * abs(rb)
        ref = [quantities.boundary_traction(H.fine, mat, U, f) for f in range(2 * s["dim"])]
        scale = max(np.abs(r).max() for r in ref)
        for f in range(2 * s["dim"]):
            t = np.array(S.boundary_traction(dU, f))
            assert np.abs(t - ref[f]).max() <= 1e-12 * scale, (f, t, ref[f])
