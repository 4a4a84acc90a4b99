"""The PDAS loop (pf_pdas_solve), the extrapolation and the loading steps on the GPU vs the oracle.

Both sides solve each correction tightly (FGMRES to 1e-12 relative, FP64 V-cycle), so the
iterates agree to rounding carried through a few Newton corrections: the tests ask for the
same number of corrections, the same final active set and |U - U_oracle| <= 1e-7 |U|.  At
full size (64^3) the converged state is checked against the complementarity conditions
(phi <= phi^old, phi = phi^old on the active set, R = -A(U) ~ 0 on sampled free rows
evaluated by the oracle cell by cell).
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import dev, gpu_solver, host, mask_to_dofs, oracle_hierarchy, rel_err
from oracle import model, pdas

pytestmark = pytest.mark.gpu


def tight(s):
    from paper_1902_08112_amd import pff
    return gpu_solver(s, gmres_rtol=1e-12, vcycle_precision=pff.PF_F64)


@pytest.mark.parametrize("name", ["small2d", "tiny3d", "small_lshape"])
def test_pdas_loop_matches_oracle(name):
    s = W.config(name)
    print(f"[case] pdas loop {name}", flush=True)
    U0, Uold, phit = W.make_state(s)
    H = oracle_hierarchy(s)
    H.opts.gmres_rtol = 1e-12
    ref = pdas.pdas_solve(H, U0, Uold, phit, tol_as=1e-10, max_iter=30)
    S = tight(s)
    U = dev(U0)
    st, rep = S.pdas_solve(U, dev(Uold), dev(phit), max_iter=30, tol_as=1e-10)
    print(f"  oracle {ref['iterations']} corrections, GPU {rep.iterations} ({rep.gmres_iters_total} FGMRES its), "
          f"|R~| {rep.residual_norm:.1e}, |A| {rep.n_active}", flush=True)
    assert ref["converged"] and rep.converged == 1
    assert rep.iterations == ref["iterations"]
    assert rep.n_active == int(ref["active"].sum()) and rep.n_changed == 0
    assert rep.residual_norm <= 1e-10
    Ug = host(U)
    assert rel_err(Ug, ref["U"]) <= 1e-7
    d, nn = s["dim"], H.fine.n_nodes
    phi, phio = Ug[d * nn:], Uold[d * nn:]
    ok = ~H.fine.hole_node
    assert np.all(phi[ok] <= phio[ok] + 1e-12)
    assert np.allclose(phi[ref["active"]], phio[ref["active"]], atol=1e-12, rtol=0)


def test_extrapolation_kernel():
    s = W.config("small_lshape")
    S = gpu_solver(s)
    H = oracle_hierarchy(s)
    nn = H.fine.n_nodes
    rng = np.random.default_rng(7)
    p1, p2 = rng.uniform(0, 1, nn), rng.uniform(0, 1, nn)
    p1[H.fine.hole_node] = 0.0
    p2[H.fine.hole_node] = 0.0
    for theta in (1.0, 0.5, 2.0):
        out = host(S.extrapolate(dev(p1), dev(p2), theta))
        assert np.allclose(out, pdas.extrapolate(p1, p2, theta), rtol=0, atol=1e-15)


def test_loading_steps_match_oracle():
    s = W.config("small2d")
    print("[case] two loading steps small2d", flush=True)
    U0, Uold, phit = W.make_state(s)
    H = oracle_hierarchy(s)
    H.opts.gmres_rtol = 1e-12
    U1 = pdas.pdas_solve(H, U0, Uold, phit)["U"]
    S = tight(s)
    p0 = s["material"]["pressure"]
    U2g, U1g = dev(U1), dev(U1)
    U2o, U1o = U1.copy(), U1.copy()
    for n, p in enumerate([1.5 * p0, 2.0 * p0]):
        ref = pdas.time_step(H, U1o, U2o, p, first=(n == 0))
        Un, rep = S.time_step(U1g, U2g, p, first=(n == 0))
        print(f"  step {n}: oracle {ref['iterations']} corrections |A| {int(ref['active'].sum())}, "
              f"GPU {rep.iterations} |A| {rep.n_active}", flush=True)
        assert rep.converged == 1 and rep.iterations == ref["iterations"]
        assert rep.n_active == int(ref["active"].sum())
        assert rel_err(host(Un), ref["U"]) <= 1e-7
        U2o, U1o = U1o, ref["U"]
        U2g, U1g = U1g, Un


def test_pdas_loop_full_size_kkt():
    """64^3 Q1: the loop converges and the result satisfies the complementarity conditions."""
    s = W.config("cfg2_3d_q1_64")
    print("[case] pdas loop cfg2_3d_q1_64", flush=True)
    U0, Uold, phit = W.make_state(s)
    S = gpu_solver(s)
    U = dev(U0)
    st, rep = S.pdas_solve(U, dev(Uold), dev(phit), max_iter=50, tol_as=1e-10)
    print(f"  {rep.iterations} corrections, {rep.gmres_iters_total} FGMRES its, |R~| {rep.residual_norm:.1e}, "
          f"|A| {rep.n_active}, {rep.t_total_s:.3f} s", flush=True)
    assert rep.converged == 1 and rep.residual_norm <= 1e-10
    H = oracle_hierarchy(s)
    fine, d, nn = H.fine, s["dim"], H.fine.n_nodes
    Ug = host(U)
    phi, phio = Ug[d * nn:], Uold[d * nn:]
    ok = ~fine.hole_node
    assert np.all(phi[ok] <= phio[ok] + 1e-12)
    # the active set at the converged state: the library's own decision
    R = S.residual(U, dev(phit))
    act, v, n_act = S.active_set(R, U, dev(Uold))
    A = host(act).astype(bool)
    assert int(A.sum()) == rep.n_active
    assert np.allclose(phi[A], phio[A], atol=1e-12, rtol=0)
    # R = -A(U) on sampled free rows, evaluated by the oracle cell by cell: at rounding level
    # compared with the residual's scale on the constrained rows (the multipliers)
    mat = model.Material(**s["material"])
    cons = H.level_constraints(len(H.levels) - 1, A)
    free = np.flatnonzero(~cons)
    rows = np.random.default_rng(3).choice(free, 400, replace=False)
    Rs = -model.residual_rows(fine, mat, Ug, phit, rows)
    scale = np.abs(host(R)).max()
    print(f"  max |R| on sampled free rows {np.abs(Rs).max():.2e}, max |R| overall {scale:.2e}", flush=True)
    assert np.abs(Rs).max() <= 1e-9 * max(1.0, scale)
