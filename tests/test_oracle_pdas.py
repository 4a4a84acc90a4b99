"""Pins of the oracle's PDAS loop and time step (Algorithm 1 repeated to convergence, Sec. 3.1).

The converged state is checked against the discrete complementarity (KKT)
conditions of the irreversibility-constrained problem, recomputed here from the
residual alone, not from the loop's own bookkeeping:
  * phi <= phi^old on every domain node (irreversibility),
  * phi = phi^old on the active set,
  * R = -A(U) vanishes on every free DoF (displacements off the Dirichlet set,
    phase-field DoFs off the active set),
  * the multiplier R_phi / M is positive on the active set (the sign the
    active-set rule selects).
The extrapolation is pinned by exactness on functions linear in time.
"""
import numpy as np
import pytest

import workloads as W
from oracle import mg, model, pdas


def setup(name):
    s = W.config(name)
    mat = model.Material(**s["material"])
    U, Uold, phit = W.make_state(s)
    H = mg.Hierarchy(s["dim"], s["degree"], s["n_cells"], s["extent"], s["domain"], s["n_levels"], s["faces"], mat)
    return s, H, U, Uold, phit


def check_kkt(H, U, Uold, phit, active, tol):
    fine = H.fine
    d, nn = fine.d, fine.n_nodes
    ok = ~fine.hole_node
    phi, phio = U[d * nn:], Uold[d * nn:]
    assert np.all(phi[ok] <= phio[ok] + 1e-12)
    assert np.allclose(phi[active], phio[active], atol=1e-12, rtol=0)
    R = -model.assemble_residual(fine, H.mat, U, phit)
    cons = H.level_constraints(len(H.levels) - 1, active)
    assert np.linalg.norm(R[~cons]) <= tol
    M = model.lumped_mass(fine)
    assert np.all(R[d * nn:][active] / M[active] > 0.0)


def test_extrapolation_reproduces_linear_in_time():
    rng = np.random.default_rng(0)
    a, b = rng.uniform(-1, 1, 50), rng.uniform(-1, 1, 50)
    t2, t1, t0 = 0.3, 0.45, 0.7          # t_{n-2}, t_{n-1}, t_n (uneven steps)
    phi = lambda t: a + b * t
    theta = (t0 - t1) / (t1 - t2)
    assert np.allclose(pdas.extrapolate(phi(t1), phi(t2), theta), phi(t0), atol=1e-14, rtol=0)
    # constant time step: 2 phi^{n-1} - phi^{n-2}
    assert np.array_equal(pdas.extrapolate(phi(t1), phi(t2)), phi(t1) + (phi(t1) - phi(t2)))


@pytest.mark.parametrize("name", ["tiny2d", "small2d", "tiny3d"])
def test_pdas_converged_state_is_a_kkt_point(name):
    s, H, U, Uold, phit = setup(name)
    out = pdas.pdas_solve(H, U, Uold, phit, tol_as=1e-10, max_iter=30, solver="dense")
    assert out["converged"]
    last = out["history"][-1]
    assert last["n_changed"] == 0 and last["rt_norm"] <= 1e-10
    assert out["iterations"] == len(out["history"]) - 1
    check_kkt(H, out["U"], Uold, phit, out["active"], 1e-9)
    # the active set changes until the last iteration (the loop is not trivially short)
    assert all(h["n_changed"] != 0 for h in out["history"][1:-1])


def test_pdas_loop_fgmres_matches_dense():
    s, H, U, Uold, phit = setup("small2d")
    dense = pdas.pdas_solve(H, U, Uold, phit, solver="dense")
    H.opts.gmres_rtol = 1e-12
    it = pdas.pdas_solve(H, U, Uold, phit, solver="fgmres")
    assert it["converged"] and it["iterations"] == dense["iterations"]
    assert np.array_equal(it["active"], dense["active"])
    assert np.linalg.norm(it["U"] - dense["U"]) <= 1e-9 * np.linalg.norm(dense["U"])


def test_time_steps_keep_irreversibility_and_follow_the_load():
    s, H, U, Uold, phit = setup("small2d")
    d, nn = H.fine.d, H.fine.n_nodes
    # a consistent previous state: converge the PDAS loop at the initial pressure
    U1 = pdas.pdas_solve(H, U, Uold, phit, solver="dense")["U"]
    U2 = U1.copy()
    p0 = H.mat.pressure
    for n, p in enumerate([p0 * 1.5, p0 * 2.0]):
        out = pdas.time_step(H, U1, U2, p, first=(n == 0), solver="dense")
        assert out["converged"]
        if n == 0:
            assert np.array_equal(out["phit"], U1[d * nn:])
        else:
            assert np.allclose(out["phit"], 2 * U1[d * nn:] - U2[d * nn:], atol=0, rtol=0)
        assert H.mat.pressure == p
        check_kkt(H, out["U"], U1, out["phit"], out["active"], 1e-9)
        U2, U1 = U1, out["U"]
