"""Pins of the oracle's transfers, Chebyshev, CG-Lanczos, FGMRES, V-cycle and Newton/PDAS step (CPU only)."""
import numpy as np
import pytest

import workloads as W
from oracle import fe, krylov, mg, model, newton


# ---------------------------------------------------------------------------
# Chebyshev: residual polynomial T_k((theta - t)/delta) / T_k(theta/delta)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("deg", [1, 2, 4, 20])
def test_chebyshev_closed_form(deg):
    lam = np.linspace(0.3, 2.0, 40)
    dvals = np.random.default_rng(1).uniform(0.5, 2.0, 40)
    A = np.diag(lam * dvals)                 # D^{-1} A has eigenvalues lam
    Dinv = 1.0 / dvals
    r = np.random.default_rng(2).uniform(-1, 1, 40)
    a, b = 0.4, 1.9
    x = mg.chebyshev(A, Dinv, r, a, b, deg)
    e0 = np.linalg.solve(A, r)
    err = e0 - x
    theta, delta = (a + b) / 2, (b - a) / 2
    Tk = np.polynomial.chebyshev.Chebyshev.basis(deg)
    expect = Tk((theta - lam) / delta) / Tk(theta / delta) * e0
    assert np.allclose(err, expect, atol=1e-12 * np.abs(e0).max())


# ---------------------------------------------------------------------------
# CG-Lanczos
# ---------------------------------------------------------------------------
def plain_lanczos(Asym, q0, k):
    """Textbook Lanczos with full reorthogonalization (independent of the CG route)."""
    n = q0.size
    Q = np.zeros((k + 1, n))
    Q[0] = q0 / np.linalg.norm(q0)
    al, be = [], []
    for j in range(k):
        w = Asym @ Q[j]
        a = Q[j] @ w
        w = w - a * Q[j] - (be[-1] * Q[j - 1] if j else 0)
        w = w - Q[: j + 1].T @ (Q[: j + 1] @ w)
        al.append(a)
        b = np.linalg.norm(w)
        be.append(b)
        Q[j + 1] = w / b
    T = np.diag(al) + np.diag(be[:-1], 1) + np.diag(be[:-1], -1)
    return np.linalg.eigvalsh(T)


def test_cg_lanczos_matches_lanczos_and_terminates():
    n = 30
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    A = Q @ np.diag(np.linspace(0.1, 5, n)) @ Q.T
    Dd = np.diag(A).copy()
    b = rng.uniform(-1, 1, n)
    res = krylov.cg_lanczos(A, 1.0 / Dd, b, 10)
    Dm = np.diag(Dd ** -0.5)
    ev = plain_lanczos(Dm @ A @ Dm, Dd ** -0.5 * b, 10)
    assert np.allclose(np.linalg.eigvalsh(res["T"]), ev, rtol=1e-9)
    true = np.linalg.eigvalsh(Dm @ A @ Dm)
    assert true[0] - 1e-12 <= res["lam_min"] and res["lam_max"] <= true[-1] + 1e-12
    # finite termination on a diagonal matrix with 6 distinct eigenvalues
    lam = np.repeat([0.5, 1, 2, 3, 7, 9.5], 3)
    res = krylov.cg_lanczos(np.diag(lam), np.ones(lam.size), np.ones(lam.size), 10)
    assert len(res["alphas"]) == 6
    assert np.allclose(np.linalg.eigvalsh(res["T"]), [0.5, 1, 2, 3, 7, 9.5], rtol=1e-10)


def test_fgmres_matches_dense_solve():
    rng = np.random.default_rng(4)
    n = 80
    A = np.eye(n) * 4 + rng.normal(size=(n, n)) * 0.3
    b = rng.normal(size=n)
    Mi = np.linalg.inv(np.diag(np.diag(A)))
    x, info = krylov.fgmres(lambda v: A @ v, lambda v: Mi @ v, b, np.zeros(n), rtol=1e-12, restart=7)
    assert info["rel_res"] <= 1e-12
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-11)


# ---------------------------------------------------------------------------
# transfers and injection
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d,p", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_prolongation_reproduces_polynomials(d, p):
    ext = (1.0, 0.7, 1.3)[:d]
    c = fe.Level(d, p, (2,) * d, ext)
    f = fe.Level(d, p, (4,) * d, ext)
    P = mg.prolongation_scalar(c, f)
    Xc, Xf = c.node_coords(), f.node_coords()
    poly = lambda X: 1 + X[:, 0] - 2 * X[:, 1] + (0.5 * X[:, 0] * X[:, 1] if p == 1 else X[:, 0] ** 2 - X[:, 1] * X[:, 0])
    if d == 3:
        poly2 = lambda X: poly(X) + X[:, 2] * (X[:, 0] if p == 2 else 1.0)
    else:
        poly2 = poly
    assert np.allclose(P @ poly2(Xc), poly2(Xf), atol=1e-13)
    # injection after prolongation is the identity
    idx = mg.injection_index(c, f)
    v = np.random.default_rng(5).uniform(size=c.n_nodes)
    assert np.allclose((P @ v)[idx], v, atol=1e-15)
    # partition of unity and the active indicator stays in {0, 1} under injection
    assert np.allclose(np.asarray(P.sum(axis=1)).ravel(), 1.0)
    a = (np.random.default_rng(6).uniform(size=f.n_nodes) < 0.3).astype(float)
    assert set(np.unique(a[idx])) <= {0.0, 1.0}


# ---------------------------------------------------------------------------
# V-cycle
# ---------------------------------------------------------------------------
def hierarchy(name, **kw):
    s = W.config(name)
    mat = model.Material(**s["material"])
    H = mg.Hierarchy(s["dim"], s["degree"], s["n_cells"], s["extent"], s["domain"], s["n_levels"],
                     s["faces"], mat, extra_u_bits=W.extra_constraint_bits(s), **kw)
    return s, H


@pytest.mark.parametrize("name", ["small2d", "tiny3d_q2"])
def test_vcycle_is_linear_and_masked(name):
    s, H = hierarchy(name)
    U, phit = W.random_linearization(s, 1)
    act = W.random_active(s, 2, 0.1)
    H.set_linearization(U, phit, act)
    n = H.fine.n_dofs
    r1 = np.random.default_rng(3).uniform(-1, 1, n)
    r2 = np.random.default_rng(4).uniform(-1, 1, n)
    z1, z2, z12 = H.vcycle(r1), H.vcycle(r2), H.vcycle(2 * r1 - 3 * r2)
    assert np.allclose(z12, 2 * z1 - 3 * z2, atol=1e-12 * np.abs(z12).max())
    c = H.mg[-1].constrained
    assert (z1[c] == 0).all()
    # as a preconditioner it contracts: the error propagator I - V G~ has norm < 1 on this problem
    G = H.mg[-1].G
    x = np.where(c, 0, np.random.default_rng(5).uniform(-1, 1, n))
    e1 = x - H.vcycle(G @ x)
    assert np.linalg.norm(e1) < 0.9 * np.linalg.norm(x)


def test_two_grid_contraction_on_phase_field_block():
    """u = 0, phi = 1: the phi-phi block is the SPD reaction-diffusion operator; MG reduces its error."""
    s, H = hierarchy("small2d")
    nn = H.fine.n_nodes
    U = np.zeros(H.fine.n_dofs)
    U[2 * nn:] = 1.0
    H.set_linearization(U, np.ones(nn))
    G = H.mg[-1].G
    x = np.zeros(H.fine.n_dofs)
    x[2 * nn:] = np.random.default_rng(6).uniform(-1, 1, nn)
    for _ in range(3):
        x_new = x - H.vcycle(G @ x)
        assert np.linalg.norm(x_new) < 0.3 * np.linalg.norm(x)
        x = x_new


@pytest.mark.parametrize("name", ["small2d", "tiny3d_q2", "small_lshape"])
def test_block_diagonal_vcycle_against_the_full_one(name):
    """P_diag = diag(MG(U~), MG(P~)) (Sec. 3.3) pinned to the full cycle through the structure of G~.

    G_u,phi = 0 (time-lagged phi~), so G~ is block lower triangular: the u rows of every
    residual inside P_full never see the phi part, and its u output equals MG(U~).  With
    r_u = 0 the u part of the full cycle stays 0, the coupling G_phi,u x_u vanishes, and its
    phi output equals MG(P~) r_phi.  P_diag must be exactly that, block by block.
    """
    s, H = hierarchy(name)
    U, phit = W.random_linearization(s, 1)
    act = W.random_active(s, 2, 0.1)
    H.set_linearization(U, phit, act)
    fine = H.fine
    du = fine.d * fine.n_nodes
    G = H.mg[-1].G
    assert abs(G[:du, du:]).max() == 0.0 and abs(G[du:, :du]).max() > 0.0
    n = fine.n_dofs
    r = np.random.default_rng(8).uniform(-1, 1, n)
    ru, rp = r.copy(), r.copy()
    ru[du:] = 0.0
    rp[:du] = 0.0
    H.opts.preconditioner = "full"
    zf, zf_p = H.vcycle(r), H.vcycle(rp)
    zf_u = H.vcycle(ru)
    H.opts.preconditioner = "diag"
    zd, zd_u, zd_p = H.vcycle(r), H.vcycle(ru), H.vcycle(rp)
    scale = np.abs(zf).max()
    assert np.allclose(zd[:du], zf[:du], rtol=0, atol=1e-13 * scale)
    assert np.allclose(zd[du:], zf_p[du:], rtol=0, atol=1e-13 * scale)
    # block diagonal: neither block's input reaches the other block's output
    assert np.abs(zd_u[du:]).max() <= 1e-14 * scale and np.abs(zd_p[:du]).max() <= 1e-14 * scale
    # while the full cycle does carry r_u into the phi part (through G_phi,u)
    assert np.abs(zf_u[du:]).max() > 1e-6 * scale
    # P_diag contracts on the block operator it inverts
    B = H.mg[-1].B
    c = H.mg[-1].constrained
    x = np.where(c, 0, np.random.default_rng(9).uniform(-1, 1, n))
    e1 = x - H.vcycle(B @ x)
    assert np.linalg.norm(e1) < 0.9 * np.linalg.norm(x)


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d"])
def test_newton_step_with_block_diagonal_preconditioner(name):
    """FGMRES preconditioned by P_diag reaches the same Newton update as the dense solve."""
    s, H = hierarchy(name, opts=mg.Options(preconditioner="diag"))
    U, Uold, phit = W.make_state(s)
    dense = newton.newton_step(H, U, Uold, phit, solver="dense")
    it = newton.newton_step(H, U, Uold, phit, solver="fgmres")
    assert it["rel_res"] <= 1e-8
    assert np.linalg.norm(it["dU"] - dense["dU"]) <= 1e-6 * np.linalg.norm(dense["dU"])


def test_unknown_preconditioner_is_rejected():
    s, H = hierarchy("tiny2d", opts=mg.Options(preconditioner="blocks"))
    U, phit = W.random_linearization(s, 1)
    H.set_linearization(U, phit)
    with pytest.raises(ValueError):
        H.vcycle(np.ones(H.fine.n_dofs))


# ---------------------------------------------------------------------------
# Newton / PDAS
# ---------------------------------------------------------------------------
def test_pdas_intact_material_has_empty_active_set():
    s, H = hierarchy("small2d")
    nn = H.fine.n_nodes
    U = np.zeros(H.fine.n_dofs)
    U[2 * nn:] = 1.0
    act, v, R = newton.active_set(H.fine, H.mat, U, U, np.ones(nn))
    # v vanishes in exact arithmetic; in FP64 it is rounding noise of the stiffness row sums
    # (G_c eps / h^2 * 1e-16), so only ties at rounding level can be "active"
    tie = H.mat.G_c * H.mat.eps / min(H.fine.h) ** 2 * 1e-13
    assert np.abs(v).max() < tie


def test_pdas_crack_nodes_become_active():
    s, H = hierarchy("cfg1_2d_q1_32")
    U, Uold, phit = W.make_state(s)
    act, v, R = newton.active_set(H.fine, H.mat, U, Uold, phit)
    nn = H.fine.n_nodes
    X = H.fine.node_coords()
    on_crack = (np.abs(X[:, 1] - 0.5) < 1e-12) & (X[:, 0] > 0.375 + 1e-9) & (X[:, 0] < 0.625 - 1e-9)
    assert on_crack.sum() > 0 and act[on_crack].all()
    # raising phi above phi^old by eta adds c*eta > 0 to v: the active set can only grow
    U2 = U.copy()
    U2[2 * nn:] += 1e-3
    act2, v2, _ = newton.active_set(H.fine, H.mat, U2, Uold, phit)
    assert (act2 >= act).all()


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d", "tiny2d_q2"])
def test_newton_step_dense_vs_fgmres(name):
    s, H = hierarchy(name)
    U, Uold, phit = W.make_state(s)
    dense = newton.newton_step(H, U, Uold, phit, solver="dense")
    it = newton.newton_step(H, U, Uold, phit, solver="fgmres")
    assert it["rel_res"] <= 1e-8
    assert np.linalg.norm(it["dU"] - dense["dU"]) <= 1e-6 * np.linalg.norm(dense["dU"])


@pytest.mark.parametrize("name", ["cfg1_2d_q1_32", "small3d_q2", "small_lshape"])
def test_newton_step_properties(name):
    s, H = hierarchy(name)
    U, Uold, phit = W.make_state(s)
    out = newton.newton_step(H, U, Uold, phit)
    assert out["rel_res"] <= 1e-8
    fine = H.fine
    d, nn = fine.d, fine.n_nodes
    Un = out["U"]
    # phi_{k+1} = phi^old on the active set
    act = out["active"]
    assert np.allclose(Un[d * nn:][act], Uold[d * nn:][act], atol=1e-14)
    # the displacement equation is linear in u for fixed phi~: its free rows vanish after one step
    A = model.assemble_residual(fine, H.mat, Un, phit)
    free_u = ~out["constrained"][: d * nn]
    scale = np.linalg.norm(model.assemble_residual(fine, H.mat, U, phit)[: d * nn][free_u]) + 1e-300
    assert np.linalg.norm(A[: d * nn][free_u]) <= 1e-6 * max(scale, np.linalg.norm(out["Rt"]))
    # constrained displacement DoFs keep their prescribed values
    cu = out["constrained"][: d * nn]
    assert np.array_equal(Un[: d * nn][cu], U[: d * nn][cu])
