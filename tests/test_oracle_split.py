"""Pins of the oracle's Miehe spectral split (Sec. 2.1) and of its consistent linearization.

Point-wise: the tension/compression decomposition E_s = E_s^+ + E_s^- against the
compressive part written independently with min(0, .), the closed forms of pure tension
(everything positive) and pure compression (nothing positive), invariance under
rotation, sigma^+ = dE_s^+/de and C^+ = dsigma^+/de by central differences (also at a
repeated eigenvalue), the major symmetry of C^+, the H(0) = 0 reading at e = 0, and 2D
plane strain against the 3D strain with a zero out-of-plane row.
Assembled: the split Jacobian against central differences of the split residual, the
displacement rows of the residual against the derivative of the bulk energy, and the
identity with the unsplit operator where g(phi~) = 1.
"""
import numpy as np
import pytest

import workloads as W
from oracle import fe, model, quantities

MAT = dict(E=1.0, nu=0.3, G_c=1.3, eps=0.07, kappa=1e-10, pressure=2e-3)


def mat(split="miehe", **kw):
    return model.Material(**dict(MAT, split=split, **kw))


def rand_rot(rng, d):
    Q, R = np.linalg.qr(rng.normal(size=(d, d)))
    return Q * np.sign(np.diag(R))


def rand_strain(rng, d, eig):
    Q = rand_rot(rng, d)
    return Q @ np.diag(eig) @ Q.T


def Es_full(m, e):
    tr = np.trace(e)
    return 0.5 * m.lam * tr * tr + m.mu * np.sum(e * e)


def sym_basis(d):
    out = []
    for i in range(d):
        for j in range(i, d):
            h = np.zeros((d, d))
            h[i, j] = h[j, i] = 1.0
            out.append(h)
    return out


EIGS = {2: [(0.7, -0.4), (-0.3, 0.2), (0.5, 0.9), (-1.0, -0.2)],
        3: [(0.7, -0.4, 0.25), (-0.3, 0.2, -0.8), (0.5, 0.9, 0.3), (-1.0, -0.2, -0.6), (0.4, 0.4, -0.3)]}


@pytest.mark.parametrize("d", [2, 3])
def test_split_energy_decomposition_and_closed_forms(d):
    m = mat()
    rng = np.random.default_rng(d)
    for eig in EIGS[d]:
        e = rand_strain(rng, d, eig)
        sp = model.miehe_split(m, e)
        # compressive part written independently: lam/2 <tr>_-^2 + mu sum <lam_i>_-^2
        l = np.asarray(eig)
        Es_neg = 0.5 * m.lam * min(0.0, l.sum()) ** 2 + m.mu * np.sum(np.minimum(l, 0.0) ** 2)
        assert np.isclose(sp["Es_pos"] + Es_neg, Es_full(m, e), rtol=1e-13)
        # rotation invariance of E_s^+ and covariance of sigma^+
        Q = rand_rot(rng, d)
        sq = model.miehe_split(m, Q @ e @ Q.T)
        assert np.isclose(sq["Es_pos"], sp["Es_pos"], rtol=1e-12, atol=1e-15)
        assert np.allclose(sq["sigma_pos"], Q @ sp["sigma_pos"] @ Q.T, rtol=0, atol=1e-13)
    # pure tension: everything is positive; pure compression: nothing is
    e = rand_strain(rng, d, np.linspace(0.2, 0.5, d))
    sp = model.miehe_split(m, e)
    assert np.isclose(sp["Es_pos"], Es_full(m, e), rtol=1e-13)
    assert np.allclose(sp["sigma_pos"], 2 * m.mu * e + m.lam * np.trace(e) * np.eye(d), atol=1e-14)
    for h in sym_basis(d):
        assert np.allclose(model.tangent_pos(m, sp, h[None]), 2 * m.mu * h + m.lam * np.trace(h) * np.eye(d),
                           atol=1e-14)
    sp = model.miehe_split(m, -e)
    assert sp["Es_pos"] == 0.0 and np.abs(sp["sigma_pos"]).max() <= 1e-16
    assert np.abs(model.tangent_pos(m, sp, np.stack(sym_basis(d)))).max() == 0.0


@pytest.mark.parametrize("d", [2, 3])
def test_split_stress_and_tangent_are_derivatives(d):
    m = mat()
    rng = np.random.default_rng(10 + d)
    t = 1e-6
    cases = [rand_strain(rng, d, eig) for eig in EIGS[d]]
    if d == 3:
        # repeated positive eigenvalue: e_+ is smooth there and the tangent must not care
        # which eigenvectors eigh returns for the double eigenvalue
        cases.append(rand_strain(rng, 3, (0.4, 0.4, -0.3)))
    for e in cases:
        sp = model.miehe_split(m, e)
        for h in sym_basis(d):
            Ep = model.miehe_split(m, e + t * h)
            Em = model.miehe_split(m, e - t * h)
            dE = (Ep["Es_pos"] - Em["Es_pos"]) / (2 * t)
            assert np.isclose(dE, np.sum(sp["sigma_pos"] * h), rtol=1e-8, atol=1e-10)
            dS = (Ep["sigma_pos"] - Em["sigma_pos"]) / (2 * t)
            Ch = model.tangent_pos(m, sp, h[None])[0]
            assert np.allclose(Ch, dS, rtol=0, atol=1e-7), (e, h)
        # major symmetry: h1 : C+ h2 = h2 : C+ h1 (C+ is the Hessian of E_s^+)
        B = np.stack(sym_basis(d))
        CB = model.tangent_pos(m, sp, B)
        M = np.einsum("kij,lij->kl", CB, B)
        assert np.allclose(M, M.T, atol=1e-13)


def test_split_tangent_at_zero_strain_and_plane_strain_embedding():
    m = mat()
    # reading: H(0) = 0, so zero strain counts as not in tension
    sp = model.miehe_split(m, np.zeros((3, 3)))
    assert sp["Es_pos"] == 0.0 and np.abs(model.tangent_pos(m, sp, np.stack(sym_basis(3)))).max() == 0.0
    # a rank-deficient strain (pure shear in a rotated frame): its zero eigenvalue comes out of
    # the eigensolver as rounding noise of either sign; the snap makes it 0, and the tangent is
    # the one of the exact zero eigenvalue (H(0) = 0)
    rng = np.random.default_rng(4)
    Q = rand_rot(rng, 3)
    ex = np.array([[0.0, 0.3, 0.0], [0.3, 0.0, 0.0], [0.0, 0.0, 0.0]])
    e = Q @ ex @ Q.T
    sp = model.miehe_split(m, e)
    assert np.sort(sp["lam"])[1] == 0.0 and sp["tr"] == 0.0 and sp["H_tr"] == 0.0
    sx = model.miehe_split(m, ex)
    assert np.sort(sx["lam"])[1] == 0.0
    for h in sym_basis(3):
        assert np.allclose(model.tangent_pos(m, sp, h[None])[0],
                           Q @ model.tangent_pos(m, sx, (Q.T @ h @ Q)[None])[0] @ Q.T, atol=1e-14)
    rng = np.random.default_rng(3)
    for eig in EIGS[2]:
        e2 = rand_strain(rng, 2, eig)
        e3 = np.zeros((3, 3))
        e3[:2, :2] = e2
        s2, s3 = model.miehe_split(m, e2), model.miehe_split(m, e3)
        assert np.isclose(s2["Es_pos"], s3["Es_pos"], rtol=1e-13)
        assert np.allclose(s2["sigma_pos"], s3["sigma_pos"][:2, :2], atol=1e-14)
        for h in sym_basis(2):
            h3 = np.zeros((3, 3))
            h3[:2, :2] = h
            assert np.allclose(model.tangent_pos(m, s2, h[None])[0], model.tangent_pos(m, s3, h3[None])[0][:2, :2],
                               atol=1e-13)


def level(d, p, n=3, domain=fe.BOX):
    return fe.Level(d, p, (n,) * d, (1.0, 0.8, 1.2)[:d], domain)


def random_state(lev, seed, amp=0.05):
    rng = np.random.default_rng(seed)
    d, nn = lev.d, lev.n_nodes
    U = np.concatenate([rng.uniform(-amp, amp, d * nn), rng.uniform(0.0, 1.0, nn)])
    phit = rng.uniform(0.0, 1.0, nn)
    hole = lev.hole_node
    for c in range(d + 1):
        U[c * nn:(c + 1) * nn][hole] = 0.0
    phit[hole] = 0.0
    return U, phit


@pytest.mark.parametrize("d,p,domain", [(2, 1, fe.BOX), (2, 2, fe.BOX), (3, 1, fe.BOX), (3, 2, fe.BOX),
                                        (3, 1, fe.LSHAPE)])
def test_split_jacobian_is_the_derivative_of_the_split_residual(d, p, domain):
    m = mat()
    lev = level(d, p, 4 if domain == fe.LSHAPE else 3, domain)
    U, phit = random_state(lev, 7 * d + p)
    G = model.assemble_jacobian(lev, m, U, phit)
    rng = np.random.default_rng(1)
    dU = rng.uniform(-1, 1, lev.n_dofs)
    for c in range(d + 1):
        dU[c * lev.n_nodes:(c + 1) * lev.n_nodes][lev.hole_node] = 0.0
    t = 1e-6
    fd = (model.assemble_residual(lev, m, U + t * dU, phit) - model.assemble_residual(lev, m, U - t * dU, phit)) / (2 * t)
    Gd = G @ dU
    assert np.linalg.norm(fd - Gd) <= 1e-7 * np.linalg.norm(Gd)
    # and it differs from the unsplit Jacobian at this state (the split is active)
    G0 = model.assemble_jacobian(lev, mat("none"), U, phit)
    assert np.linalg.norm(G0 @ dU - Gd) > 1e-3 * np.linalg.norm(Gd)


@pytest.mark.parametrize("d,p", [(2, 1), (3, 1), (3, 2)])
def test_split_displacement_residual_is_the_derivative_of_the_bulk_energy(d, p):
    """u rows of A(U) = d/du of int g(phi~) E_s^+ + E_s^- + phi~^2 p div u, i.e. the bulk
    energy evaluated with phi~ in the phase-field slot."""
    m = mat()
    lev = level(d, p)
    U, phit = random_state(lev, 3 + d + p)
    V = U.copy()
    V[d * lev.n_nodes:] = phit
    A = model.assemble_residual(lev, m, U, phit)
    rng = np.random.default_rng(2)
    w = np.zeros(lev.n_dofs)
    w[: d * lev.n_nodes] = rng.uniform(-1, 1, d * lev.n_nodes)
    t = 1e-6
    dE = (quantities.energies(lev, m, V + t * w)[1] - quantities.energies(lev, m, V - t * w)[1]) / (2 * t)
    assert np.isclose(A @ w, dE, rtol=1e-7)


@pytest.mark.parametrize("d,p", [(2, 1), (3, 2)])
def test_split_equals_unsplit_where_nothing_is_degraded(d, p):
    """g(phi~) = 1 (phi~ = 1): g sigma^+ + sigma^- = sigma, so the displacement rows of the
    residual and of the Jacobian are the unsplit ones for any u."""
    lev = level(d, p)
    U, _ = random_state(lev, 11)
    phit = np.ones(lev.n_nodes)
    du = d * lev.n_nodes
    Gs = model.assemble_jacobian(lev, mat(), U, phit)
    Gn = model.assemble_jacobian(lev, mat("none"), U, phit)
    assert abs(Gs[:du] - Gn[:du]).max() <= 1e-12 * abs(Gn[:du]).max()
    As = model.assemble_residual(lev, mat(), U, phit)
    An = model.assemble_residual(lev, mat("none"), U, phit)
    assert np.allclose(As[:du], An[:du], rtol=0, atol=1e-14 * np.abs(An[:du]).max())


def test_split_flag_of_the_workloads():
    s = W.config("small_lshape_miehe")
    assert s["material"]["split"] == "miehe"
    assert model.Material(**s["material"]).split == "miehe"


@pytest.mark.parametrize("name", ["tiny2d_miehe", "tiny3d_miehe", "tiny2d_q2_miehe"])
def test_split_newton_step_dense_vs_fgmres(name):
    from oracle import mg, newton
    s = W.config(name)
    H = mg.Hierarchy(s["dim"], s["degree"], s["n_cells"], s["extent"], s["domain"], s["n_levels"], s["faces"],
                     model.Material(**s["material"]), extra_u_bits=W.extra_constraint_bits(s))
    U, Uold, phit = W.make_state(s)
    dense = newton.newton_step(H, U, Uold, phit, solver="dense")
    it = newton.newton_step(H, U, Uold, phit, solver="fgmres")
    assert it["rel_res"] <= 1e-8
    assert np.linalg.norm(it["dU"] - dense["dU"]) <= 1e-6 * np.linalg.norm(dense["dU"])


def test_split_pdas_loop_converges_to_a_kkt_point():
    """With the split the displacement equation is nonlinear: the loop takes Newton steps until
    the active set settles and the eliminated residual vanishes."""
    from oracle import mg, pdas
    s = W.config("small2d_miehe")
    H = mg.Hierarchy(s["dim"], s["degree"], s["n_cells"], s["extent"], s["domain"], s["n_levels"], s["faces"],
                     model.Material(**s["material"]), extra_u_bits=W.extra_constraint_bits(s))
    H.opts.gmres_rtol = 1e-12
    U0, Uold, phit = W.make_state(s)
    out = pdas.pdas_solve(H, U0, Uold, phit, tol_as=1e-10, max_iter=30)
    assert out["converged"]
    d, nn = s["dim"], H.fine.n_nodes
    U = out["U"]
    assert np.all(U[d * nn:] <= Uold[d * nn:] + 1e-12)
    A = model.assemble_residual(H.fine, H.mat, U, phit)
    cons = H.level_constraints(len(H.levels) - 1, out["active"])
    assert np.abs(A[~cons]).max() <= 1e-9
