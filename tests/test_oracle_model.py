"""Pins of the oracle's residual, Jacobian, lumped mass and constraints (CPU only).

Each test checks the oracle against something other than itself: rigid-body
invariance, finite differences of A with the exact cubic remainder removed by
Richardson extrapolation, patch tests with closed-form values, and Kronecker
products of textbook 1D element matrices.
"""
import numpy as np
import pytest

from oracle import fe, model

MAT = model.Material(E=1.0, nu=0.3, G_c=1.0, eps=0.1, kappa=1e-10, pressure=1e-3)
MAT_P = model.Material(E=2.0, nu=0.25, G_c=0.7, eps=0.13, kappa=1e-3, pressure=0.05)


def random_state(lev, seed, uamp=1e-2):
    r = np.random.default_rng(seed)
    U = np.concatenate([r.uniform(-uamp, uamp, lev.d * lev.n_nodes), r.uniform(0, 1, lev.n_nodes)])
    return U, r.uniform(0, 1, lev.n_nodes)


def rigid_modes(lev):
    X = lev.node_coords()
    d, nn = lev.d, lev.n_nodes
    modes = []
    for c in range(d):
        v = np.zeros(lev.n_dofs)
        v[c * nn:(c + 1) * nn] = 1.0
        modes.append(v)
    pairs = [(0, 1)] if d == 2 else [(0, 1), (1, 2), (0, 2)]
    for i, j in pairs:                      # infinitesimal rotation in the (i, j) plane
        v = np.zeros(lev.n_dofs)
        v[i * nn:(i + 1) * nn] = -X[:, j]
        v[j * nn:(j + 1) * nn] = X[:, i]
        modes.append(v)
    return modes


LEVELS = [(2, 1, (3, 4), (1.0, 0.7)), (2, 2, (3, 2), (0.8, 1.0)),
          (3, 1, (2, 3, 2), (1.0, 0.6, 0.9)), (3, 2, (2, 2, 1), (1.0, 1.0, 0.5))]


@pytest.mark.parametrize("d,p,n,ext", LEVELS)
def test_rigid_body_null_space(d, p, n, ext):
    lev = fe.Level(d, p, n, ext)
    U, phit = random_state(lev, 1)
    G = model.assemble_jacobian(lev, MAT_P, U, phit)
    A0 = model.assemble_residual(lev, MAT_P, U, phit)
    scale = abs(G).max()
    for r in rigid_modes(lev):
        assert np.abs(G @ r).max() < 1e-12 * scale * np.abs(r).max()
        A1 = model.assemble_residual(lev, MAT_P, U + 1e-2 * r, phit)
        assert np.abs(A1 - A0).max() < 1e-12 * max(1.0, np.abs(A0).max())


@pytest.mark.parametrize("d,p,n,ext", LEVELS)
def test_jacobian_matches_richardson_finite_differences(d, p, n, ext):
    """A is cubic in U with phi~ fixed, so (4 D(h/2) - D(h))/3 equals G v up to rounding."""
    lev = fe.Level(d, p, n, ext)
    U, phit = random_state(lev, 2, uamp=0.3)
    v = np.random.default_rng(3).uniform(-1, 1, lev.n_dofs)
    G = model.assemble_jacobian(lev, MAT_P, U, phit)
    A = lambda W: model.assemble_residual(lev, MAT_P, W, phit)

    def D(h):
        return (A(U + h * v) - A(U - h * v)) / (2 * h)
    h = 0.05
    rich = (4 * D(h / 2) - D(h)) / 3
    Gv = G @ v
    assert np.linalg.norm(rich - Gv) < 1e-11 * np.linalg.norm(Gv)
    # the plain central difference is off by exactly the cubic remainder (so the test is sensitive)
    assert np.linalg.norm(D(h) - Gv) > 1e-6 * np.linalg.norm(Gv)
    # G_{u phi} = 0: perturbing phi alone leaves the displacement rows unchanged
    vphi = v.copy()
    vphi[: d * lev.n_nodes] = 0
    du = (A(U + h * vphi) - A(U - h * vphi))[: d * lev.n_nodes]
    assert np.abs(du).max() < 1e-14


@pytest.mark.parametrize("d,p", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_patch_test_linear_displacement(d, p):
    n = (4,) * d if d == 2 else (3,) * d
    lev = fe.Level(d, p, n, (1.0,) * d)
    X = lev.node_coords()
    rng = np.random.default_rng(4)
    Egrad = rng.uniform(-0.1, 0.1, (d, d))        # u(x) = Egrad x (constant strain)
    phi_c, phit_c = 0.6, 0.8
    U = np.zeros(lev.n_dofs)
    for i in range(d):
        U[i * lev.n_nodes:(i + 1) * lev.n_nodes] = X @ Egrad[i]
    U[d * lev.n_nodes:] = phi_c
    phit = np.full(lev.n_nodes, phit_c)
    A = model.assemble_residual(lev, MAT_P, U, phit)
    interior = ~lev.boundary_face_nodes((1 << (2 * d)) - 1)
    nn = lev.n_nodes
    for i in range(d):
        assert np.abs(A[i * nn:(i + 1) * nn][interior]).max() < 1e-14
    # phi rows: constant integrand times the integral of the test function
    e = 0.5 * (Egrad + Egrad.T)
    tr = np.trace(e)
    Es = 0.5 * MAT_P.lam * tr ** 2 + MAT_P.mu * np.sum(e * e)
    integrand = ((1 - MAT_P.kappa) * phi_c * Es + 2 * phi_c * MAT_P.pressure * tr
                 - MAT_P.G_c / MAT_P.eps * (1 - phi_c))
    Mcons = model.assemble_jacobian(lev, model.Material(1, 0.3, 1.0, 1.0, 0.0, 0.0),
                                    np.zeros(lev.n_dofs), np.ones(nn))
    # consistent-mass row sums = integral of psi_i, from the phi-phi block with G_c/eps = 1, G_c eps = 1:
    # the stiffness part has zero row sums, so the row sum is exactly the mass row sum
    int_psi = np.asarray(Mcons[d * nn:, d * nn:].sum(axis=1)).ravel()
    assert np.allclose(A[d * nn:], integrand * int_psi, rtol=1e-12, atol=1e-15)
    # cross-check int psi for Q1 interior nodes: h^d
    if p == 1:
        assert np.allclose(int_psi[interior], np.prod(lev.h), rtol=1e-13)


def test_pressure_term_closed_form():
    """u = 0, phi~ = a + b x: interior u_x rows equal -2 p b (a + b x_i) * int N_i (Q1)."""
    lev = fe.Level(2, 1, (6, 5), (1.0, 1.0))
    X = lev.node_coords()
    a, b = 0.3, 0.5
    phit = a + b * X[:, 0]
    U = np.zeros(lev.n_dofs)
    U[2 * lev.n_nodes:] = 1.0
    A = model.assemble_residual(lev, MAT_P, U, phit)
    interior = ~lev.boundary_face_nodes(0b1111)
    expect = -2 * MAT_P.pressure * b * (a + b * X[:, 0]) * np.prod(lev.h)
    assert np.allclose(A[: lev.n_nodes][interior], expect[interior], rtol=1e-12)
    assert np.abs(A[lev.n_nodes: 2 * lev.n_nodes][interior]).max() < 1e-15
    # phi == 1 and u == 0 with constant phi~: every phase-field row vanishes
    A1 = model.assemble_residual(lev, MAT_P, U, np.ones(lev.n_nodes))
    assert np.abs(A1[2 * lev.n_nodes:]).max() < 1e-15


# ---------------------------------------------------------------------------
# Kronecker stencils from textbook 1D element matrices
# ---------------------------------------------------------------------------
def elem_1d(p, h):
    """Closed-form 1D element matrices: K = int N'N', M = int N N, C = int N_a' N_b."""
    if p == 1:
        K = np.array([[1, -1], [-1, 1]]) / h
        M = np.array([[2, 1], [1, 2]]) * h / 6
        C = np.array([[-0.5, -0.5], [0.5, 0.5]])
    else:
        K = np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / (3 * h)
        M = np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) * h / 30
        C = np.array([[-0.5, -2 / 3, 1 / 6], [2 / 3, 0, -2 / 3], [-1 / 6, 2 / 3, 0.5]])
    return K, M, C


def global_1d(p, n, h):
    K1, M1, C1 = elem_1d(p, h)
    m = p * n + 1
    K, M, C = (np.zeros((m, m)) for _ in range(3))
    for c in range(n):
        s = slice(p * c, p * c + p + 1)
        K[s, s] += K1
        M[s, s] += M1
        C[s, s] += C1
    return K, M, C


def kron_term(mats1d, test_deriv, trial_deriv):
    """int (d_i N_A or N_A)(d_j N_B or N_B) over the box, as a Kronecker product (x fastest)."""
    factors = []
    for k, (K, M, C) in enumerate(mats1d):
        a = test_deriv == k
        b = trial_deriv == k
        factors.append(K if (a and b) else C if a else C.T if b else M)
    out = factors[-1]
    for f in reversed(factors[:-1]):
        out = np.kron(out, f)
    return out


@pytest.mark.parametrize("d,p,n,ext", LEVELS)
def test_kronecker_stencils(d, p, n, ext):
    lev = fe.Level(d, p, n, ext)
    mats = [global_1d(p, n[k], lev.h[k]) for k in range(d)]
    X = lev.node_coords()
    nn = lev.n_nodes
    rng = np.random.default_rng(5)
    Egrad = rng.uniform(-0.2, 0.2, (d, d))
    phi_c, phit_c = 0.7, 0.45
    U = np.zeros(lev.n_dofs)
    for i in range(d):
        U[i * nn:(i + 1) * nn] = X @ Egrad[i]
    U[d * nn:] = phi_c
    m = MAT_P
    G = model.assemble_jacobian(lev, m, U, np.full(nn, phit_c)).toarray()
    S = {(i, j): kron_term(mats, i, j) for i in range(d) for j in range(d)}
    Mass = kron_term(mats, -1, -1)
    g = (1 - m.kappa) * phit_c ** 2 + m.kappa
    for c in range(d):
        for cp in range(d):
            blk = m.mu * S[(cp, c)] + m.lam * S[(c, cp)]
            if c == cp:
                blk = blk + m.mu * sum(S[(j, j)] for j in range(d))
            assert np.allclose(G[c * nn:(c + 1) * nn, cp * nn:(cp + 1) * nn], g * blk,
                               atol=1e-12 * np.abs(blk).max())
        # u-phi block is zero
        assert np.abs(G[c * nn:(c + 1) * nn, d * nn:]).max() == 0.0
    e = 0.5 * (Egrad + Egrad.T)
    tr = np.trace(e)
    sig = 2 * m.mu * e + m.lam * tr * np.eye(d)
    T = (1 - m.kappa) * phi_c * sig + 2 * m.pressure * phi_c * np.eye(d)
    for cp in range(d):
        blk = sum(T[cp, j] * kron_term(mats, -1, j) for j in range(d))
        assert np.allclose(G[d * nn:, cp * nn:(cp + 1) * nn], blk, atol=1e-12 * max(1e-30, np.abs(blk).max()))
    Es = 0.5 * m.lam * tr ** 2 + m.mu * np.sum(e * e)
    cmass = (1 - m.kappa) * Es + 2 * m.pressure * tr + m.G_c / m.eps
    blk = cmass * Mass + m.G_c * m.eps * sum(S[(j, j)] for j in range(d))
    assert np.allclose(G[d * nn:, d * nn:], blk, atol=1e-12 * np.abs(blk).max())


def test_block_diagonal_operator_drops_only_phi_u():
    lev = fe.Level(2, 1, (3, 3), (1, 1))
    U, phit = random_state(lev, 6)
    G = model.assemble_jacobian(lev, MAT, U, phit).toarray()
    B = model.assemble_jacobian(lev, MAT, U, phit, couple=False).toarray()
    nu_ = 2 * lev.n_nodes
    assert np.array_equal(G[:nu_], B[:nu_])
    assert np.array_equal(G[nu_:, nu_:], B[nu_:, nu_:])
    assert np.abs(B[nu_:, :nu_]).max() == 0 and np.abs(G[nu_:, :nu_]).max() > 0
    # uu and phi-phi blocks are symmetric (the smoother's requirement)
    assert np.allclose(B, B.T, atol=1e-14 * np.abs(B).max())


@pytest.mark.parametrize("d,p,dom,vol", [(2, 1, fe.BOX, 0.56), (2, 2, fe.BOX, 0.56),
                                         (3, 1, fe.LSHAPE, 0.75), (3, 2, fe.LSHAPE, 0.75)])
def test_lumped_mass(d, p, dom, vol):
    ext = (0.8, 0.7) if d == 2 else (1.0, 1.0, 1.0)
    lev = fe.Level(d, p, (4,) * d, ext, dom)
    M = model.lumped_mass(lev)
    assert abs(M.sum() - vol) < 1e-14
    assert (M[lev.hole_node] == 0).all() and (M[~lev.hole_node] > 0).all()
    if p == 1:
        interior = ~lev.boundary_face_nodes((1 << (2 * d)) - 1) & ~lev.hole_node
        X = lev.node_coords()
        near_hole = (X[:, 0] > 0.5 - 1e-9) & (X[:, 1] > 0.5 - 1e-9)
        inner = interior & ~near_hole if dom == fe.LSHAPE else interior
        assert np.allclose(M[inner], np.prod(lev.h), rtol=1e-14)


def test_constraint_elimination():
    lev = fe.Level(2, 1, (4, 4), (1, 1))
    U, phit = random_state(lev, 7)
    G = model.assemble_jacobian(lev, MAT, U, phit)
    act = np.zeros(lev.n_nodes, dtype=bool)
    act[[6, 7, 12]] = True
    c = model.constrained_dofs(lev, 0b1111, act)
    Gt = model.constrain_matrix(G, c).toarray()
    Gd = G.toarray()
    F = ~c
    assert np.array_equal(Gt[np.ix_(F, F)], Gd[np.ix_(F, F)])
    assert np.array_equal(Gt[np.ix_(c, c)], np.eye(c.sum()))
    assert np.abs(Gt[np.ix_(F, c)]).max() == 0 and np.abs(Gt[np.ix_(c, F)]).max() == 0
    # R~ with a lift: the solution of G~ x = R~ satisfies x_C = d and the free rows of G x = R
    R = np.random.default_rng(8).uniform(-1, 1, lev.n_dofs)
    dl = np.zeros(lev.n_dofs)
    dl[c] = np.random.default_rng(9).uniform(-1, 1, c.sum())
    x = np.linalg.solve(Gt, model.constrain_rhs(G, R, c, dl))
    assert np.allclose(x[c], dl[c])
    assert np.allclose((Gd @ x)[F], R[F], atol=1e-10)
