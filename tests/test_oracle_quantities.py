"""Pins of the oracle's energies and boundary loads (quantities of interest, Sec. 5).

Closed forms for fields the discrete spaces reproduce exactly (constants, linear phase
fields, linear displacements with constant strain and stress), rigid motions, the
divergence theorem for a constant stress, and the continuum crack energy of a straight
crack G_c L (1 - exp(-2a/eps)) approached at second order under mesh refinement.
"""
import numpy as np
import pytest

from oracle import fe, model, quantities

MAT = dict(E=1.0, nu=0.3, G_c=1.3, eps=0.07, kappa=1e-10, pressure=2e-3)


def level(d, p, n, ext, domain=fe.BOX):
    return fe.Level(d, p, (n,) * d, ext[:d], domain)


def state(lev, u_fun, phi_fun):
    X = lev.node_coords()
    d, nn = lev.d, lev.n_nodes
    U = np.zeros(lev.n_dofs)
    u = u_fun(X)
    for i in range(d):
        U[i * nn:(i + 1) * nn] = u[:, i]
    U[d * nn:] = phi_fun(X)
    return U


def box_volume(ext, d):
    return float(np.prod(ext[:d]))


@pytest.mark.parametrize("d,p", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_crack_energy_constant_and_linear_phase_fields(d, p):
    mat = model.Material(**MAT)
    ext = (1.0, 0.8, 1.2)
    lev = level(d, p, 4, ext)
    V = box_volume(ext, d)
    zero_u = lambda X: np.zeros((X.shape[0], d))
    Ec, Eb = quantities.energies(lev, mat, state(lev, zero_u, lambda X: np.ones(X.shape[0])))
    assert abs(Ec) <= 1e-28 and Eb == 0.0   # 1 - sum_a N_a is rounding
    Ec, _ = quantities.energies(lev, mat, state(lev, zero_u, lambda X: np.zeros(X.shape[0])))
    assert np.isclose(Ec, 0.5 * mat.G_c / mat.eps * V, rtol=1e-13)
    rng = np.random.default_rng(d * 10 + p)
    alpha, beta = 0.3, rng.uniform(-1, 1, d)
    Ec, _ = quantities.energies(lev, mat, state(lev, zero_u, lambda X: alpha + X @ beta))
    E = np.array(ext[:d])
    m2 = ((1.0 - alpha) - beta @ (E / 2)) ** 2 + np.sum(beta ** 2 * E ** 2 / 12.0)
    exact = 0.5 * mat.G_c * (V * m2 / mat.eps + mat.eps * float(beta @ beta) * V)
    assert np.isclose(Ec, exact, rtol=1e-12)


def test_crack_energy_of_a_straight_crack_converges_at_second_order():
    mat = model.Material(**dict(MAT, eps=0.05))
    x0, a, L = 0.5, 0.5, 1.0
    exact = mat.G_c * L * (1.0 - np.exp(-2.0 * a / mat.eps))
    errs = []
    for n in (40, 80, 160):
        lev = level(2, 1, n, (1.0, 1.0))
        U = state(lev, lambda X: np.zeros((X.shape[0], 2)), lambda X: 1.0 - np.exp(-np.abs(X[:, 0] - x0) / mat.eps))
        errs.append(abs(quantities.energies(lev, mat, U)[0] - exact) / exact)
    assert errs[-1] < 2e-3
    for e0, e1 in zip(errs, errs[1:]):
        assert 0.2 < e1 / e0 < 0.3


@pytest.mark.parametrize("d,p", [(2, 1), (3, 1), (3, 2)])
def test_bulk_energy_of_constant_strain_and_rigid_rotation(d, p):
    mat = model.Material(**MAT)
    ext = (1.0, 0.8, 1.2)
    lev = level(d, p, 3, ext)
    V = box_volume(ext, d)
    rng = np.random.default_rng(5 + d + p)
    A = rng.uniform(-1e-2, 1e-2, (d, d))
    c = 0.6
    _, Eb = quantities.energies(lev, mat, state(lev, lambda X: X @ A.T, lambda X: np.full(X.shape[0], c)))
    e = 0.5 * (A + A.T)
    Es = 0.5 * mat.lam * np.trace(e) ** 2 + mat.mu * np.sum(e * e)
    assert np.isclose(Eb, (mat.g(c) * Es + c * c * mat.pressure * np.trace(A)) * V, rtol=1e-12)
    W = A - A.T
    _, Eb = quantities.energies(lev, mat, state(lev, lambda X: X @ W.T, lambda X: np.full(X.shape[0], c)))
    assert abs(Eb) <= 1e-15


@pytest.mark.parametrize("d,p,domain", [(2, 1, fe.BOX), (2, 2, fe.BOX), (3, 1, fe.BOX), (3, 2, fe.BOX),
                                        (3, 1, fe.LSHAPE)])
def test_boundary_traction_of_a_constant_stress(d, p, domain):
    mat = model.Material(**MAT)
    ext = (1.0, 0.8, 1.2)
    lev = level(d, p, 4, ext, domain)
    rng = np.random.default_rng(11 + d + p)
    A = rng.uniform(-1e-2, 1e-2, (d, d))
    c = 0.7
    U = state(lev, lambda X: X @ A.T, lambda X: np.full(X.shape[0], c))
    e = 0.5 * (A + A.T)
    sig = mat.g(c) * (2 * mat.mu * e + mat.lam * np.trace(e) * np.eye(d))
    total = np.zeros(d)
    for face in range(2 * d):
        k, side = face // 2, face % 2
        area = float(np.prod([ext[j] for j in range(d) if j != k]))
        if domain == fe.LSHAPE and k in (0, 1) and side == 1:
            area *= 0.5      # the box face x_k = extent_k borders the hole on half its width
        if domain == fe.LSHAPE and k == 2:
            area *= 0.75     # the z-faces miss the hole's quarter
        t = quantities.boundary_traction(lev, mat, U, face)
        n = np.zeros(d)
        n[k] = 1.0 if side else -1.0
        assert np.allclose(t, sig @ n * area, rtol=1e-12, atol=1e-17)
        total += t
    if domain == fe.BOX:
        assert np.allclose(total, 0.0, atol=1e-16)
