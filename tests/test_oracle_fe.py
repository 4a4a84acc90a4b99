"""Pins of the oracle's reference element, meshes, constants and generator (CPU only)."""
import math

import numpy as np
import pytest

from conftest import golden
from oracle import fe, model, rng


@pytest.mark.parametrize("n", [2, 3])
def test_gauss_exact_for_degree_2n_minus_1(n):
    x, w = fe.gauss_legendre_01(n)
    for k in range(2 * n):
        assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-15
    # and not for degree 2n (a Gauss rule is exact to 2n-1 exactly)
    assert abs(np.sum(w * x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-6


@pytest.mark.parametrize("p", [1, 2])
def test_lobatto_rules(p):
    x, w = fe.gauss_lobatto_01(p)
    for k in range(2 * p):       # trapezoid exact to 1, Simpson to 3
        assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-15


@pytest.mark.parametrize("p", [1, 2])
def test_lagrange_basis(p):
    t = np.linspace(0, 1, 7)
    L, dL = fe.lagrange_1d(p, t)
    assert np.allclose(L.sum(1), 1.0, atol=1e-15)
    assert np.allclose(dL.sum(1), 0.0, atol=1e-13)
    Ln, _ = fe.lagrange_1d(p, np.arange(p + 1) / p)
    assert np.allclose(Ln, np.eye(p + 1), atol=1e-15)
    # derivative against a centred difference of the polynomial (exact for degree <= 2)
    hstep = 1e-3
    Lp, _ = fe.lagrange_1d(p, t + hstep)
    Lm, _ = fe.lagrange_1d(p, t - hstep)
    assert np.allclose((Lp - Lm) / (2 * hstep), dL, atol=1e-10)


@pytest.mark.parametrize("d,p", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_reference_cell_integrates_polynomials(d, p):
    ref = fe.RefCell(d, p)
    # sum of weights = 1; gradients of the interpolant of x_0 are e_0
    assert abs(ref.w.sum() - 1.0) < 1e-15
    xnodes = np.array([a[0] / p for a in ref.nodes])
    g = np.einsum("qaj,a->qj", ref.dN_ref, xnodes)
    assert np.allclose(g, np.eye(d)[0][None, :], atol=1e-14)


def test_paper_lame_constants():
    c = golden("paper_constants.txt")
    m = model.Material(E=c["mf_E"], nu=c["mf_nu"], G_c=1, eps=1, kappa=1e-10, pressure=0)
    # printed values are truncated to one decimal
    assert 0 <= m.mu - c["mf_mu"] < 0.1
    assert 0 <= m.lam - c["mf_lambda"] < 0.1
    assert abs(m.lam - 2083.3) > 100   # not plane stress


def test_eps_equals_element_diameter():
    c = golden("paper_constants.txt")
    ext = c["mf_domain"]
    lev = fe.Level(2, 1, (int(c["mf_cells"]),) * 2, (ext, ext))
    assert abs(fe.cell_diameter(lev) - c["mf_eps"]) < 5e-4
    ls = fe.Level(2, 1, (int(c["ls_cells"]),) * 2, (c["ls_domain"],) * 2)
    assert abs(fe.cell_diameter(ls) - c["ls_eps"]) < 0.1
    # side length would be 0.03125 and 7.8: far from the printed values
    assert abs(ext / c["mf_cells"] - c["mf_eps"]) > 0.01


def test_scaling_dof_counts():
    c = golden("paper_constants.txt")
    for l, key in [(7, "scale_l7_dofs"), (8, "scale_l8_dofs")]:
        n = 4 * 2 ** l
        lev_nodes = (n + 1) ** 2
        assert abs(3 * lev_nodes - c[key]) / c[key] < 0.02


def test_level_layout_and_lshape():
    lev = fe.Level(3, 1, (4, 4, 4), (1, 1, 1), fe.LSHAPE)
    assert lev.n_cells == 64 - 16
    X = lev.node_coords()
    hole_expected = (X[:, 0] > 0.5 + 1e-12) & (X[:, 1] > 0.5 + 1e-12)
    assert np.array_equal(lev.hole_node, hole_expected)
    lev2 = fe.Level(3, 2, (2, 3, 4), (1, 2, 3))
    assert lev2.nn == (5, 7, 9)
    assert lev2.n_dofs == 4 * 5 * 7 * 9
    # x fastest
    X2 = lev2.node_coords()
    assert X2[1, 0] > 0 and X2[1, 1] == 0 and X2[5, 1] > 0


def test_splitmix64_reference_outputs():
    c = golden("paper_constants.txt")
    z = rng.stream(0, 3)
    assert int(z[0]) == c["splitmix64_seed0_0"]
    assert int(z[1]) == c["splitmix64_seed0_1"]
    assert int(z[2]) == c["splitmix64_seed0_2"]
    u = rng.uniform_pm1(5, 10000)
    assert u.min() >= -1 and u.max() < 1 and abs(u.mean()) < 0.05
