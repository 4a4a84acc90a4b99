"""Pins of the oracle's row-sampled checkers (CPU only).

jacobian_rows and residual_rows evaluate (G(U) x)[rows] and A(U)[rows] from the
element arrays of the cells around the requested nodes only; the full-size GPU
parity tests use them where the assembled CSR matrix would not fit.  Here they
are checked against the fully assembled operator (every cell, SciPy CSR) on
small meshes: every row of the level, and hand-picked rows where a cell could
plausibly be missed -- lattice corners, Dirichlet faces, the nodes on the faces
of the L-shape's hole and its re-entrant edge, and the phase-field rows.
"""
import numpy as np
import pytest

from oracle import fe, model

MAT = model.Material(E=1.3, nu=0.27, G_c=0.9, eps=0.11, kappa=1e-3, pressure=0.02)
MAT_SPLIT = model.Material(E=1.3, nu=0.27, G_c=0.9, eps=0.11, kappa=1e-3, pressure=0.02, split="miehe")

MESHES = [
    (2, 1, (5, 4), (1.0, 0.8), fe.BOX),
    (2, 2, (3, 4), (1.0, 1.0), fe.BOX),
    (3, 1, (4, 3, 3), (1.0, 0.9, 0.7), fe.BOX),
    (3, 2, (2, 2, 3), (1.0, 1.0, 1.0), fe.BOX),
    (3, 1, (4, 4, 2), (1.0, 1.0, 1.0), fe.LSHAPE),
    (3, 2, (2, 4, 1), (1.0, 1.0, 1.0), fe.LSHAPE),
]


def state(lev, seed):
    r = np.random.default_rng(seed)
    U = np.concatenate([r.uniform(-2e-2, 2e-2, lev.d * lev.n_nodes), r.uniform(0, 1, lev.n_nodes)])
    phit = r.uniform(0, 1, lev.n_nodes)
    for c in range(lev.d + 1):
        U[c * lev.n_nodes:(c + 1) * lev.n_nodes][lev.hole_node] = 0.0
    phit[lev.hole_node] = 0.0
    return U, phit, r.uniform(-1, 1, lev.n_dofs)


def special_nodes(lev):
    """Corners, face nodes and the hole-adjacent nodes of the lattice (those a cell search can miss)."""
    idx = lev.node_lattice_index()
    sel = np.zeros(lev.n_nodes, dtype=bool)
    corner = np.ones(lev.n_nodes, dtype=bool)
    for k in range(lev.d):
        at_end = (idx[:, k] == 0) | (idx[:, k] == lev.nn[k] - 1)
        corner &= at_end
        sel |= idx[:, k] == lev.nn[k] - 1
    sel |= corner
    if lev.domain == fe.LSHAPE:
        X = lev.node_coords()
        hx, hy = 0.5 * lev.ext[0], 0.5 * lev.ext[1]
        on_x = (np.abs(X[:, 0] - hx) < 1e-12) & (X[:, 1] >= hy - 1e-12)
        on_y = (np.abs(X[:, 1] - hy) < 1e-12) & (X[:, 0] >= hx - 1e-12)
        assert on_x.any() and on_y.any()
        sel |= (on_x | on_y) & ~lev.hole_node
    return np.nonzero(sel & ~lev.hole_node)[0]


def all_rows_and_special(lev):
    nodes = special_nodes(lev)
    special = np.concatenate([c * lev.n_nodes + nodes for c in range(lev.d + 1)])
    return [np.arange(lev.n_dofs), special, special[::-3]]


@pytest.mark.parametrize("d,p,n,ext,dom", MESHES)
@pytest.mark.parametrize("couple", [True, False])
def test_jacobian_rows_equal_assembled_product(d, p, n, ext, dom, couple):
    lev = fe.Level(d, p, n, ext, dom)
    U, phit, x = state(lev, 3 + d + p)
    ref = model.assemble_jacobian(lev, MAT, U, phit, couple=couple) @ x
    scale = np.abs(ref).max()
    for rows in all_rows_and_special(lev):
        got = model.jacobian_rows(lev, MAT, U, phit, x, rows, couple=couple)
        assert got.shape == rows.shape
        assert np.abs(got - ref[rows]).max() <= 1e-14 * scale


@pytest.mark.parametrize("d,p,n,ext,dom", MESHES)
def test_residual_rows_equal_assembled_residual(d, p, n, ext, dom):
    lev = fe.Level(d, p, n, ext, dom)
    U, phit, _ = state(lev, 11 + d + p)
    ref = model.assemble_residual(lev, MAT, U, phit)
    scale = np.abs(ref).max()
    for rows in all_rows_and_special(lev):
        got = model.residual_rows(lev, MAT, U, phit, rows)
        assert np.abs(got - ref[rows]).max() <= 1e-14 * scale


@pytest.mark.parametrize("d,p,n,ext,dom", [MESHES[0], MESHES[2], MESHES[4]])
def test_row_checkers_with_the_split(d, p, n, ext, dom):
    lev = fe.Level(d, p, n, ext, dom)
    U, phit, x = state(lev, 23 + d)
    Gx = model.assemble_jacobian(lev, MAT_SPLIT, U, phit) @ x
    A = model.assemble_residual(lev, MAT_SPLIT, U, phit)
    rows = all_rows_and_special(lev)[1]
    assert np.abs(model.jacobian_rows(lev, MAT_SPLIT, U, phit, x, rows) - Gx[rows]).max() <= 1e-14 * np.abs(Gx).max()
    assert np.abs(model.residual_rows(lev, MAT_SPLIT, U, phit, rows) - A[rows]).max() <= 1e-14 * np.abs(A).max()


def test_row_checker_catches_a_missing_cell():
    """A cell search that drops the cells on one side of a node gives a different row: the
    comparison above is sharp enough to see one missing cell (its contribution is not small)."""
    lev = fe.Level(3, 1, (4, 4, 2), (1.0, 1.0, 1.0), fe.LSHAPE)
    U, phit, x = state(lev, 5)
    ref = model.assemble_jacobian(lev, MAT, U, phit) @ x
    node = special_nodes(lev)[len(special_nodes(lev)) // 2]
    cells = model.cells_touching_nodes(lev, [node])
    assert len(cells) >= 2
    tab = model.CellTables(lev)
    y = np.zeros(lev.n_dofs)
    c = cells[1:]
    K = model.element_jacobian(lev, tab, MAT, U, phit, c, True)
    ld = model.local_dofs(lev, c)
    np.add.at(y, ld, np.einsum("ckl,cl->ck", K, x[ld]))
    rows = np.array([c_ * lev.n_nodes + node for c_ in range(lev.d + 1)])
    assert np.abs(y[rows] - ref[rows]).max() > 1e-6 * np.abs(ref).max()
