"""Reference element, quadrature and uniform level meshes (oracle, test infrastructure only).

Discretization of Sec. 2.4: conforming Q_p Lagrange elements on a uniform
Cartesian quadrilateral (2D) / hexahedral (3D) mesh, the same element for the
displacement components and the phase field, (d+1) unknowns per node.

Vector layout (shared interface with the library): component-major blocks
[u_1 | ... | u_d | phi], each block over the level's bounding-box node lattice
with x fastest, then y, then z.  Lattice nodes that belong to no active cell
(the hole of the L-shaped domain) are stored and held at zero.
"""
from __future__ import annotations

import math
from itertools import product

import numpy as np

BOX = 0
LSHAPE = 1


# --------------------------------------------------------------------------
# 1D rules and bases
# --------------------------------------------------------------------------
def gauss_legendre_01(n: int):
    """n-point Gauss-Legendre rule mapped to [0, 1] (the cell quadrature).

    The paper does not name the cell rule; (p+1) Gauss points per direction
    integrate the Q_p stiffness and mass exactly.  Pinned by exact integration
    of monomials up to degree 2n-1 (tests/test_oracle_fe.py).
    """
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_lobatto_01(p: int):
    """Gauss-Lobatto rule whose points are the Q_p nodes (Sec. 3.1, remark on M).

    p=1: trapezoid (0, 1; 1/2, 1/2).  p=2: Simpson (0, 1/2, 1; 1/6, 4/6, 1/6).
    Used only for the lumped (diagonal) mass matrix.
    """
    if p == 1:
        return np.array([0.0, 1.0]), np.array([0.5, 0.5])
    if p == 2:
        return np.array([0.0, 0.5, 1.0]), np.array([1.0, 4.0, 1.0]) / 6.0
    raise ValueError("degree must be 1 or 2")


def lagrange_1d(p: int, t):
    """Values and derivatives of the 1D Lagrange basis on nodes k/p, k=0..p.

    Returns (L, dL) of shape (len(t), p+1): L[:, k] = prod_{m!=k} (t-t_m)/(t_k-t_m).
    """
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    nodes = np.arange(p + 1) / p
    L = np.ones((t.size, p + 1))
    dL = np.zeros((t.size, p + 1))
    for k in range(p + 1):
        others = [m for m in range(p + 1) if m != k]
        for m in others:
            L[:, k] *= (t - nodes[m]) / (nodes[k] - nodes[m])
        # product rule: d/dt prod_m f_m = sum_j f_j' prod_{m!=j} f_m
        for j in others:
            term = np.full(t.size, 1.0 / (nodes[k] - nodes[j]))
            for m in others:
                if m != j:
                    term = term * (t - nodes[m]) / (nodes[k] - nodes[m])
            dL[:, k] += term
    return L, dL


# --------------------------------------------------------------------------
# Reference cell tables (tensor products, x-fastest local numbering)
# --------------------------------------------------------------------------
def local_multi_indices(d: int, n: int):
    """Multi-indices (i_0, ..., i_{d-1}) of an n^d tensor grid, i_0 fastest."""
    out = []
    for rev in product(range(n), repeat=d):
        out.append(tuple(reversed(rev)))
    return out


class RefCell:
    """Shape values / reference gradients of Q_p at the Gauss points of [0,1]^d."""

    def __init__(self, d: int, p: int):
        self.d, self.p = d, p
        n = p + 1
        xq, wq = gauss_legendre_01(n)
        L, dL = lagrange_1d(p, xq)                  # (n_q, p+1)
        self.nodes = local_multi_indices(d, p + 1)  # local node a -> (a_0..)
        self.qpts = local_multi_indices(d, n)       # qp q -> (q_0..)
        nq, nl = len(self.qpts), len(self.nodes)
        self.N = np.zeros((nq, nl))
        self.dN_ref = np.zeros((nq, nl, d))
        self.w = np.zeros(nq)
        for iq, q in enumerate(self.qpts):
            self.w[iq] = np.prod([wq[qk] for qk in q])
            for ia, a in enumerate(self.nodes):
                self.N[iq, ia] = np.prod([L[q[k], a[k]] for k in range(d)])
                for j in range(d):
                    v = 1.0
                    for k in range(d):
                        v *= dL[q[k], a[k]] if k == j else L[q[k], a[k]]
                    self.dN_ref[iq, ia, j] = v
        self.xq = xq


# --------------------------------------------------------------------------
# Uniform level mesh
# --------------------------------------------------------------------------
class Level:
    """One uniform level: N cells per axis on [0, extent]^d, Q_p node lattice.

    Cells of the L-shaped domain: a cell is in the hole when its centre has
    x > extent_x/2 and y > extent_y/2 (all z), i.e. [0,1]^3 minus
    [0.5,1] x [0.5,1] x [0,1].
    """

    def __init__(self, d, p, n_cells, extent, domain=BOX):
        self.d, self.p = int(d), int(p)
        self.N = tuple(int(v) for v in n_cells[:d])
        self.ext = tuple(float(v) for v in extent[:d])
        self.h = tuple(e / n for e, n in zip(self.ext, self.N))
        self.nn = tuple(self.p * n + 1 for n in self.N)
        self.n_nodes = int(np.prod(self.nn))
        self.n_dofs = (self.d + 1) * self.n_nodes
        self.domain = domain
        self.ref = RefCell(self.d, self.p)

        nstride = [1]
        for k in range(1, d):
            nstride.append(nstride[-1] * self.nn[k - 1])
        self.nstride = nstride

        ncell = int(np.prod(self.N))
        cid = np.arange(ncell)
        cidx = np.zeros((ncell, d), dtype=np.int64)
        rem = cid.copy()
        for k in range(d):
            cidx[:, k] = rem % self.N[k]
            rem //= self.N[k]
        active = np.ones(ncell, dtype=bool)
        if domain == LSHAPE:
            cx = (cidx[:, 0] + 0.5) * self.h[0]
            cy = (cidx[:, 1] + 0.5) * self.h[1]
            active = ~((cx > 0.5 * self.ext[0]) & (cy > 0.5 * self.ext[1]))
        self.cell_index = cidx[active]
        nl = len(self.ref.nodes)
        conn = np.zeros((self.cell_index.shape[0], nl), dtype=np.int64)
        for ia, a in enumerate(self.ref.nodes):
            g = np.zeros(self.cell_index.shape[0], dtype=np.int64)
            for k in range(d):
                g += (self.p * self.cell_index[:, k] + a[k]) * nstride[k]
            conn[:, ia] = g
        self.conn = conn
        self.n_cells = conn.shape[0]
        self.jxw_scale = float(np.prod(self.h))

        used = np.zeros(self.n_nodes, dtype=bool)
        used[conn.ravel()] = True
        self.hole_node = ~used

    # lattice coordinates ---------------------------------------------------
    def node_lattice_index(self):
        """(n_nodes, d) integer lattice index of every node (x fastest)."""
        idx = np.zeros((self.n_nodes, self.d), dtype=np.int64)
        rem = np.arange(self.n_nodes)
        for k in range(self.d):
            idx[:, k] = rem % self.nn[k]
            rem //= self.nn[k]
        return idx

    def node_coords(self):
        idx = self.node_lattice_index()
        return idx * (np.array(self.h) / self.p)

    def boundary_face_nodes(self, faces: int):
        """Nodes on the selected faces: bit 2k = {x_k = 0}, bit 2k+1 = {x_k = extent_k}."""
        idx = self.node_lattice_index()
        sel = np.zeros(self.n_nodes, dtype=bool)
        for k in range(self.d):
            if faces & (1 << (2 * k)):
                sel |= idx[:, k] == 0
            if faces & (1 << (2 * k + 1)):
                sel |= idx[:, k] == self.nn[k] - 1
        return sel

    def dof(self, comp: int, node):
        return comp * self.n_nodes + np.asarray(node)


def level_hierarchy(d, p, n_cells_fine, extent, domain, n_levels):
    """Nested uniform levels l = 0 (coarsest) .. L-1 (finest); N_l = N_fine / 2^(L-1-l)."""
    levels = []
    for l in range(n_levels):
        s = 2 ** (n_levels - 1 - l)
        nc = []
        for k in range(d):
            if n_cells_fine[k] % s:
                raise ValueError("cells per axis must be divisible by 2^(levels-1)")
            nc.append(n_cells_fine[k] // s)
        levels.append(Level(d, p, nc, extent, domain))
    return levels


def cell_diameter(level: Level) -> float:
    """Element diameter h (Sec. 5.1: eps is given in multiples of it)."""
    return math.sqrt(sum(hk * hk for hk in level.h))
