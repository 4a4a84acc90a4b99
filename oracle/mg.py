"""Geometric multigrid pieces (oracle, test infrastructure only).

* nodal injection U_l = R_l U of the linearization point, phi~ and the active
  indicator to every coarser level (Sec. 4.2: a_l = R_l a with a_l in {0,1}
  because every coarse vertex is also a fine vertex; G_l(U_l) replaces G_l(U));
* canonical prolongation P (coarse Q_p function evaluated at the fine nodes)
  and restriction P^T (Sec. 3.2);
* level operators G~_l rediscretized from (U_l, phi~_l, A_l), the
  block-diagonal smoother operator B~_l = diag(G_uu, G_phiphi) and its diagonal
  (Sec. 3.2.1, Sec. 3.3 S_full);
* Chebyshev-Jacobi smoothing over [1.2 lam/5, 1.2 lam] with degree 4
  (Sec. 3.2.1) and the Chebyshev coarse solve over [0.9 lam_min, 1.2 lam_max]
  (Sec. 3.2.2);
* the V-cycle P_full^{-1} = MG(G~) (Sec. 3.3), and the block-diagonal
  alternative P_diag^{-1} = diag(MG(U~), MG(P~)) of the same section: one
  multigrid per diagonal block, i.e. the same cycle with every residual formed
  with B~ instead of G~ (the transfers, smoothers and coarse solves are per
  block already, so the two block cycles never mix).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from . import model
from .fe import Level, lagrange_1d, level_hierarchy, local_multi_indices
from .krylov import cg_lanczos
from .rng import eig_start_seed, uniform_pm1


# --------------------------------------------------------------------------
# Injection and transfers
# --------------------------------------------------------------------------
def injection_index(coarse: Level, fine: Level):
    """Fine node index of every coarse node (the fine node at the same position)."""
    ci = coarse.node_lattice_index()
    g = np.zeros(coarse.n_nodes, dtype=np.int64)
    for k in range(coarse.d):
        g += (2 * ci[:, k]) * fine.nstride[k]
    return g


def inject_nodal(coarse, fine, v_fine, ncomp):
    """Nodal injection of an ncomp-component vector (component-major blocks)."""
    idx = injection_index(coarse, fine)
    return np.concatenate([v_fine[c * fine.n_nodes + idx] for c in range(ncomp)])


def prolongation_scalar(coarse: Level, fine: Level):
    """P (fine nodes x coarse nodes): coarse Q_p basis functions evaluated at fine nodes."""
    d, p = fine.d, fine.p
    fi = fine.node_lattice_index()
    rows, cols, vals = [], [], []
    # per axis: containing coarse cell and local coordinate of every fine node
    cell = np.zeros((fine.n_nodes, d), dtype=np.int64)
    t = np.zeros((fine.n_nodes, d))
    for k in range(d):
        x = fi[:, k] / (2.0 * p)                  # position in coarse-cell units
        ck = np.minimum(np.floor(x).astype(np.int64), coarse.N[k] - 1)
        cell[:, k] = ck
        t[:, k] = x - ck
    Ls = [lagrange_1d(p, t[:, k])[0] for k in range(d)]  # (n_fine, p+1)
    for a in local_multi_indices(d, p + 1):
        w = np.ones(fine.n_nodes)
        col = np.zeros(fine.n_nodes, dtype=np.int64)
        for k in range(d):
            w *= Ls[k][:, a[k]]
            col += (p * cell[:, k] + a[k]) * coarse.nstride[k]
        nz = np.abs(w) > 0
        rows.append(np.nonzero(nz)[0])
        cols.append(col[nz])
        vals.append(w[nz])
    P = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(fine.n_nodes, coarse.n_nodes)).tocsr()
    P.sum_duplicates()
    return P


def prolongation(coarse, fine):
    """Block-diagonal P over the (d+1) components."""
    Ps = prolongation_scalar(coarse, fine)
    return sp.block_diag([Ps] * (fine.d + 1), format="csr")


# --------------------------------------------------------------------------
# Chebyshev iteration (textbook three-term recurrence; Saad 2003 Alg. 12.1)
# --------------------------------------------------------------------------
def chebyshev(A, Dinv, r, a, b, degree):
    """Approximate A^{-1} r with `degree` Chebyshev-Jacobi steps from zero.

    The residual polynomial is T_k((theta - t)/delta) / T_k(theta/delta) in
    t = eigenvalue of D^{-1} A, theta = (a+b)/2, delta = (b-a)/2; degree k
    uses k-1 products with A.  Pinned against that closed form on diagonal
    matrices (tests/test_oracle_solvers.py).
    """
    theta = 0.5 * (b + a)
    delta = 0.5 * (b - a)
    sigma = theta / delta
    rho = 1.0 / sigma
    dvec = Dinv * r / theta
    x = dvec.copy()
    res = r.copy()
    for _ in range(1, degree):
        res = res - A @ dvec
        rho_new = 1.0 / (2.0 * sigma - rho)
        dvec = rho_new * rho * dvec + (2.0 * rho_new / delta) * (Dinv * res)
        x = x + dvec
        rho = rho_new
    return x


# --------------------------------------------------------------------------
# Level operators
# --------------------------------------------------------------------------
@dataclass
class Options:
    cheb_degree: int = 4
    cheb_ratio: float = 5.0          # smoothing range [1.2 lam / 5, 1.2 lam]
    cheb_safety: float = 1.2
    eig_cg_steps: int = 10
    coarse_degree: int = 20
    coarse_sweeps: int = 2
    coarse_lo_factor: float = 0.9    # coarse range [0.9 lam_min, 1.2 lam_max]
    gmres_restart: int = 50
    gmres_max_iter: int = 500
    gmres_rtol: float = 1e-8
    gmres_atol: float = 0.0          # absolute floor: stop at max(rtol ||R~||, atol)
    pdas_c: float = 100.0
    eig_seed: int = 12345
    preconditioner: str = "full"     # "full": MG(G~); "diag": diag(MG(U~), MG(P~)) (Sec. 3.3)


@dataclass
class MGLevel:
    lev: Level
    U: np.ndarray
    phit: np.ndarray
    constrained: np.ndarray
    G: sp.csr_matrix = None       # G~ (constrained full Jacobian)
    B: sp.csr_matrix = None       # B~ (constrained block-diagonal operator)
    D: np.ndarray = None          # diag(G~)
    eig: dict = field(default_factory=dict)   # block -> (lam_min, lam_max) raw Ritz values


class Hierarchy:
    """Level data for one linearization point (U, phi~, active set) on all levels."""

    def __init__(self, d, p, n_cells, extent, domain, n_levels, dirichlet_faces, mat,
                 opts: Options = None, extra_u_bits=None):
        self.levels = level_hierarchy(d, p, n_cells, extent, domain, n_levels)
        self.d, self.p = d, p
        self.mat = mat
        self.faces = dirichlet_faces
        self.opts = opts or Options()
        self.extra_fine = None if extra_u_bits is None else np.asarray(extra_u_bits, dtype=np.uint8)
        self.P = [None] + [prolongation(self.levels[l - 1], self.levels[l]) for l in range(1, n_levels)]
        self.mg = None

    @property
    def fine(self):
        return self.levels[-1]

    def level_constraints(self, l, active_fine):
        """Constraint flags on level l: geometric Dirichlet faces and hole, injected extras and active set."""
        L = len(self.levels) - 1
        extra, act = self.extra_fine, active_fine
        for k in range(L, l, -1):
            idx = injection_index(self.levels[k - 1], self.levels[k])
            if extra is not None:
                extra = extra[idx]
            if act is not None:
                act = act[idx]
        return model.constrained_dofs(self.levels[l], self.faces, act, extra)

    def set_linearization(self, U, phit, active_fine=None, eig_bounds=None):
        """Injection of (U, phi~, a) to every level, operators, diagonals and eigenvalue estimates."""
        L = len(self.levels) - 1
        mgl = [None] * (L + 1)
        Ul, pl = np.asarray(U, dtype=np.float64), np.asarray(phit, dtype=np.float64)
        for l in range(L, -1, -1):
            if l < L:
                Ul = inject_nodal(self.levels[l], self.levels[l + 1], Ul, self.d + 1)
                pl = inject_nodal(self.levels[l], self.levels[l + 1], pl, 1)
            lev = self.levels[l]
            c = self.level_constraints(l, active_fine)
            G = model.assemble_jacobian(lev, self.mat, Ul, pl, couple=True)
            B = model.assemble_jacobian(lev, self.mat, Ul, pl, couple=False)
            m = MGLevel(lev, Ul.copy(), pl.copy(), c)
            m.G = model.constrain_matrix(G, c)
            m.B = model.constrain_matrix(B, c)
            m.D = m.B.diagonal().copy()
            mgl[l] = m
        self.mg = mgl
        for l in range(L + 1):
            if eig_bounds is not None and eig_bounds[l] is not None:
                self.mg[l].eig = dict(eig_bounds[l])
            else:
                self.mg[l].eig = self.estimate_eigs(l)
        return self

    # ------------------------------------------------------------------
    def blocks(self, l):
        nn = self.levels[l].n_nodes
        return {"u": np.arange(0, self.d * nn), "phi": np.arange(self.d * nn, (self.d + 1) * nn)}

    def estimate_eigs(self, l):
        """lam_min / lam_max of D^{-1} B~_bb per block from eig_cg_steps PCG steps (Sec. 3.2.1)."""
        m = self.mg[l]
        out = {}
        for bi, (name, idx) in enumerate(self.blocks(l).items()):
            A = m.B[idx][:, idx]
            Dinv = 1.0 / m.D[idx]
            free = ~m.constrained[idx]
            s = uniform_pm1(eig_start_seed(self.opts.eig_seed, l, bi), len(idx))
            s = np.where(free, s, 0.0)
            if not free.any():
                out[name] = (1.0, 1.0)
                continue
            res = cg_lanczos(A, Dinv, s, self.opts.eig_cg_steps)
            out[name] = (res["lam_min"], res["lam_max"])
        return out

    # ------------------------------------------------------------------
    def cycle_operator(self, l):
        """The operator the V-cycle forms its residuals with: G~ for P_full, B~ for P_diag."""
        if self.opts.preconditioner == "full":
            return self.mg[l].G
        if self.opts.preconditioner == "diag":
            return self.mg[l].B
        raise ValueError(f"unknown preconditioner {self.opts.preconditioner!r}")

    def smooth(self, l, b, x):
        """One smoothing step: r = b - G~ x (the cycle's operator), x += Cheb_B(r) per block."""
        m = self.mg[l]
        r = b - self.cycle_operator(l) @ x
        e = np.zeros_like(x)
        o = self.opts
        for name, idx in self.blocks(l).items():
            lmax = o.cheb_safety * m.eig[name][1]
            lo = lmax / o.cheb_ratio
            e[idx] = chebyshev(m.B[idx][:, idx], 1.0 / m.D[idx], r[idx], lo, lmax, o.cheb_degree)
        return x + e

    def coarse_solve(self, b):
        m = self.mg[0]
        o = self.opts
        x = np.zeros_like(b)
        A = self.cycle_operator(0)
        for _ in range(o.coarse_sweeps):
            r = b - A @ x
            for name, idx in self.blocks(0).items():
                lo = o.coarse_lo_factor * m.eig[name][0]
                hi = o.cheb_safety * m.eig[name][1]
                x[idx] += chebyshev(m.B[idx][:, idx], 1.0 / m.D[idx], r[idx], lo, hi, o.coarse_degree)
        return x

    def vcycle_level(self, l, b):
        if l == 0:
            return self.coarse_solve(b)
        m = self.mg[l]
        x = self.smooth(l, b, np.zeros_like(b))
        r = b - self.cycle_operator(l) @ x
        bc = self.P[l].T @ r
        bc[self.mg[l - 1].constrained] = 0.0
        e = self.vcycle_level(l - 1, bc)
        corr = self.P[l] @ e
        corr[m.constrained] = 0.0
        x = x + corr
        return self.smooth(l, b, x)

    def vcycle(self, r):
        """z = P^{-1} r on the fine level (P_full or P_diag); input and output vanish on constrained DoFs."""
        L = len(self.levels) - 1
        c = self.mg[L].constrained
        b = np.where(c, 0.0, r)
        z = self.vcycle_level(L, b)
        z[c] = 0.0
        return z
