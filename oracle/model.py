"""Residual A(U), Jacobian G(U), lumped mass and constraints (oracle, test infrastructure only).

Follows the quasi-monolithic semi-linear form (Sec. 2.3, eq. semilinear) with
either no stress split (E_s^+ = E_s, sigma^- = 0) or the Miehe spectral split
(Sec. 2.1), the time-lagged extrapolation phi~ in the displacement equation,
and its discrete Jacobian G_ij = A'(U)(Phi_i, Phi_j) (Sec. 2.4).  Everything is
computed by per-cell Gauss quadrature into dense element arrays and assembled
into SciPy CSR.

Miehe split (Sec. 2.1): with e = sum_i lam_i n_i n_i^T,
  E_s^+ = lam/2 <tr e>_+^2 + mu tr(e_+^2),  e_+ = sum_i <lam_i>_+ n_i n_i^T,
  sigma^+ = dE_s^+/de = lam <tr e>_+ I + 2 mu e_+,  E_s^- = E_s - E_s^+,
  sigma^- = sigma - sigma^+.
Its tangent dsigma^+/de [h] = lam H(tr e) tr(h) I + 2 mu De_+[h], where the
derivative of the spectral function e -> e_+ is the Daleckii-Krein formula
De_+[h] = N (F o (N^T h N)) N^T with F_ij the divided difference of <.>_+ at
(lam_i, lam_j) (its derivative H(lam_i) when lam_i = lam_j); the eigenpairs come
from numpy.linalg.eigh.

Readings of the paper used here (also listed in the design notes):
* the factor 1/2 in front of d_phi g_kappa(phi) E_s in the phase-field
  equation is taken literally (ES_FACTOR = 1/2), so that term is
  (1-kappa) phi E_s(e(u));
* g_kappa and phi^2 in the displacement equation use phi~ (the extrapolation),
  which makes the u/phi block of the Jacobian zero (Sec. 3.3);
* 2D is plane strain: lambda = E nu / ((1+nu)(1-2nu)) in every dimension
  (the multiple-fracture parameter table lists mu = 4166.6, lambda = 2777.7
  for E = 1e4, nu = 0.2);
* split: the Heaviside step H = d<x>_+/dx is taken as 0 at x = 0 (a zero
  eigenvalue or trace counts as not in tension; at e = 0 the tangent is the
  undegraded C); an eigenvalue, or tr e, within SPLIT_SNAP times the spectral
  radius of e of zero is taken as zero (its sign is rounding noise of the
  eigensolver, and the tangent jumps there); in 2D the split acts on the in-plane 2x2 strain (the
  out-of-plane eigenvalue of plane strain is 0 and adds nothing to e_+, tr e,
  or the in-plane tangent).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .fe import Level, gauss_lobatto_01, local_multi_indices

ES_FACTOR = 0.5
SPLIT_SNAP = 1e-13


@dataclass
class Material:
    E: float
    nu: float
    G_c: float
    eps: float
    kappa: float
    pressure: float
    split: str = "none"     # "none" (E_s^+ = E_s) or "miehe" (spectral split, Sec. 2.1)

    @property
    def mu(self) -> float:
        """Lame mu = E / (2(1+nu))."""
        return self.E / (2.0 * (1.0 + self.nu))

    @property
    def lam(self) -> float:
        """Lame lambda = E nu / ((1+nu)(1-2nu)) (3D and plane strain)."""
        return self.E * self.nu / ((1.0 + self.nu) * (1.0 - 2.0 * self.nu))

    def g(self, s):
        """Degradation g_kappa(s) = (1-kappa) s^2 + kappa (Sec. 2.1)."""
        return (1.0 - self.kappa) * s * s + self.kappa

    def dg(self, s):
        return 2.0 * (1.0 - self.kappa) * s

    def d2g(self, s):
        return 2.0 * (1.0 - self.kappa) + 0.0 * s


# --------------------------------------------------------------------------
# Miehe spectral split (Sec. 2.1)
# --------------------------------------------------------------------------
def positive_part(x):
    """<x>_+ = max(0, x)."""
    return np.maximum(x, 0.0)


def heaviside(x):
    """d<x>_+/dx, taken as 0 at x = 0."""
    return (x > 0.0).astype(np.float64)


def miehe_split(mat: Material, e):
    """Positive parts of the Miehe split at strains e (..., d, d).

    Returns the eigenpairs, tr e, E_s^+, sigma^+, the divided-difference matrix F of
    <.>_+ at the eigenvalue pairs and H(tr e) (what the tangent needs).
    """
    d = e.shape[-1]
    lam_i, N = np.linalg.eigh(e)                       # ascending, eigenvectors in columns
    tr = np.trace(e, axis1=-2, axis2=-1)
    rad = np.abs(lam_i).max(axis=-1)
    lam_i = np.where(np.abs(lam_i) <= SPLIT_SNAP * rad[..., None], 0.0, lam_i)
    tr = np.where(np.abs(tr) <= SPLIT_SNAP * rad, 0.0, tr)
    lp = positive_part(lam_i)
    e_pos = np.einsum("...ia,...a,...ja->...ij", N, lp, N)
    Es_pos = 0.5 * mat.lam * positive_part(tr) ** 2 + mat.mu * np.sum(lp * lp, axis=-1)
    sigma_pos = mat.lam * positive_part(tr)[..., None, None] * np.eye(d) + 2.0 * mat.mu * e_pos
    li, lj = lam_i[..., :, None], lam_i[..., None, :]
    same = li == lj
    F = np.where(same, heaviside(np.broadcast_to(li, same.shape)),
                 (positive_part(li) - positive_part(lj)) / np.where(same, 1.0, li - lj))
    return dict(lam=lam_i, N=N, tr=tr, e_pos=e_pos, Es_pos=Es_pos, sigma_pos=sigma_pos, F=F,
                H_tr=heaviside(tr))


def tangent_pos(mat: Material, sp, h):
    """dsigma^+/de [h] for strain increments h (..., k, d, d) at the split sp (shape ...)."""
    d = h.shape[-1]
    N = sp["N"][..., None, :, :]
    ht = np.einsum("...ai,...ab,...bj->...ij", N, h, N)            # N^T h N
    De = np.einsum("...ia,...ab,...jb->...ij", N, sp["F"][..., None, :, :] * ht, N)
    trh = np.trace(h, axis1=-2, axis2=-1)
    return mat.lam * (sp["H_tr"][..., None] * trh)[..., None, None] * np.eye(d) + 2.0 * mat.mu * De


# --------------------------------------------------------------------------
# Reference tables in physical scale for a level (affine box cells)
# --------------------------------------------------------------------------
class CellTables:
    def __init__(self, lev: Level):
        d, ref = lev.d, lev.ref
        self.d = d
        self.nl = len(ref.nodes)
        self.N = ref.N                                      # (nq, nl)
        self.dN = ref.dN_ref / np.array(lev.h)[None, None, :]  # (nq, nl, d)
        self.JxW = ref.w * lev.jxw_scale                    # (nq,)
        nq, nl = self.N.shape
        # displacement test/trial functions Phi_(i,a) = N_a e_i, local index k = i*nl + a
        grad = np.zeros((nq, d * nl, d, d))
        for i in range(d):
            for a in range(nl):
                grad[:, i * nl + a, i, :] = self.dN[:, a, :]
        self.grad_w = grad                                  # grad Phi_k (row i = comp)
        self.eps_w = 0.5 * (grad + np.swapaxes(grad, 2, 3))  # e(Phi_k)
        self.div_w = np.trace(grad, axis1=2, axis2=3)       # div Phi_k


def gather(lev: Level, vec, comp, cells):
    """Nodal values of one component on the given cells: (nc, nl)."""
    return vec[comp * lev.n_nodes + lev.conn[cells]]


def qp_state(lev: Level, tab: CellTables, mat: Material, U, phit, cells):
    """Linearization-point quantities at the Gauss points of the given cells."""
    d = lev.d
    ue = np.stack([gather(lev, U, i, cells) for i in range(d)], axis=1)   # (nc,d,nl)
    phie = gather(lev, U, d, cells)                                        # (nc,nl)
    ptle = phit[lev.conn[cells]]                                           # (nc,nl)
    grad_u = np.einsum("qaj,cia->cqij", tab.dN, ue)                        # (nc,nq,d,d)
    e = 0.5 * (grad_u + np.swapaxes(grad_u, 2, 3))
    tr = np.trace(e, axis1=2, axis2=3)
    eye = np.eye(d)
    sigma = 2.0 * mat.mu * e + mat.lam * tr[..., None, None] * eye
    Es = 0.5 * mat.lam * tr * tr + mat.mu * np.einsum("cqij,cqij->cq", e, e)
    phi = np.einsum("qa,ca->cq", tab.N, phie)
    grad_phi = np.einsum("qaj,ca->cqj", tab.dN, phie)
    phit_q = np.einsum("qa,ca->cq", tab.N, ptle)
    out = dict(e=e, sigma=sigma, Es=Es, div_u=tr, phi=phi, grad_phi=grad_phi, phit=phit_q,
               Es_pos=Es, sigma_pos=sigma, split=None)
    if mat.split == "miehe":
        sp = miehe_split(mat, e)
        out.update(Es_pos=sp["Es_pos"], sigma_pos=sp["sigma_pos"], split=sp)
    elif mat.split != "none":
        raise ValueError(f"unknown split {mat.split!r}")
    return out


# --------------------------------------------------------------------------
# Element residual and element Jacobian (local order: comp-major, x-fastest nodes)
# --------------------------------------------------------------------------
def element_residual(lev, tab, mat, U, phit, cells):
    """Element vectors of A(U)(Phi_i) on the given cells: (nc, (d+1) nl).

    u rows:   (g(phi~) sigma^+(u) + sigma^-(u), e(w)) + (phi~^2 p, div w)
    phi rows: (1/2 g'(phi) E_s^+(e(u)) + 2 phi p div u - G_c/eps (1-phi), psi)
              + G_c eps (grad phi, grad psi)
    """
    s = qp_state(lev, tab, mat, U, phit, cells)
    p = mat.pressure
    gq = mat.g(s["phit"])
    # g sigma^+ + sigma^- = sigma - (1 - g) sigma^+
    sig_u = s["sigma"] - (1.0 - gq)[..., None, None] * s["sigma_pos"]
    ru = np.einsum("q,cqij,qkij->ck", tab.JxW, sig_u, tab.eps_w)
    ru += np.einsum("q,cq,qk->ck", tab.JxW, s["phit"] ** 2 * p, tab.div_w)
    val = (ES_FACTOR * mat.dg(s["phi"]) * s["Es_pos"] + 2.0 * s["phi"] * p * s["div_u"]
           - mat.G_c / mat.eps * (1.0 - s["phi"]))
    rphi = np.einsum("q,cq,qa->ca", tab.JxW, val, tab.N)
    rphi += mat.G_c * mat.eps * np.einsum("q,cqj,qaj->ca", tab.JxW, s["grad_phi"], tab.dN)
    return np.concatenate([ru, rphi], axis=1)


def element_jacobian(lev, tab, mat, U, phit, cells, couple=True):
    """Dense element Jacobians A'(U)(Phi_i, Phi_j) on the given cells: (nc, nloc, nloc).

    Blocks (rows = test, cols = trial):
      uu:     (g(phi~) C^+[e(du)] + C^-[e(du)], e(w)), C^+- = dsigma^+-/de at e(u)
              (no split: C^+ = C, so g(phi~) sigma(du))
      u phi:  0   (phi~ is fixed; Sec. 3.3)
      phi u:  (1/2 g'(phi) sigma^+(u):e(du) + 2 phi p div du, psi)
      phi phi:(1/2 g''(phi) E_s^+(e(u)) dphi + 2 p div u dphi + G_c/eps dphi, psi)
              + G_c eps (grad dphi, grad psi)
    couple=False drops the phi-u block (the block-diagonal operator B of the smoother).
    """
    d, nl = lev.d, tab.nl
    s = qp_state(lev, tab, mat, U, phit, cells)
    p = mat.pressure
    nc = len(cells)
    nu_ = d * nl
    K = np.zeros((nc, nu_ + nl, nu_ + nl))
    eye = np.eye(d)
    # sigma of every displacement trial function: (nq, k, d, d)
    sig_w = 2.0 * mat.mu * tab.eps_w + mat.lam * tab.div_w[..., None, None] * eye
    gq = mat.g(s["phit"])
    if s["split"] is None:
        K[:, :nu_, :nu_] = np.einsum("q,cq,qlij,qkij->ckl", tab.JxW, gq, sig_w, tab.eps_w)
    else:
        # C - (1 - g) C^+ applied to the strain of every trial function
        h = np.broadcast_to(tab.eps_w[None], (nc,) + tab.eps_w.shape)
        Cp = tangent_pos(mat, s["split"], h)                                # (nc, nq, k, d, d)
        sig_t = sig_w[None] - (1.0 - gq)[..., None, None, None] * Cp
        K[:, :nu_, :nu_] = np.einsum("q,cqlij,qkij->ckl", tab.JxW, sig_t, tab.eps_w)
    if couple:
        sig_e = np.einsum("cqij,qlij->cql", s["sigma_pos"], tab.eps_w)      # sigma^+(u):e(du)
        coef = ES_FACTOR * mat.dg(s["phi"])[..., None] * sig_e \
            + 2.0 * p * s["phi"][..., None] * tab.div_w[None, :, :]
        K[:, nu_:, :nu_] = np.einsum("q,cql,qa->cal", tab.JxW, coef, tab.N)
    cphi = ES_FACTOR * mat.d2g(s["phi"]) * s["Es_pos"] + 2.0 * p * s["div_u"] + mat.G_c / mat.eps
    K[:, nu_:, nu_:] = np.einsum("q,cq,qb,qa->cab", tab.JxW, cphi, tab.N, tab.N)
    K[:, nu_:, nu_:] += mat.G_c * mat.eps * np.einsum("q,qbj,qaj->ab", tab.JxW, tab.dN, tab.dN)[None]
    return K


def local_dofs(lev: Level, cells):
    """Global DoF indices of the element arrays, comp-major: (nc, (d+1) nl)."""
    return np.concatenate([comp * lev.n_nodes + lev.conn[cells] for comp in range(lev.d + 1)], axis=1)


# --------------------------------------------------------------------------
# Assembly
# --------------------------------------------------------------------------
def _chunks(n, size):
    for s in range(0, n, size):
        yield np.arange(s, min(n, s + size))


def chunk_size(lev):
    nloc = (lev.d + 1) * len(lev.ref.nodes)
    return max(64, int(2.0e7 // (nloc * nloc)))


def assemble_residual(lev, mat, U, phit):
    """A(U) as a global vector (the Newton residual is R = -A(U))."""
    tab = CellTables(lev)
    A = np.zeros(lev.n_dofs)
    for cells in _chunks(lev.n_cells, chunk_size(lev)):
        np.add.at(A, local_dofs(lev, cells), element_residual(lev, tab, mat, U, phit, cells))
    return A


def assemble_jacobian(lev, mat, U, phit, couple=True):
    """Assembled CSR Jacobian G(U) (no constraints)."""
    tab = CellTables(lev)
    rows, cols, vals = [], [], []
    for cells in _chunks(lev.n_cells, chunk_size(lev)):
        K = element_jacobian(lev, tab, mat, U, phit, cells, couple)
        ld = local_dofs(lev, cells)
        rows.append(np.repeat(ld, ld.shape[1], axis=1).ravel())
        cols.append(np.tile(ld, (1, ld.shape[1])).ravel())
        vals.append(K.ravel())
    G = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(lev.n_dofs, lev.n_dofs)).tocsr()
    G.sum_duplicates()
    return G


def cells_touching_nodes(lev, nodes):
    """Indices of active cells that contain any of the given nodes."""
    hit = np.zeros(lev.n_nodes, dtype=bool)
    hit[np.asarray(nodes)] = True
    return np.nonzero(hit[lev.conn].any(axis=1))[0]


def jacobian_rows(lev, mat, U, phit, x, rows, couple=True):
    """Selected entries (G(U) x)[rows], from the element arrays of the cells around them."""
    rows = np.asarray(rows)
    nodes = rows % lev.n_nodes
    cells = cells_touching_nodes(lev, nodes)
    tab = CellTables(lev)
    y = np.zeros(lev.n_dofs)
    for sl in _chunks(len(cells), chunk_size(lev)):
        c = cells[sl]
        K = element_jacobian(lev, tab, mat, U, phit, c, couple)
        ld = local_dofs(lev, c)
        np.add.at(y, ld, np.einsum("ckl,cl->ck", K, x[ld]))
    return y[rows]


def residual_rows(lev, mat, U, phit, rows):
    rows = np.asarray(rows)
    cells = cells_touching_nodes(lev, rows % lev.n_nodes)
    tab = CellTables(lev)
    A = np.zeros(lev.n_dofs)
    np.add.at(A, local_dofs(lev, cells), element_residual(lev, tab, mat, U, phit, cells))
    return A[rows]


# --------------------------------------------------------------------------
# Lumped mass (Sec. 3.1, remark on M: Gauss-Lobatto quadrature -> diagonal)
# --------------------------------------------------------------------------
def lumped_mass(lev: Level):
    """Diagonal M_ii = sum over cells of the Gauss-Lobatto weight of node i times |cell|.

    The Gauss-Lobatto points of Q_p are its nodes, so N_j(x_i) = delta_ij and the
    quadrature mass matrix is diagonal.  Pinned: sum_i M_ii = |domain|.
    """
    _, w1 = gauss_lobatto_01(lev.p)
    M = np.zeros(lev.n_nodes)
    for ia, a in enumerate(local_multi_indices(lev.d, lev.p + 1)):
        wa = np.prod([w1[ak] for ak in a]) * lev.jxw_scale
        np.add.at(M, lev.conn[:, ia], wa)
    return M


# --------------------------------------------------------------------------
# Constraints (Sec. 3.1 Algorithm 1 step 4; Sec. 4 constraint matrix C)
# --------------------------------------------------------------------------
def constrained_dofs(lev: Level, dirichlet_faces: int, active_phi=None, extra_u_bits=None):
    """Boolean per-DoF constraint flag.

    Displacement DoFs: Dirichlet faces, extra per-node component bits
    (bit i = u_i), hole nodes.  Phase-field DoFs: active set, hole nodes.
    """
    d, nn = lev.d, lev.n_nodes
    c = np.zeros(lev.n_dofs, dtype=bool)
    bnd = lev.boundary_face_nodes(dirichlet_faces)
    for i in range(d):
        ci = bnd | lev.hole_node
        if extra_u_bits is not None:
            ci = ci | ((np.asarray(extra_u_bits) >> i) & 1).astype(bool)
        c[i * nn:(i + 1) * nn] = ci
    cphi = lev.hole_node.copy()
    if active_phi is not None:
        cphi |= np.asarray(active_phi).astype(bool)
    c[d * nn:] = cphi
    return c


def constrain_matrix(G, constrained):
    """G~ = Pi_F G Pi_F + Pi_C: eliminate constrained rows and columns, unit diagonal."""
    free = (~constrained).astype(np.float64)
    F = sp.diags(free)
    return (F @ G @ F + sp.diags(constrained.astype(np.float64))).tocsr()


def constrain_rhs(G, R, constrained, d_lift):
    """R~ = Pi_F (R - G d) + d with the lift d supported on the constrained DoFs."""
    d_lift = np.where(constrained, d_lift, 0.0)
    out = R - G @ d_lift
    out[constrained] = d_lift[constrained]
    return out
