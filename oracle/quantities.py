"""Energies and boundary loads (oracle, test infrastructure only: used by tests/, never by the library).

Quantities of interest of Sec. 5, evaluated cell by cell with the cell
quadrature (p+1 Gauss points per direction), with the state U = (u, phi):

  crack energy  E_c = int G_c/2 ( (1 - phi)^2 / eps + eps grad phi . grad phi ) dx
  bulk energy   E_b = int g_kappa(phi) E_s^+(e(u)) + E_s^-(e(u)) + phi^2 p div u dx
                (no stress split: E_s^+ = E_s, E_s^- = 0; Miehe split as in model.py)
  boundary load L = int_Gamma sigma n ds over one face of the box,
                with sigma = g_kappa(phi) sigma^+(u) + sigma^-(u) (reading: the degraded
                stress of the displacement equation, current phi), on the face's p+1 Gauss points
                per tangential direction; faces of hole cells are not part of the box
                face.
"""
from __future__ import annotations

import numpy as np

from .fe import gauss_legendre_01, lagrange_1d, local_multi_indices
from .model import CellTables, miehe_split, qp_state


def energies(lev, mat, U):
    """(E_c, E_b) of the state U on the level."""
    tab = CellTables(lev)
    cells = np.arange(lev.n_cells)
    d, nn = lev.d, lev.n_nodes
    s = qp_state(lev, tab, mat, U, U[d * nn:], cells)   # phi~ slot unused here
    phi, gphi = s["phi"], s["grad_phi"]
    crack = 0.5 * mat.G_c * ((1.0 - phi) ** 2 / mat.eps + mat.eps * np.einsum("cqj,cqj->cq", gphi, gphi))
    # g E_s^+ + E_s^- = E_s - (1 - g) E_s^+
    bulk = s["Es"] - (1.0 - mat.g(phi)) * s["Es_pos"] + phi ** 2 * mat.pressure * s["div_u"]
    return float(np.einsum("q,cq->", tab.JxW, crack)), float(np.einsum("q,cq->", tab.JxW, bulk))


def face_cells(lev, face):
    """Active cells with a facet on box face `face` (2k: x_k = 0, 2k+1: x_k = extent_k)."""
    k, side = face // 2, face % 2
    target = 0 if side == 0 else lev.N[k] - 1
    return np.flatnonzero(lev.cell_index[:, k] == target)


def boundary_traction(lev, mat, U, face):
    """int_face g(phi) sigma(u) n ds: a d-vector."""
    d, p, nn = lev.d, lev.p, lev.n_nodes
    k, side = face // 2, face % 2
    n_vec = np.zeros(d)
    n_vec[k] = 1.0 if side == 1 else -1.0
    tq, wq = gauss_legendre_01(p + 1)
    L, dL = lagrange_1d(p, tq)                       # tangential directions: Gauss points
    Lf, dLf = lagrange_1d(p, np.array([float(side)]))  # normal direction: the facet
    nodes = lev.ref.nodes
    tang = [j for j in range(d) if j != k]
    fq = local_multi_indices(d - 1, p + 1)
    nq, nl = len(fq), len(nodes)
    N = np.zeros((nq, nl))
    dN = np.zeros((nq, nl, d))
    w = np.zeros(nq)
    for iq, q in enumerate(fq):
        w[iq] = np.prod([wq[qi] for qi in q]) * np.prod([lev.h[j] for j in tang])
        for ia, a in enumerate(nodes):
            def val(j, der):
                if j == k:
                    return (dLf if der else Lf)[0, a[j]]
                qi = q[tang.index(j)]
                return (dL if der else L)[qi, a[j]]
            N[iq, ia] = np.prod([val(j, False) for j in range(d)])
            for jj in range(d):
                dN[iq, ia, jj] = np.prod([val(j, j == jj) for j in range(d)]) / lev.h[jj]
    cells = face_cells(lev, face)
    conn = lev.conn[cells]
    ue = np.stack([U[i * nn + conn] for i in range(d)], axis=1)      # (nc, d, nl)
    phi = np.einsum("qa,ca->cq", N, U[d * nn + conn])
    gu = np.einsum("qaj,cia->cqij", dN, ue)
    e = 0.5 * (gu + np.swapaxes(gu, 2, 3))
    tr = np.trace(e, axis1=2, axis2=3)
    sig = 2.0 * mat.mu * e + mat.lam * tr[..., None, None] * np.eye(d)
    if mat.split == "miehe":
        sig = sig - (1.0 - mat.g(phi))[..., None, None] * miehe_split(mat, e)["sigma_pos"]
    else:
        sig = mat.g(phi)[..., None, None] * sig
    t = np.einsum("cqij,j->cqi", sig, n_vec)
    return np.einsum("q,cqi->i", w, t)
