"""One primal-dual active-set (semi-smooth Newton) step (oracle, test infrastructure only).

Algorithm 1 of Sec. 3.1, iteration k:
  1. R_k = -A(U_k)
  2. G_k = A'(U_k)
  3. A_k = { i ~ phi : (M^{-1} R_k)_i + c (U_k - U^old)_i > 0 }, M the
     Gauss-Lobatto lumped mass, c = 100
  4. eliminate the rows and columns of A_k (and of the Dirichlet DoFs):
     G~ = Pi_F G Pi_F + Pi_C, R~ = Pi_F (R - G d) + d with the lift
     d = phi^old - phi_k on A_k (so that phi_{k+1} = phi^old there)
  5. solve G~ dU = R~ (FGMRES preconditioned by the monolithic V-cycle, or a
     dense solve on tiny meshes)
  6. U_{k+1} = U_k + dU
Dirichlet targets are the current values of U_k on those DoFs (the iterate
already satisfies the boundary data), so the lift is zero there.
"""
from __future__ import annotations

import numpy as np

from . import model
from .krylov import fgmres


def active_set(lev, mat, U, U_old, phit, c=100.0):
    """Returns (active flag per node, decision value v per node, R = -A(U))."""
    d, nn = lev.d, lev.n_nodes
    R = -model.assemble_residual(lev, mat, U, phit)
    M = model.lumped_mass(lev)
    ok = ~lev.hole_node
    v = np.zeros(nn)
    v[ok] = R[d * nn:][ok] / M[ok] + c * (U[d * nn:] - U_old[d * nn:])[ok]
    return ok & (v > 0.0), v, R


def newton_step(hier, U, U_old, phit, solver="fgmres", eig_bounds=None):
    fine = hier.fine
    d, nn = fine.d, fine.n_nodes
    L = len(hier.levels) - 1
    o = hier.opts
    active, v, R = active_set(fine, hier.mat, U, U_old, phit, o.pdas_c)
    cons = hier.level_constraints(L, active)
    lift = np.zeros(fine.n_dofs)
    lift[d * nn:][active] = (U_old[d * nn:] - U[d * nn:])[active]
    G = model.assemble_jacobian(fine, hier.mat, U, phit, couple=True)
    Rt = model.constrain_rhs(G, R, cons, lift)
    Gt = model.constrain_matrix(G, cons)
    info = {}
    if solver == "dense":
        dU = np.linalg.solve(Gt.toarray(), Rt)
        info = dict(iters=0)
    else:
        hier.set_linearization(U, phit, active, eig_bounds=eig_bounds)
        dU, info = fgmres(lambda x: Gt @ x, hier.vcycle, Rt, lift.copy(),
                          rtol=o.gmres_rtol, restart=o.gmres_restart, max_iter=o.gmres_max_iter,
                          atol=o.gmres_atol)
    res = float(np.linalg.norm(Rt - Gt @ dU))
    return dict(U=U + dU, dU=dU, active=active, v=v, R=R, Rt=Rt, Gt=Gt, constrained=cons,
                n_active=int(active.sum()), rel_res=res / float(np.linalg.norm(Rt)), info=info)
