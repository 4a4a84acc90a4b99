"""The primal-dual active-set loop and the time step around it (oracle, test
infrastructure only: used by tests/, never by the library).

Algorithm 1 of Sec. 3.1 repeated for k = 0, 1, ... until the active set no
longer changes (A_k = A_{k-1}) and the eliminated residual is small in the
absolute norm (||R~_k|| <= eps_as, eps_as = 1e-10 in Sec. 5).  The check uses
the quantities of iteration k (residual, active set, elimination) before its
linear solve; a converged iteration does not solve.

Time stepping (Sec. 2.3, Sec. 5.1): phi~ is the linear extrapolation of the
two previous phase fields in time (the reading used here:
phi~ = phi^{n-1} + theta (phi^{n-1} - phi^{n-2}), theta = dt_n / dt_{n-1},
and phi~ = phi^{n-1} at the first step); the constraint phi <= phi^old
uses phi^old = phi^{n-1}; the pressure follows the loading p(t_n); the PDAS
loop starts from U^{n-1}.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import model, newton


def extrapolate(phi_1, phi_2, theta=1.0):
    """Linear extrapolation in time from phi^{n-1} (phi_1) and phi^{n-2} (phi_2)."""
    return phi_1 + theta * (phi_1 - phi_2)


def eliminated_residual(hier, U, U_old, phit):
    """Steps 1, 3 and 4 of one iteration: (active set, R, R~, constrained flags, lift)."""
    fine = hier.fine
    d, nn = fine.d, fine.n_nodes
    L = len(hier.levels) - 1
    active, v, R = newton.active_set(fine, hier.mat, U, U_old, phit, hier.opts.pdas_c)
    cons = hier.level_constraints(L, active)
    lift = np.zeros(fine.n_dofs)
    lift[d * nn:][active] = (U_old[d * nn:] - U[d * nn:])[active]
    G = model.assemble_jacobian(fine, hier.mat, U, phit, couple=True)
    Rt = model.constrain_rhs(G, R, cons, lift)
    return active, R, Rt, cons, lift


def pdas_solve(hier, U, U_old, phit, tol_as=1e-10, max_iter=50, solver="fgmres", eig_bounds=None):
    """Repeat Algorithm 1 until A_k = A_{k-1} and ||R~_k|| <= tol_as.

    Returns dict(U, iterations (linear solves done), converged, history) where history
    holds per iteration k: n_active, n_changed (vs A_{k-1}, -1 at k = 0), rt_norm, gmres iters.
    """
    U = U.copy()
    prev = None
    hist = []
    for k in range(max_iter + 1):
        active, R, Rt, cons, lift = eliminated_residual(hier, U, U_old, phit)
        rt = float(np.linalg.norm(Rt))
        changed = -1 if prev is None else int(np.count_nonzero(active != prev))
        rec = dict(k=k, n_active=int(active.sum()), n_changed=changed, rt_norm=rt, gmres_iters=0)
        if prev is not None and changed == 0 and rt <= tol_as:
            hist.append(rec)
            return dict(U=U, iterations=k, converged=True, history=hist, active=active)
        if k == max_iter:
            hist.append(rec)
            break
        out = newton.newton_step(hier, U, U_old, phit, solver=solver, eig_bounds=eig_bounds)
        rec["gmres_iters"] = int(out["info"].get("iters", 0))
        hist.append(rec)
        U = out["U"]
        prev = active
    return dict(U=U, iterations=max_iter, converged=False, history=hist, active=prev)


def time_step(hier, U_1, U_2, pressure, theta=1.0, first=False, **kw):
    """One loading step: U^n from U^{n-1} (U_1) and U^{n-2} (U_2) at pressure p(t_n)."""
    d, nn = hier.fine.d, hier.fine.n_nodes
    phi_1, phi_2 = U_1[d * nn:], U_2[d * nn:]
    phit = phi_1.copy() if first else extrapolate(phi_1, phi_2, theta)
    hier.mat = dataclasses.replace(hier.mat, pressure=pressure)
    out = pdas_solve(hier, U_1, U_1, phit, **kw)
    out["phit"] = phit
    return out
