"""Krylov pieces (oracle, test infrastructure only).

* cg_lanczos: Jacobi-preconditioned CG whose coefficients give the Lanczos
  tridiagonal matrix (Saad 2003, Sec. 6.7.3); its extreme eigenvalues estimate
  the spectrum of D^{-1} A (Sec. 3.2.1: 10 CG iterations, safety factor 1.2).
* fgmres: right-preconditioned restarted FGMRES with modified Gram-Schmidt
  (GMRES of Saad & Schultz as the outer solver, Sec. 3 and Sec. 5); the
  stopping test is on the true residual.
"""
from __future__ import annotations

import numpy as np


def cg_lanczos(A, Dinv, b, steps):
    """`steps` PCG iterations on A x = b from x = 0; returns alphas, betas, T and its extreme eigenvalues.

    T_00 = 1/alpha_0, T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
    T_{j,j+1} = sqrt(beta_j)/alpha_j.  Stops early if r.z falls below
    1e-24 of its start value or p.Ap <= 0 (exact convergence / breakdown).
    """
    r = b.copy()
    z = Dinv * r
    pvec = z.copy()
    rz = float(r @ z)
    rz0 = rz
    alphas, betas = [], []
    for _ in range(steps):
        if rz <= 0.0 or rz <= 1e-24 * rz0:
            break
        Ap = A @ pvec
        pAp = float(pvec @ Ap)
        if pAp <= 0.0:
            break
        alpha = rz / pAp
        alphas.append(alpha)
        r = r - alpha * Ap
        z = Dinv * r
        rz_new = float(r @ z)
        beta = rz_new / rz
        betas.append(beta)
        rz = rz_new
        pvec = z + beta * pvec
    k = len(alphas)
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    ev = np.linalg.eigvalsh(T) if k else np.array([1.0])
    return dict(alphas=np.array(alphas), betas=np.array(betas), T=T,
                lam_min=float(ev[0]), lam_max=float(ev[-1]))


def fgmres(apply_A, precond, b, x0, rtol=1e-8, restart=50, max_iter=500, atol=0.0):
    """Right-preconditioned FGMRES(m) with MGS; stop when ||b - A x|| <= max(rtol ||b||, atol).

    Returns (x, info) with info = {iters, res_norm, rel_res, history}.
    """
    x = x0.copy()
    bnorm = float(np.linalg.norm(b))
    tol = max(rtol * bnorm, atol)
    total = 0
    history = []
    r = b - apply_A(x)
    beta = float(np.linalg.norm(r))
    history.append(beta)
    while beta > tol and total < max_iter:
        m = restart
        V = np.zeros((m + 1, b.size))
        Z = np.zeros((m, b.size))
        H = np.zeros((m + 1, m))
        V[0] = r / beta
        g = np.zeros(m + 1)
        g[0] = beta
        cs, sn = np.zeros(m), np.zeros(m)
        j_end = 0
        for j in range(m):
            Z[j] = precond(V[j])
            w = apply_A(Z[j])
            for i in range(j + 1):
                H[i, j] = float(w @ V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = (1.0, 0.0) if den == 0 else (H[j, j] / den, H[j + 1, j] / den)
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            j_end = j + 1
            history.append(abs(g[j + 1]))
            if abs(g[j + 1]) <= tol or total >= max_iter or H[j, j] == 0:
                break
        y = np.linalg.solve(np.triu(H[:j_end, :j_end]), g[:j_end])
        x = x + Z[:j_end].T @ y
        r = b - apply_A(x)
        beta = float(np.linalg.norm(r))
    return x, dict(iters=total, res_norm=beta, rel_res=beta / bnorm if bnorm else 0.0, history=history)
