"""Full-size GPU checks: the workloads at their real sizes, compared with the oracle on sampled rows.

The oracle assembles only the cells around a seeded sample of rows (plus
boundary and hole-adjacent rows), so the check runs at 1e6-5e7 DoFs.
Apply tolerance: 1e-12 relative to the largest sampled entry (FP64).
Newton step: the library's own FP64 true residual reaches 1e-8; the oracle
re-evaluates A(U_{k+1}) on sampled free displacement rows (linear in u for
fixed phi~, so they vanish with the linear residual) and checks phi = phi^old
on the active set the library used.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import dev, gpu_solver, host
from oracle import fe, model

pytestmark = pytest.mark.gpu

FULL = ["cfg2_3d_q1_64", "cfg3_3d_q2_96", "cfg5_3d_q1_lshape_256"]


def sample_rows(s, lev, n=3000, seed=0):
    rng = np.random.default_rng(seed)
    rows = set(rng.integers(0, lev.n_dofs, n).tolist())
    # boundary nodes and (L-shape) nodes on the hole's faces, every component
    X = lev.node_coords()
    special = np.nonzero(lev.boundary_face_nodes((1 << (2 * lev.d)) - 1))[0]
    if s["domain"] == fe.LSHAPE:
        ex, ey = s["extent"][0], s["extent"][1]
        near = (np.abs(X[:, 0] - 0.5 * ex) < 1e-12) & (X[:, 1] >= 0.5 * ey - 1e-12)
        special = np.concatenate([special, np.nonzero(near)[0]])
    pick = rng.choice(special, size=min(n // 15, special.size), replace=False)
    for node in pick:
        for c in range(lev.d + 1):
            rows.add(int(c * lev.n_nodes + node))
    return np.array(sorted(rows))


_LEVELS = {}


def oracle_level(s):
    key = s["name"]
    if key not in _LEVELS:
        _LEVELS.clear()
        _LEVELS[key] = fe.Level(s["dim"], s["degree"], s["n_cells"], s["extent"], s["domain"])
    return _LEVELS[key]


def n_samples(s, n):
    return n // 4 if s["degree"] == 2 else n


@pytest.mark.parametrize("name", FULL)
def test_fullsize(name):
    check_apply(name)
    check_newton(name)


def check_apply(name):
    print(f"[case] full-size apply {name}", flush=True)
    s = W.config(name)
    U, phit = W.random_linearization(s, 41)
    act = W.random_active(s, 42, 0.05)
    lev = oracle_level(s)
    bits = W.extra_constraint_bits(s)
    cons = model.constrained_dofs(lev, s["faces"], act, bits)
    mat = model.Material(**s["material"])
    S = gpu_solver(s, eig_cg_steps=1)
    S.set_linearization(dev(U), dev(phit), dev(act))
    x = np.random.default_rng(43).uniform(-1, 1, lev.n_dofs)
    y = host(S.jacobian_apply(-1, dev(x)))
    rows = sample_rows(s, lev, n=n_samples(s, 3000))
    ref = model.jacobian_rows(lev, mat, U, phit, np.where(cons, 0.0, x), rows)
    ref = np.where(cons[rows], x[rows], ref)
    err = np.abs(y[rows] - ref).max() / np.abs(ref).max()
    print(f"  {len(rows)} sampled rows, max rel err {err:.2e}", flush=True)
    assert err <= 1e-12
    assert np.isfinite(y).all()
    # full-vector property: identity on every constrained DoF
    assert np.array_equal(y[cons], x[cons])
    # the Newton residual -A(U) on the same sampled rows (every row, constrained ones included)
    R = host(S.residual(dev(U), dev(phit)))
    refR = -model.residual_rows(lev, mat, U, phit, rows)
    errR = np.abs(R[rows] - refR).max() / np.abs(refR).max()
    print(f"  residual: max rel err {errR:.2e} on the sampled rows", flush=True)
    assert errR <= 1e-12
    assert np.isfinite(R).all()


def check_newton(name):
    print(f"[case] full-size Newton step {name}", flush=True)
    s = W.config(name)
    U, Uold, phit = W.make_state(s)
    S = gpu_solver(s)
    Ud = dev(U)
    st, rep = S.newton_step(Ud, dev(Uold), dev(phit))
    Un = host(Ud)
    _, _, mk = S.level_data(-1)
    mk = host(mk)
    nn = S.n_nodes()
    d = s["dim"]
    print(f"  gmres {rep.gmres_iters}, rel res {rep.rel_residual:.2e}, |A| {rep.n_active} "
          f"({rep.n_active / nn:.3f} of phi nodes), t {rep.t_total_s:.3f} s", flush=True)
    assert rep.converged and rep.rel_residual <= 1e-8
    lev = oracle_level(s)
    active = ((mk >> 3) & 1).astype(bool) & ~lev.hole_node
    assert np.allclose(Un[d * nn:][active], Uold[d * nn:][active], atol=1e-12)
    # sampled free displacement rows of A(U_{k+1}) vanish (linear in u for fixed phi~)
    mat = model.Material(**s["material"])
    cons = model.constrained_dofs(lev, s["faces"], active, W.extra_constraint_bits(s))
    rows = sample_rows(s, lev, n=n_samples(s, 1500), seed=7)
    rows = rows[(rows < d * nn) & ~cons[rows]]
    A1 = model.residual_rows(lev, mat, Un, phit, rows)
    A0 = model.residual_rows(lev, mat, U, phit, rows)
    # A_u(U1) on free rows is minus the linear residual there: bounded by 1e-8 ||R~||
    bound = 2e-8 * rep.rhs_norm + 1e-13 * np.linalg.norm(A0)
    print(f"  sampled free u-rows: |A(U1)| = {np.linalg.norm(A1):.2e} (|A(U0)| = {np.linalg.norm(A0):.2e}, "
          f"bound {bound:.2e})", flush=True)
    assert np.linalg.norm(A1) <= bound
