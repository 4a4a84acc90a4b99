"""Edge cases of the GPU path against the oracle.

* one-level hierarchies: the V-cycle is the coarse Chebyshev solve alone (every coarse-solve
  path: the dense matrix, the single-workgroup kernel, per-step launches);
* anisotropic non-cubic meshes with non-unit aspect ratio, whose marching tiles, bricks and
  chunks are ragged in every direction;
* a phase field that is active on every node (every phi row is an identity row);
* the degenerate material kappa = 0 (no residual stiffness: g(0) = 0) with p = 0;
* the Chebyshev steps fused into marching-tile block applies on ragged tiles and chunks.
Same bars as the main parity tests: FP64 operators 1e-12, FP32 2e-6, V-cycles 1e-11, Newton
updates 1e-5 (both solves at 1e-8).
"""
import math

import numpy as np
import pytest

import workloads as W
from gpu_common import EIG_DUMMY, dev, gpu_solver, host, inject_bounds, oracle_hierarchy, rel_err
from oracle import newton

pytestmark = pytest.mark.gpu


def custom(name, dim, degree, cells, levels, extent=None, **kw):
    s = W.spec(name, dim, degree, cells[0], levels, **kw)
    s["n_cells"] = tuple(cells)
    s["extent"] = tuple(extent or (1.0,) * dim)
    h = math.sqrt(sum((e / n) ** 2 for e, n in zip(s["extent"], s["n_cells"])))
    s["h"] = h
    s["material"] = dict(s["material"], eps=2.0 * h)
    return s


CASES = {
    "one_level_2d": custom("one_level_2d", 2, 1, (6, 4), 1, cracks=[("segment", (0.3, 0.5), (0.7, 0.5))],
                           u_amp=1e-3, u_seed=1),
    "one_level_3d": custom("one_level_3d", 3, 1, (4, 4, 2), 1, cracks=[("disc", (0.5, 0.5, 0.5), 0.3)],
                           u_amp=1e-3, u_seed=2),
    "one_level_3d_q2": custom("one_level_3d_q2", 3, 2, (2, 2, 2), 1, cracks=[("disc", (0.5, 0.5, 0.5), 0.3)],
                              u_amp=1e-3, u_seed=3),
    "aniso_3d": custom("aniso_3d", 3, 1, (24, 12, 8), 3, extent=(1.5, 1.0, 0.5),
                       cracks=[("disc", (0.75, 0.5, 0.25), 0.2)], u_amp=1e-3, u_seed=4),
    "aniso_2d": custom("aniso_2d", 2, 1, (40, 12), 3, extent=(2.0, 0.6),
                       cracks=[("segment", (0.7, 0.3), (1.3, 0.3))], u_amp=1e-3, u_seed=5),
    "aniso_3d_q2": custom("aniso_3d_q2", 3, 2, (8, 4, 4), 2, extent=(1.0, 0.5, 0.5),
                          cracks=[("disc", (0.5, 0.25, 0.25), 0.15)], u_amp=1e-3, u_seed=6),
    "kappa0_p0": custom("kappa0_p0", 2, 1, (16, 16), 3, kappa=0.0, pressure=0.0,
                        cracks=[("segment", (0.3, 0.5), (0.7, 0.5))], u_amp=1e-3, u_seed=7),
}


def setup(name, seed=1, active=None):
    s = CASES[name]
    print(f"[case] edge {name} cells {s['n_cells']} levels {s['n_levels']}", flush=True)
    U, phit = W.random_linearization(s, seed)
    act = W.random_active(s, seed + 1, 0.1) if active is None else active(s)
    H = oracle_hierarchy(s)
    H.set_linearization(U, phit, act, eig_bounds=[EIG_DUMMY] * s["n_levels"])
    S = gpu_solver(s)
    S.set_linearization(dev(U), dev(phit), dev(act))
    return s, U, phit, act, H, S


def check_operators(s, H, S, variants):
    from paper_1902_08112_amd import pff
    torch = __import__("torch")
    for l in range(s["n_levels"]):
        x = np.random.default_rng(100 + l).uniform(-1, 1, H.levels[l].n_dofs)
        refG, refB = H.mg[l].G @ x, H.mg[l].B @ x
        for v, zc in variants:
            if v is not None and s["degree"] == 1:
                for mode in (0, 1):
                    pff.pf_set_tuning(S.ctx, l, pff.PF_F64, mode, v, zc)
                    pff.pf_set_tuning(S.ctx, l, pff.PF_F32, mode, v, zc)
            y, yb = host(S.jacobian_apply(l, dev(x))), host(S.block_apply(l, dev(x)))
            y32 = host(S.jacobian_apply(l, dev(x).to(torch.float32))).astype(np.float64)
            e, eb, e32 = rel_err(y, refG), rel_err(yb, refB), rel_err(y32, refG)
            print(f"  level {l} shape {v},{zc}: {e:.1e} {eb:.1e} FP32 {e32:.1e}", flush=True)
            assert e <= 1e-12 and eb <= 1e-12 and e32 <= 2e-6
            c = H.mg[l].constrained
            assert np.array_equal(y[c], x[c])


def check_vcycle(s, U, phit, act, H, S):
    from paper_1902_08112_amd import pff
    H.set_linearization(U, phit, act)
    inject_bounds(S, H)
    r = np.random.default_rng(23).uniform(-1, 1, H.fine.n_dofs)
    z_ref = H.vcycle(r)
    for mode in (pff.PF_COARSE_AUTO, pff.PF_COARSE_FUSED, pff.PF_COARSE_STEPS):
        S.set_coarse_mode(mode)
        e = rel_err(host(S.vcycle(dev(r))), z_ref)
        print(f"  coarse mode {mode}: vcycle rel {e:.2e}", flush=True)
        assert e <= 1e-11
    S.set_coarse_mode(pff.PF_COARSE_AUTO)


def check_newton(s):
    U, Uold, phit = W.make_state(s)
    H = oracle_hierarchy(s)
    ref = newton.newton_step(H, U, Uold, phit)
    S = gpu_solver(s)
    Ud = dev(U)
    _, rep = S.newton_step(Ud, dev(Uold), dev(phit))
    e = rel_err(host(Ud) - U, ref["dU"])
    print(f"  newton: gmres {rep.gmres_iters} (oracle {ref['info']['iters']}), rel res {rep.rel_residual:.1e}, "
          f"|A| {rep.n_active} (oracle {ref['n_active']}), rel {e:.1e}", flush=True)
    assert rep.converged and rep.rel_residual <= 1e-8
    assert rep.n_active == ref["n_active"]
    assert e <= 1e-5


@pytest.mark.parametrize("name", ["one_level_2d", "one_level_3d", "one_level_3d_q2"])
def test_one_level_hierarchy(name):
    s, U, phit, act, H, S = setup(name)
    check_operators(s, H, S, [(None, None)])
    check_vcycle(s, U, phit, act, H, S)
    check_newton(s)


@pytest.mark.parametrize("name", ["aniso_3d", "aniso_2d", "aniso_3d_q2"])
def test_anisotropic_ragged_meshes(name):
    s, U, phit, act, H, S = setup(name, seed=5)
    variants = [(2, -1), (3, -1), (4, -1), (0, 3), (0, 5)] + ([(1, 3), (1, 7), (5, 3), (5, 7)] if s["dim"] == 3 else [])
    check_operators(s, H, S, variants if s["degree"] == 1 else [(None, None)])
    check_vcycle(s, U, phit, act, H, S)
    check_newton(s)


@pytest.mark.parametrize("name", ["aniso_3d", "one_level_3d"])
def test_fused_smoother_on_ragged_tiles(name):
    """The Chebyshev steps fused into marching-tile B~ applies on meshes whose tiles and chunks
    are ragged (and on a one-level hierarchy, where the coarse solve's per-step launches use
    them): V-cycles match the oracle in every coarse-solve path."""
    from paper_1902_08112_amd import pff
    s, U, phit, act, H, S = setup(name, seed=21)
    for l in range(s["n_levels"]):
        for prec in (pff.PF_F64, pff.PF_F32):
            pff.pf_set_tuning(S.ctx, l, prec, 1, 1, 3)
    S.set_smoother_fusion(pff.PF_FUSE_ALWAYS)
    check_vcycle(s, U, phit, act, H, S)


def test_phase_field_active_everywhere():
    name = "aniso_3d"
    s, U, phit, act, H, S = setup(name, seed=9, active=lambda s: W.random_active(s, 0, 1.0 + 1e-9))
    assert act.sum() == act.size
    check_operators(s, H, S, [(2, -1), (0, 8)])
    check_vcycle(s, U, phit, act, H, S)


def test_kappa_zero_and_no_pressure():
    s, U, phit, act, H, S = setup("kappa0_p0", seed=13)
    check_operators(s, H, S, [(2, -1), (0, 8)])
    check_vcycle(s, U, phit, act, H, S)
    check_newton(s)
