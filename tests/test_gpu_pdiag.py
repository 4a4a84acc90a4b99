"""The block-diagonal preconditioner P_diag = diag(MG(U~), MG(P~)) (Sec. 3.3) on the GPU vs the oracle.

Same bars as the full cycle: the FP64 V-cycle agrees with the oracle's P_diag to 1e-11 relative,
the FP32-level cycle to 1e-4 (the FP32 rounding of the smoothing carried through the cycle), and
Newton steps solved to 1e-8 with either side's P_diag agree to 1e-5 relative.  The single-context
and the batched solver are both covered.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import dev, gpu_solver, host, inject_batch_bounds, inject_bounds, oracle_hierarchy, rel_err
from oracle import mg

pytestmark = pytest.mark.gpu


def diag_opts():
    return mg.Options(preconditioner="diag")


@pytest.mark.parametrize("name", ["small2d", "tiny3d_q2", "small3d", "small_lshape"])
def test_block_diagonal_vcycle_matches_oracle(name):
    from paper_1902_08112_amd import pff
    print(f"[case] P_diag vcycle {name}", flush=True)
    s = W.config(name)
    U, phit = W.random_linearization(s, 19)
    act = W.random_active(s, 20, 0.1)
    S = gpu_solver(s, preconditioner=pff.PF_PREC_DIAG)
    S.set_linearization(dev(U), dev(phit), dev(act))
    H = oracle_hierarchy(s, opts=diag_opts())
    H.set_linearization(U, phit, act)
    inject_bounds(S, H)
    r = np.random.default_rng(23).uniform(-1, 1, H.fine.n_dofs)
    z_ref = H.vcycle(r)
    z = host(S.vcycle(dev(r)))
    e = rel_err(z, z_ref)
    z32 = host(S.vcycle(dev(r), pff.PF_F32))
    e32 = rel_err(z32, z_ref)
    print(f"  vcycle rel {e:.2e}, FP32 levels rel {e32:.2e}", flush=True)
    assert e <= 1e-11 and e32 <= 1e-4
    # block diagonal on the device too: r_u alone leaves the phi part at zero
    du = s["dim"] * H.fine.n_nodes
    ru = r.copy()
    ru[du:] = 0.0
    assert np.abs(host(S.vcycle(dev(ru)))[du:]).max() == 0.0


@pytest.mark.parametrize("name,prec", [("cfg1_2d_q1_32", "f64"), ("small3d", "f32"), ("small_lshape", "f64")])
def test_newton_step_with_block_diagonal_preconditioner(name, prec):
    from oracle import newton
    from paper_1902_08112_amd import pff
    print(f"[case] P_diag newton {name} {prec}", flush=True)
    s = dict(W.config(name))
    s["vcycle"] = prec
    U, Uold, phit = W.make_state(s)
    H = oracle_hierarchy(s, opts=diag_opts())
    ref = newton.newton_step(H, U, Uold, phit)
    S = gpu_solver(s, preconditioner=pff.PF_PREC_DIAG)
    Ud = dev(U)
    _, rep = S.newton_step(Ud, dev(Uold), dev(phit))
    Sf = gpu_solver(s)
    _, rep_full = Sf.newton_step(dev(U), dev(Uold), dev(phit))
    e = rel_err(host(Ud) - U, ref["dU"])
    print(f"  P_diag gmres {rep.gmres_iters} (oracle {ref['info']['iters']}), P_full gmres {rep_full.gmres_iters}; "
          f"rel res {rep.rel_residual:.2e}; |dU - dU_oracle|/|dU_oracle| = {e:.2e}", flush=True)
    assert rep.converged and rep.rel_residual <= 1e-8
    assert rep.n_active == ref["n_active"]
    assert e <= 1e-5


def test_batch_block_diagonal_vcycle_matches_oracle():
    from paper_1902_08112_amd import pff
    specs = [W.spec(f"d{i}", 2, 1, n, 3, eps_h=2.0, pressure=1e-3,
                    cracks=[("segment", (0.4, 0.5), (0.6, 0.5))], u_amp=1e-3, u_seed=200 + i)
             for i, n in enumerate([8, 16, 24])]
    print(f"[case] batch P_diag vcycle n={len(specs)}", flush=True)
    o = pff.pf_default_options()
    o.preconditioner = pff.PF_PREC_DIAG
    BS = pff.BatchSolver(specs, o)
    Us, pts, acts = [], [], []
    for b, s in enumerate(specs):
        U, phit = W.random_linearization(s, 50 + b)
        Us.append(U), pts.append(phit), acts.append(W.random_active(s, 60 + b, 0.1))
    BS.set_linearization(BS.pack(Us), BS.pack(pts, nodes=True), BS.pack(acts, nodes=True))
    rs = [np.random.default_rng(70 + b).uniform(-1, 1, u.size) for b, u in enumerate(Us)]
    Hs = []
    for b, s in enumerate(specs):
        H = oracle_hierarchy(s, opts=diag_opts())
        H.set_linearization(Us[b], pts[b], acts[b])
        inject_batch_bounds(BS, b, H)
        Hs.append(H)
    zs = BS.unpack(BS.vcycle(BS.pack(rs)))
    for b, s in enumerate(specs):
        err = rel_err(zs[b], Hs[b].vcycle(rs[b]))
        print(f"  inst {b}: rel {err:.2e}", flush=True)
        assert err <= 1e-11
