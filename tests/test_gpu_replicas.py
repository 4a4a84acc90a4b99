"""Scaled-down replicas of the two large workloads (the 256^3 L-shape and the 96^3 two-crack Q2
mesh: the same recipes, eps at the same multiple of h, on 48^3 and 12^3 cells), each solved for
one Newton step by the FP64 oracle (assembled operators, V-cycle-preconditioned FGMRES to 1e-8)
and by the library with the FP64 and the FP32 V-cycle: the error of each library result against
the oracle's update, and the oracle's own residual of the library's update (Algorithm 1,
steps 3-6).  The oracle part takes about a minute per case on one core."""
import time

import numpy as np
import pytest

import workloads as W
from gpu_common import dev, gpu_solver, host, oracle_hierarchy, oracle_residual_of, rel_err

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

CASES = [("cfg5_3d_q1_lshape_256", 48, 4), ("cfg3_3d_q2_96", 12, 3)]


@pytest.mark.parametrize("base,n,levels", CASES)
def test_replica_newton_step_against_oracle(base, n, levels):
    from oracle import newton
    from paper_1902_08112_amd import PF_F32, PF_F64
    s = W.scaled(W.config(base), n, levels)
    U, Uold, phit = W.make_state(s)
    print(f"[case] replica {s['name']}, {levels} levels: oracle hierarchy", flush=True)
    t0 = time.perf_counter()
    H = oracle_hierarchy(s)
    print(f"  oracle Newton step ({H.fine.n_dofs} stored DoFs)", flush=True)
    ref = newton.newton_step(H, U, Uold, phit)
    live = int((~H.fine.hole_node).sum())
    print(f"  oracle: {ref['info']['iters']} FGMRES iterations, |A| {ref['n_active']} "
          f"({ref['n_active'] / live:.4f} of the phi-nodes), {time.perf_counter() - t0:.1f} s", flush=True)
    S = gpu_solver(s)
    for prec, tag in ((PF_F64, "FP64"), (PF_F32, "FP32")):
        S.set_vcycle_precision(prec)
        Ud = dev(U)
        st, rep = S.newton_step(Ud, dev(Uold), dev(phit))
        dU = host(Ud) - U
        e = rel_err(dU, ref["dU"])
        res = oracle_residual_of(ref, dU)
        print(f"  library, {tag} V-cycle: {rep.gmres_iters} FGMRES iterations, rel res {rep.rel_residual:.2e}, "
              f"|A| {rep.n_active}; |dU - dU_oracle| / |dU_oracle| = {e:.2e}, oracle residual {res:.2e}",
              flush=True)
        assert rep.converged and rep.rel_residual <= 1e-8
        assert rep.n_active == ref["n_active"]
        # both solves reach 1e-8 of the same linear system
        assert res <= 1.1e-8
        assert e <= 1e-5
        d, nn = s["dim"], H.fine.n_nodes
        act = ref["active"]
        assert np.allclose(host(Ud)[d * nn:][act], Uold[d * nn:][act], atol=1e-12)
    S.close()
