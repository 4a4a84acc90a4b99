"""Energies and face loads (pf_energies, pf_boundary_traction) vs the oracle's quantities.

FP64 reductions over cells in a different order than the oracle's: 1e-12 relative per
quantity (1e-12 of the largest face load for the traction components).
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import dev, gpu_solver, oracle_hierarchy
from oracle import model, quantities

pytestmark = pytest.mark.gpu


def check(s, U):
    H = oracle_hierarchy(s)
    mat = model.Material(**s["material"])
    S = gpu_solver(s)
    dU = dev(U)
    ec, eb = S.energies(dU)
    rc, rb = quantities.energies(H.fine, mat, U)
    print(f"  energies GPU ({ec:.12e}, {eb:.12e}) oracle ({rc:.12e}, {rb:.12e})", flush=True)
    assert abs(ec - rc) <= 1e-12 * abs(rc) and abs(eb - rb) <= 1e-12 * abs(rb)
    ref = [quantities.boundary_traction(H.fine, mat, U, f) for f in range(2 * s["dim"])]
    scale = max(np.abs(r).max() for r in ref)
    for f in range(2 * s["dim"]):
        t = np.array(S.boundary_traction(dU, f))
        assert np.abs(t - ref[f]).max() <= 1e-12 * scale, (f, t, ref[f])
    return S, dU


@pytest.mark.parametrize("name", ["small2d", "tiny2d_q2", "small3d", "small3d_q2", "small_lshape"])
def test_quantities_match_oracle(name):
    s = W.config(name)
    print(f"[case] quantities {name}", flush=True)
    U, Uold, phit = W.make_state(s)
    check(s, U)
    Ur, _ = W.random_linearization(s, 41)
    check(s, Ur)


def test_quantities_full_size():
    s = W.config("cfg2_3d_q1_64")
    print("[case] quantities cfg2_3d_q1_64", flush=True)
    U, Uold, phit = W.make_state(s)
    S, dU = check(s, U)
    import time
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        S.energies(dU)
    t_e = (time.perf_counter() - t0) / 10
    t0 = time.perf_counter()
    for _ in range(10):
        S.boundary_traction(dU, 5)
    t_t = (time.perf_counter() - t0) / 10
    print(f"  energies {t_e * 1e6:.0f} us, face load {t_t * 1e6:.0f} us per call (synchronizing)", flush=True)
