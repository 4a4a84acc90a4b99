"""The allocation-free entry point pf_energies_noalloc (GPU), through the C ABI: on two calls in a
row, the second on a smaller mesh, it must give what pf_energies gives on the same state (the same
kernels and reduction grid, so the same bits), and match the oracle's energies to 1e-12."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from gpu_common import dev
from oracle import fe, model, quantities

pytestmark = pytest.mark.gpu


def _energies_both(name):
    import torch
    from paper_1902_08112_amd import pff
    s = W.config(name)
    U, _, _ = W.make_state(s)
    S = pff.solver_from_spec(s)
    Ud = dev(U)
    ref = S.energies(Ud)                                   # pf_energies: workspace scratch, read-back
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    st = pff.lib().pf_energies_noalloc(S.ctx, C.c_void_p(Ud.data_ptr()), C.c_void_p(out.data_ptr()),
                                       C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == pff.PF_OK, pff.pf_last_error()
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    # argument checks come before any device work
    assert pff.lib().pf_energies_noalloc(S.ctx, C.c_void_p(Ud.data_ptr()), None, None) == pff.PF_ERR_INVALID_ARG
    assert pff.lib().pf_energies_noalloc(None, C.c_void_p(Ud.data_ptr()), C.c_void_p(out.data_ptr()), None) \
        == pff.PF_ERR_INVALID_ARG
    S.close()
    mat = model.Material(**s["material"])
    lev = fe.Level(s["dim"], s["degree"], s["n_cells"], s["extent"], s["domain"])
    orc = quantities.energies(lev, mat, U)
    return s, np.array(ref), got, np.array(orc)


def test_noalloc_energies_two_calls():
    # the first call on the larger mesh leaves its partial sums in the shared scratch; the second,
    # on a smaller mesh with fewer reduction blocks, must not pick any of them up
    for name in ("small3d", "tiny3d"):
        s, ref, got, orc = _energies_both(name)
        print(f"{name}: noalloc {got}, pf_energies {ref}, oracle {orc}", flush=True)
        assert np.array_equal(got, ref), (name, got, ref)
        assert np.all(np.abs(got - orc) <= 1e-12 * np.abs(orc).max()), (name, got, orc)
