"""C ABI checks that need no GPU: the library loads, exports every declared symbol, validates arguments."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "pff.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_header_symbol():
    from paper_1902_08112_amd import pff
    L = pff.lib()
    syms = header_symbols()
    assert len(syms) >= 20
    for name in syms:
        assert hasattr(L, name), name
    assert sorted(pff.SIGNATURES) == syms


def test_status_strings_and_defaults():
    from paper_1902_08112_amd import pff
    assert pff.pf_status_string(0) == "PF_OK"
    assert pff.pf_status_string(6) == "PF_ERR_NONFINITE"
    o = pff.pf_default_options()
    assert o.cheb_degree == 4 and abs(o.cheb_ratio - 5) < 1e-15 and abs(o.cheb_safety - 1.2) < 1e-15
    assert o.eig_cg_steps == 10 and o.coarse_degree == 20 and abs(o.coarse_lo_factor - 0.9) < 1e-15
    assert abs(o.pdas_c - 100) < 1e-15 and o.gmres_restart == 50 and abs(o.gmres_rtol - 1e-8) < 1e-20
    assert o.gmres_atol == 0.0 and o.preconditioner == pff.PF_PREC_FULL and o.stress_split == pff.PF_SPLIT_NONE


@pytest.mark.parametrize("field,value,code", [("dim", 4, 2), ("degree", 3, 2), ("n_levels", 0, 1),
                                              ("domain", 7, 1), ("dirichlet_faces", 1 << 7, 1)])
def test_mesh_validation(field, value, code):
    from paper_1902_08112_amd import pff
    m = pff.make_mesh(3, 1, (8, 8, 8), (1, 1, 1), 0, 3, 63)
    setattr(m, field, value)
    with pytest.raises(pff.PffError) as e:
        pff.pf_workspace_size(m)
    assert e.value.status == code


def test_divisibility_and_lshape_checks():
    from paper_1902_08112_amd import pff
    m = pff.make_mesh(3, 1, (10, 8, 8), (1, 1, 1), 0, 3, 63)
    with pytest.raises(pff.PffError):
        pff.pf_workspace_size(m)
    m = pff.make_mesh(3, 1, (4, 4, 4), (1, 1, 1), pff.PF_LSHAPE, 3, 4)   # coarsest 1 cell: odd
    with pytest.raises(pff.PffError):
        pff.pf_workspace_size(m)


def test_setup_validates_before_device_work():
    """Bad material or a missing workspace fail before any HIP call (works without a GPU)."""
    from paper_1902_08112_amd import pff
    m = pff.make_mesh(2, 1, (8, 8), (1, 1), 0, 2, 15)
    o = pff.pf_default_options()
    n = pff.pf_workspace_size(m, o)
    assert n > 0
    for bad in [dict(E=-1.0), dict(nu=0.5), dict(G_c=0.0), dict(eps=0.0), dict(kappa=1.0), dict(pressure=float("nan"))]:
        args = dict(E=1.0, nu=0.3, G_c=1.0, eps=0.1, kappa=1e-10, pressure=1e-3)
        args.update(bad)
        with pytest.raises(pff.PffError) as e:
            pff.pf_setup(m, args["E"], args["nu"], args["G_c"], args["eps"], args["kappa"], args["pressure"], o,
                         0x1000, n, 0)
        assert e.value.status == pff.PF_ERR_INVALID_ARG
    with pytest.raises(pff.PffError) as e:
        pff.pf_setup(m, 1.0, 0.3, 1.0, 0.1, 1e-10, 0.0, o, None, n, 0)
    assert e.value.status == pff.PF_ERR_WORKSPACE
    with pytest.raises(pff.PffError) as e:
        pff.pf_setup(m, 1.0, 0.3, 1.0, 0.1, 1e-10, 0.0, o, 0x1000, n - 1, 0)
    assert e.value.status == pff.PF_ERR_WORKSPACE
    with pytest.raises(pff.PffError) as e:
        pff.pf_setup(m, 1.0, 0.3, 1.0, 0.1, 1e-10, 0.0, o, 0x1001, n, 0)
    assert e.value.status == pff.PF_ERR_WORKSPACE


def test_options_validation():
    from paper_1902_08112_amd import pff
    m = pff.make_mesh(2, 1, (8, 8), (1, 1), 0, 2, 15)
    for field, value in [("vcycle_precision", 3), ("cheb_degree", 0), ("cheb_ratio", 1.0), ("eig_cg_steps", 0),
                         ("gmres_restart", 0), ("gmres_rtol", 0.0), ("pdas_c", float("inf")),
                         ("gmres_atol", -1.0), ("preconditioner", 2), ("stress_split", 2)]:
        o = pff.pf_default_options()
        setattr(o, field, value)
        with pytest.raises(pff.PffError):
            pff.pf_workspace_size(m, o)


def test_null_context_calls_fail_cleanly():
    from paper_1902_08112_amd import pff
    L = pff.lib()
    assert L.pf_jacobian_apply(None, 0, 0, None, None, None) == pff.PF_ERR_INVALID_ARG
    assert L.pf_vcycle(None, 0, None, None, None) == pff.PF_ERR_INVALID_ARG
    assert L.pf_newton_step(None, None, None, None, None, None) == pff.PF_ERR_INVALID_ARG
    assert "NULL" in pff.pf_last_error()
    L.pf_destroy(None)


def test_workspace_scales_with_restart():
    from paper_1902_08112_amd import pff
    m = pff.make_mesh(3, 1, (16, 16, 16), (1, 1, 1), 0, 3, 63)
    o = pff.pf_default_options()
    a = pff.pf_workspace_size(m, o)
    o.gmres_restart = 10
    b = pff.pf_workspace_size(m, o)
    nd = 4 * 17 ** 3
    assert a - b >= 2 * 40 * nd * 8        # V and Z lose 40 vectors each
