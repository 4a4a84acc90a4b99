"""Shared set-up of the GPU parity tests: one oracle hierarchy and one library context per workload."""
import numpy as np

import workloads as W
from oracle import mg, model

EIG_DUMMY = dict(u=(0.5, 2.0), phi=(0.5, 2.0))


def oracle_bounds(H):
    """The oracle's own eigenvalue estimates per level: [lam_min_u, lam_max_u, lam_min_phi, lam_max_phi]."""
    return [[m.eig["u"][0], m.eig["u"][1], m.eig["phi"][0], m.eig["phi"][1]] for m in H.mg]


def inject_bounds(S, H):
    """Fix the library's smoother intervals to the oracle's estimates (oracle -> library, never back)."""
    for l, b in enumerate(oracle_bounds(H)):
        S.set_eig_bounds(l, b)


def inject_batch_bounds(BS, b, H):
    for l, e in enumerate(oracle_bounds(H)):
        BS.set_eig_bounds(l, b, e)


def torch_mod():
    import torch
    return torch


def oracle_hierarchy(s, opts=None):
    mat = model.Material(**s["material"])
    return mg.Hierarchy(s["dim"], s["degree"], s["n_cells"], s["extent"], s["domain"], s["n_levels"], s["faces"],
                        mat, opts=opts, extra_u_bits=W.extra_constraint_bits(s))


def gpu_solver(s, **opt):
    from paper_1902_08112_amd import pff
    torch = torch_mod()
    S = pff.solver_from_spec(s, **opt)
    bits = W.extra_constraint_bits(s)
    if bits is not None:
        S.set_constraints(torch.from_numpy(bits).cuda())
    return S


def dev(a):
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def mask_to_dofs(mask, d):
    """Per-node constraint bits -> per-DoF bool (component-major)."""
    mask = np.asarray(mask).astype(np.int64)
    parts = [(mask >> c) & 1 for c in range(d)] + [(mask >> 3) & 1]
    return np.concatenate(parts).astype(bool)


def rel_err(a, b):
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def block_rel_errs(a, b, nn, d):
    out = {}
    out["u"] = rel_err(a[: d * nn], b[: d * nn])
    out["phi"] = rel_err(a[d * nn:], b[d * nn:])
    return out


def oracle_residual_of(ref, dU):
    """True relative residual ||R~ - G~ dU|| / ||R~|| of an update, with the oracle's own R~ and G~."""
    return float(np.linalg.norm(ref["Rt"] - ref["Gt"] @ dU) / np.linalg.norm(ref["Rt"]))


def tie_band(v):
    """Nodes whose active-set decision value is at rounding level (|v| <= 1e-10 max|v|)."""
    v = np.asarray(v)
    return int((np.abs(v) <= 1e-10 * np.abs(v).max()).sum())
