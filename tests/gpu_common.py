"""Shared set-up of the GPU parity tests: one oracle hierarchy and one library context per workload."""
import numpy as np

import workloads as W
from oracle import mg, model

EIG_DUMMY = dict(u=(0.5, 2.0), phi=(0.5, 2.0))


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
