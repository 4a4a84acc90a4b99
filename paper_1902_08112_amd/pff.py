"""ctypes binding of libpff.so (the C ABI declared in include/pff.h).

Argument marshalling only: every computation runs in the HIP library.  The
pf_* functions mirror the C entry points one to one (pointers are Python ints);
``Solver`` is a small convenience wrapper that keeps a torch-allocated
workspace and passes tensor data pointers and the current HIP stream.
The library must be built (``python -m paper_1902_08112_amd.build``); loading
fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import json
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpff.so")

PF_OK, PF_ERR_INVALID_ARG, PF_ERR_UNSUPPORTED, PF_ERR_DEVICE = 0, 1, 2, 3
PF_ERR_WORKSPACE, PF_ERR_NOT_CONVERGED, PF_ERR_NONFINITE = 4, 5, 6
PF_F64, PF_F32 = 0, 1
PF_PREC_FULL, PF_PREC_DIAG = 0, 1
PF_SPLIT_NONE, PF_SPLIT_MIEHE = 0, 1
PF_COARSE_AUTO, PF_COARSE_FUSED, PF_COARSE_STEPS = 0, 1, 2
PF_KTIME_JACOBIAN, PF_KTIME_BLOCK, PF_KTIME_BLOCK_CHEB = 1, 2, 4
PF_FUSE_OFF, PF_FUSE_TUNED, PF_FUSE_ALWAYS = 0, 1, 2
PF_BOX, PF_LSHAPE = 0, 1
PF_MASK_PHI = 8


class PffError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


class Mesh(C.Structure):
    _fields_ = [("dim", C.c_int), ("degree", C.c_int), ("n_cells", C.c_int * 3), ("extent", C.c_double * 3),
                ("domain", C.c_int), ("n_levels", C.c_int), ("dirichlet_faces", C.c_uint)]


class Options(C.Structure):
    _fields_ = [("vcycle_precision", C.c_int), ("cheb_degree", C.c_int), ("cheb_ratio", C.c_double),
                ("cheb_safety", C.c_double), ("eig_cg_steps", C.c_int), ("coarse_degree", C.c_int),
                ("coarse_sweeps", C.c_int), ("coarse_lo_factor", C.c_double), ("gmres_restart", C.c_int),
                ("gmres_max_iter", C.c_int), ("gmres_rtol", C.c_double), ("pdas_c", C.c_double),
                ("eig_seed", C.c_uint64), ("gmres_atol", C.c_double), ("preconditioner", C.c_int),
                ("stress_split", C.c_int)]


class NewtonReport(C.Structure):
    _fields_ = [("gmres_iters", C.c_int), ("converged", C.c_int), ("rel_residual", C.c_double),
                ("rhs_norm", C.c_double), ("n_active", C.c_int64), ("t_residual_s", C.c_double),
                ("t_setup_s", C.c_double), ("t_solve_s", C.c_double), ("t_total_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PdasReport(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("gmres_iters_total", C.c_int),
                ("n_active", C.c_int64), ("n_changed", C.c_int64), ("residual_norm", C.c_double),
                ("t_total_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LevelInfo(C.Structure):
    _fields_ = [("n_cells", C.c_int * 3), ("n_nodes_axis", C.c_int * 3), ("n_nodes", C.c_int64),
                ("n_dofs", C.c_int64), ("n_active_cells", C.c_int64), ("h", C.c_double * 3),
                ("precision", C.c_int), ("n_domain_nodes", C.c_int64)]


_lib = None
VP, I, D, I64 = C.c_void_p, C.c_int, C.c_double, C.c_int64
SIGNATURES = {
    "pf_default_options": (None, [C.POINTER(Options)]),
    "pf_workspace_size": (I, [C.POINTER(Mesh), C.POINTER(Options), C.POINTER(C.c_size_t)]),
    "pf_setup": (I, [C.POINTER(Mesh), D, D, D, D, D, D, C.POINTER(Options), VP, C.c_size_t, VP, C.POINTER(VP)]),
    "pf_set_constraints": (I, [VP, VP, VP]),
    "pf_set_linearization": (I, [VP, VP, VP, VP, VP]),
    "pf_jacobian_apply": (I, [VP, I, I, VP, VP, VP]),
    "pf_block_apply": (I, [VP, I, I, VP, VP, VP]),
    "pf_residual": (I, [VP, VP, VP, VP, VP]),
    "pf_get_diagonal": (I, [VP, I, VP, VP]),
    "pf_get_lumped_mass": (I, [VP, VP, VP]),
    "pf_get_level_data": (I, [VP, I, VP, VP, VP, VP]),
    "pf_active_set": (I, [VP, VP, VP, VP, VP, VP, C.POINTER(I64), VP]),
    "pf_transfer": (I, [VP, I, I, VP, VP, VP]),
    "pf_get_eig_bounds": (I, [VP, I, C.POINTER(D)]),
    "pf_set_eig_bounds": (I, [VP, I, C.POINTER(D)]),
    "pf_vcycle": (I, [VP, I, VP, VP, VP]),
    "pf_newton_step": (I, [VP, VP, VP, VP, C.POINTER(NewtonReport), VP]),
    "pf_get_level_info": (I, [VP, I, C.POINTER(LevelInfo)]),
    "pf_set_vcycle_precision": (I, [VP, I]),
    "pf_autotune": (I, [VP, I, VP]),
    "pf_set_graphs": (I, [VP, I]),
    "pf_get_graph_captures": (I, [VP, C.POINTER(C.c_int64)]),
    "pf_set_coarse_mode": (I, [VP, I]),
    "pf_get_tuning": (I, [VP, I, I, I, C.POINTER(I), C.POINTER(I)]),
    "pf_set_tuning": (I, [VP, I, I, I, I, I]),
    "pf_tuning_report": (I, [VP, C.c_char_p, C.c_size_t]),
    "pf_set_kernel_timing": (I, [VP, I, I]),
    "pf_set_smoother_fusion": (I, [VP, I]),
    "pf_set_level_fusion": (I, [VP, I, I, I]),
    "pf_pdas_solve": (I, [VP, VP, VP, VP, I, D, C.POINTER(PdasReport), VP]),
    "pf_extrapolate": (I, [VP, VP, VP, D, VP, VP]),
    "pf_set_pressure": (I, [VP, D]),
    "pf_energies": (I, [VP, VP, C.POINTER(D), VP]),
    "pf_energies_noalloc": (I, [VP, VP, VP, VP]),
    "pf_boundary_traction": (I, [VP, VP, I, C.POINTER(D), VP]),
    "pf_get_kernel_timing": (I, [VP, C.POINTER(I), C.POINTER(D), C.POINTER(D), C.POINTER(D)]),
    "pf_get_kernel_timing_op": (I, [VP, I, C.POINTER(C.c_int64), C.POINTER(I), C.POINTER(D), C.POINTER(D),
                                    C.POINTER(D)]),
    "pf_batch_workspace_size": (I, [C.POINTER(Mesh), I, C.POINTER(Options), C.POINTER(C.c_size_t)]),
    "pf_batch_setup": (I, [C.POINTER(Mesh), C.POINTER(D), I, C.POINTER(Options), VP, C.c_size_t, VP,
                           C.POINTER(VP)]),
    "pf_batch_layout": (I, [VP, I, C.POINTER(I64), C.POINTER(I64)]),
    "pf_batch_set_constraints": (I, [VP, VP, VP]),
    "pf_batch_set_linearization": (I, [VP, VP, VP, VP, VP]),
    "pf_batch_jacobian_apply": (I, [VP, I, I, VP, VP, VP]),
    "pf_batch_vcycle": (I, [VP, I, VP, VP, VP]),
    "pf_batch_get_eig_bounds": (I, [VP, I, I, C.POINTER(D)]),
    "pf_batch_set_eig_bounds": (I, [VP, I, I, C.POINTER(D)]),
    "pf_batch_set_vcycle_precision": (I, [VP, I]),
    "pf_batch_set_graphs": (I, [VP, I]),
    "pf_batch_autotune": (I, [VP, I, VP]),
    "pf_batch_get_tuning": (I, [VP, I, I, I, C.POINTER(I), C.POINTER(I), C.POINTER(D)]),
    "pf_batch_set_tuning": (I, [VP, I, I, I, I, I]),
    "pf_batch_newton_step": (I, [VP, VP, VP, VP, C.POINTER(NewtonReport), VP]),
    "pf_batch_destroy": (None, [VP]),
    "pf_destroy": (None, [VP]),
    "pf_status_string": (C.c_char_p, [I]),
    "pf_last_error": (C.c_char_p, []),
}


def lib():
    """Load libpff.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # Load torch's HIP runtime first so libpff.so binds to the same runtime
        # (same soname) as the tensors and streams it is handed.
        try:
            import torch  # noqa: F401
        except ImportError:  # pragma: no cover - the C ABI itself does not need torch
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1902_08112_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(SIGNATURES)


def _check(status, what):
    if status != PF_OK:
        L = lib()
        raise PffError(status, f"{what}: {L.pf_status_string(status).decode()}: {L.pf_last_error().decode()}")


def check(status, what="pff"):
    _check(status, what)
    return status


# --------------------------------------------------------------------------
# one-to-one wrappers of the C entry points (pointers as ints)
# --------------------------------------------------------------------------
def pf_default_options():
    o = Options()
    lib().pf_default_options(C.byref(o))
    return o


def pf_workspace_size(mesh: Mesh, opt: Options = None) -> int:
    n = C.c_size_t(0)
    _check(lib().pf_workspace_size(C.byref(mesh), C.byref(opt) if opt else None, C.byref(n)), "pf_workspace_size")
    return n.value


def pf_setup(mesh, E, nu, G_c, eps, kappa, pressure, opt, ws_ptr, ws_bytes, stream=0):
    out = VP()
    _check(lib().pf_setup(C.byref(mesh), E, nu, G_c, eps, kappa, pressure, C.byref(opt) if opt else None,
                          ws_ptr, ws_bytes, stream, C.byref(out)), "pf_setup")
    return out.value


def pf_set_constraints(ctx, bits_ptr, stream=0):
    _check(lib().pf_set_constraints(ctx, bits_ptr, stream), "pf_set_constraints")


def pf_set_linearization(ctx, U_ptr, phit_ptr, active_ptr=None, stream=0):
    _check(lib().pf_set_linearization(ctx, U_ptr, phit_ptr, active_ptr, stream), "pf_set_linearization")


def pf_jacobian_apply(ctx, level, prec, x_ptr, y_ptr, stream=0):
    _check(lib().pf_jacobian_apply(ctx, level, prec, x_ptr, y_ptr, stream), "pf_jacobian_apply")


def pf_block_apply(ctx, level, prec, x_ptr, y_ptr, stream=0):
    _check(lib().pf_block_apply(ctx, level, prec, x_ptr, y_ptr, stream), "pf_block_apply")


def pf_residual(ctx, U_ptr, phit_ptr, R_ptr, stream=0):
    _check(lib().pf_residual(ctx, U_ptr, phit_ptr, R_ptr, stream), "pf_residual")


def pf_get_diagonal(ctx, level, out_ptr, stream=0):
    _check(lib().pf_get_diagonal(ctx, level, out_ptr, stream), "pf_get_diagonal")


def pf_get_lumped_mass(ctx, out_ptr, stream=0):
    _check(lib().pf_get_lumped_mass(ctx, out_ptr, stream), "pf_get_lumped_mass")


def pf_get_level_data(ctx, level, U_ptr, phit_ptr, mask_ptr, stream=0):
    _check(lib().pf_get_level_data(ctx, level, U_ptr, phit_ptr, mask_ptr, stream), "pf_get_level_data")


def pf_active_set(ctx, R_ptr, U_ptr, Uold_ptr, active_ptr, v_ptr=None, want_count=True, stream=0):
    n = I64(0)
    _check(lib().pf_active_set(ctx, R_ptr, U_ptr, Uold_ptr, active_ptr, v_ptr,
                               C.byref(n) if want_count else None, stream), "pf_active_set")
    return n.value


def pf_transfer(ctx, level, op, in_ptr, out_ptr, stream=0):
    _check(lib().pf_transfer(ctx, level, op, in_ptr, out_ptr, stream), "pf_transfer")


def pf_get_eig_bounds(ctx, level):
    out = (D * 4)()
    _check(lib().pf_get_eig_bounds(ctx, level, out), "pf_get_eig_bounds")
    return list(out)


def pf_set_eig_bounds(ctx, level, bounds):
    arr = None if bounds is None else (D * 4)(*bounds)
    _check(lib().pf_set_eig_bounds(ctx, level, arr), "pf_set_eig_bounds")


def pf_vcycle(ctx, prec, r_ptr, z_ptr, stream=0):
    _check(lib().pf_vcycle(ctx, prec, r_ptr, z_ptr, stream), "pf_vcycle")


def pf_newton_step(ctx, U_ptr, Uold_ptr, phit_ptr, stream=0, raise_on_error=True):
    rep = NewtonReport()
    st = lib().pf_newton_step(ctx, U_ptr, Uold_ptr, phit_ptr, C.byref(rep), stream)
    if raise_on_error:
        _check(st, "pf_newton_step")
    return st, rep


def pf_pdas_solve(ctx, U_ptr, Uold_ptr, phit_ptr, max_iter=50, tol_as=1e-10, stream=0, raise_on_error=True):
    rep = PdasReport()
    st = lib().pf_pdas_solve(ctx, U_ptr, Uold_ptr, phit_ptr, max_iter, tol_as, C.byref(rep), stream)
    if raise_on_error:
        _check(st, "pf_pdas_solve")
    return st, rep


def pf_extrapolate(ctx, phi1_ptr, phi2_ptr, theta, out_ptr, stream=0):
    _check(lib().pf_extrapolate(ctx, phi1_ptr, phi2_ptr, theta, out_ptr, stream), "pf_extrapolate")


def pf_set_pressure(ctx, pressure):
    _check(lib().pf_set_pressure(ctx, pressure), "pf_set_pressure")


def pf_get_level_info(ctx, level):
    info = LevelInfo()
    _check(lib().pf_get_level_info(ctx, level, C.byref(info)), "pf_get_level_info")
    return info


def pf_set_vcycle_precision(ctx, prec):
    _check(lib().pf_set_vcycle_precision(ctx, prec), "pf_set_vcycle_precision")


def pf_autotune(ctx, reps=20, stream=0):
    _check(lib().pf_autotune(ctx, reps, stream), "pf_autotune")


def pf_get_tuning(ctx, level, prec, mode):
    v, z = I(0), I(0)
    _check(lib().pf_get_tuning(ctx, level, prec, mode, C.byref(v), C.byref(z)), "pf_get_tuning")
    return v.value, z.value


def pf_set_tuning(ctx, level, prec, mode, variant, zc):
    _check(lib().pf_set_tuning(ctx, level, prec, mode, variant, zc), "pf_set_tuning")


def pf_tuning_report(ctx):
    buf = C.create_string_buffer(1 << 16)
    _check(lib().pf_tuning_report(ctx, buf, len(buf)), "pf_tuning_report")
    return json.loads(buf.value.decode())


def pf_destroy(ctx):
    lib().pf_destroy(ctx)


def pf_status_string(s):
    return lib().pf_status_string(s).decode()


def pf_last_error():
    return lib().pf_last_error().decode()


# --------------------------------------------------------------------------
# torch convenience wrapper
# --------------------------------------------------------------------------
def make_mesh(dim, degree, n_cells, extent, domain, n_levels, faces) -> Mesh:
    m = Mesh()
    m.dim, m.degree = dim, degree
    nc = list(n_cells) + [1] * (3 - len(n_cells))
    ex = list(extent) + [1.0] * (3 - len(extent))
    for k in range(3):
        m.n_cells[k] = int(nc[k])
        m.extent[k] = float(ex[k])
    m.domain, m.n_levels, m.dirichlet_faces = int(domain), int(n_levels), int(faces)
    return m


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


class Solver:
    """Owns a context and its torch-allocated device workspace."""

    def __init__(self, mesh: Mesh, material: dict, opt: Options = None, device="cuda"):
        import torch
        self.torch = torch
        self.mesh = mesh
        self.opt = Options.from_buffer_copy(opt) if opt is not None else pf_default_options()
        if "split" in material:   # the model's energy split comes with the material
            self.opt.stress_split = {"none": PF_SPLIT_NONE, "miehe": PF_SPLIT_MIEHE}[material["split"]]
        self.ws_bytes = pf_workspace_size(mesh, self.opt)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        aligned = (base + 255) & ~255
        m = material
        self.ctx = pf_setup(mesh, m["E"], m["nu"], m["G_c"], m["eps"], m["kappa"], m["pressure"], self.opt,
                            aligned, self.ws_bytes, _stream())
        self.device = device
        self.levels = [pf_get_level_info(self.ctx, l) for l in range(mesh.n_levels)]

    def close(self):
        if self.ctx:
            pf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # helpers -------------------------------------------------------------
    def n_dofs(self, level=-1):
        return self.levels[level].n_dofs

    def n_nodes(self, level=-1):
        return self.levels[level].n_nodes

    def set_constraints(self, bits):
        pf_set_constraints(self.ctx, _ptr(bits), _stream())

    def set_linearization(self, U, phit, active=None):
        pf_set_linearization(self.ctx, _ptr(U), _ptr(phit), _ptr(active), _stream())

    def _empty(self, n, dtype):
        return self.torch.empty(n, dtype=dtype, device=self.device)

    def jacobian_apply(self, level, x, out=None):
        prec = PF_F64 if x.dtype == self.torch.float64 else PF_F32
        y = out if out is not None else self._empty(x.numel(), x.dtype)
        pf_jacobian_apply(self.ctx, level % len(self.levels), prec, x.data_ptr(), y.data_ptr(), _stream())
        return y

    def block_apply(self, level, x, out=None):
        prec = PF_F64 if x.dtype == self.torch.float64 else PF_F32
        y = out if out is not None else self._empty(x.numel(), x.dtype)
        pf_block_apply(self.ctx, level % len(self.levels), prec, x.data_ptr(), y.data_ptr(), _stream())
        return y

    def residual(self, U, phit):
        R = self._empty(U.numel(), self.torch.float64)
        pf_residual(self.ctx, U.data_ptr(), phit.data_ptr(), R.data_ptr(), _stream())
        return R

    def diagonal(self, level):
        lv = level % len(self.levels)
        out = self._empty(self.levels[lv].n_dofs, self.torch.float64)
        pf_get_diagonal(self.ctx, lv, out.data_ptr(), _stream())
        return out

    def lumped_mass(self):
        out = self._empty(self.n_nodes(), self.torch.float64)
        pf_get_lumped_mass(self.ctx, out.data_ptr(), _stream())
        return out

    def level_data(self, level):
        lv = level % len(self.levels)
        info = self.levels[lv]
        U = self._empty(info.n_dofs, self.torch.float64)
        pt = self._empty(info.n_nodes, self.torch.float64)
        mk = self._empty(info.n_nodes, self.torch.uint8)
        pf_get_level_data(self.ctx, lv, U.data_ptr(), pt.data_ptr(), mk.data_ptr(), _stream())
        return U, pt, mk

    def active_set(self, R, U, Uold):
        act = self._empty(self.n_nodes(), self.torch.uint8)
        v = self._empty(self.n_nodes(), self.torch.float64)
        n = pf_active_set(self.ctx, R.data_ptr(), U.data_ptr(), Uold.data_ptr(), act.data_ptr(), v.data_ptr(),
                          True, _stream())
        return act, v, n

    def transfer(self, level, op, x):
        lv = level % len(self.levels)
        n_out = self.levels[lv - 1].n_dofs if op in (0, 2) else self.levels[lv].n_dofs
        out = self._empty(n_out, self.torch.float64)
        pf_transfer(self.ctx, lv, op, x.data_ptr(), out.data_ptr(), _stream())
        return out

    def eig_bounds(self, level):
        return pf_get_eig_bounds(self.ctx, level % len(self.levels))

    def set_eig_bounds(self, level, bounds):
        pf_set_eig_bounds(self.ctx, level % len(self.levels), bounds)

    def vcycle(self, r, prec=PF_F64):
        z = self._empty(r.numel(), self.torch.float64)
        pf_vcycle(self.ctx, prec, r.data_ptr(), z.data_ptr(), _stream())
        return z

    def newton_step(self, U, Uold, phit, raise_on_error=True):
        st, rep = pf_newton_step(self.ctx, U.data_ptr(), Uold.data_ptr(), phit.data_ptr(), _stream(),
                                 raise_on_error)
        return st, rep

    def pdas_solve(self, U, Uold, phit, max_iter=50, tol_as=1e-10, raise_on_error=True):
        """Algorithm 1 repeated until the active set settles and ||R~|| <= tol_as (U updated in place)."""
        return pf_pdas_solve(self.ctx, U.data_ptr(), Uold.data_ptr(), phit.data_ptr(), max_iter, tol_as,
                             _stream(), raise_on_error)

    def extrapolate(self, phi_1, phi_2, theta=1.0):
        """phi~ = phi_1 + theta (phi_1 - phi_2) on the finest level's nodes (a new tensor)."""
        out = self._empty(phi_1.numel(), self.torch.float64)
        pf_extrapolate(self.ctx, phi_1.data_ptr(), phi_2.data_ptr(), theta, out.data_ptr(), _stream())
        return out

    def set_pressure(self, pressure):
        pf_set_pressure(self.ctx, pressure)

    def energies(self, U):
        """(crack energy, bulk energy) of the state U (finest level, FP64)."""
        out = (D * 2)()
        _check(lib().pf_energies(self.ctx, U.data_ptr(), out, _stream()), "pf_energies")
        return out[0], out[1]

    def energies_noalloc(self, U, out):
        """pf_energies_noalloc: (crack energy, bulk energy) into the device tensor out (2 FP64),
        asynchronous on the current stream, with the library's static scratch (no allocation)."""
        assert out.dtype == self.torch.float64 and out.numel() >= 2 and out.is_cuda
        _check(lib().pf_energies_noalloc(self.ctx, U.data_ptr(), out.data_ptr(), _stream()), "pf_energies_noalloc")
        return out

    def boundary_traction(self, U, face):
        """int over box face `face` (2k: x_k = 0, 2k+1: x_k = extent_k) of g(phi) sigma(u) n."""
        out = (D * 3)()
        _check(lib().pf_boundary_traction(self.ctx, U.data_ptr(), face, out, _stream()), "pf_boundary_traction")
        nn = self.n_nodes()
        d = U.numel() // nn - 1
        return [out[i] for i in range(d)]

    def time_step(self, U_1, U_2, pressure, theta=1.0, first=False, max_iter=50, tol_as=1e-10):
        """One loading step: U^n from U^{n-1} (U_1) and U^{n-2} (U_2) at pressure p(t_n).

        phi~ is the linear extrapolation of the two previous phase fields (phi^{n-1} at the first
        step), phi^old = phi^{n-1}, and the PDAS loop starts from U^{n-1}.  Returns (U^n, report)."""
        nn = self.n_nodes()
        d = U_1.numel() // nn - 1
        phi_1, phi_2 = U_1[d * nn:], U_2[d * nn:]
        phit = phi_1.clone() if first else self.extrapolate(phi_1, phi_2, theta)
        self.set_pressure(pressure)
        U = U_1.clone()
        st, rep = self.pdas_solve(U, U_1, phit, max_iter, tol_as)
        return U, rep

    def set_vcycle_precision(self, prec):
        pf_set_vcycle_precision(self.ctx, prec)

    def set_graphs(self, enable):
        _check(lib().pf_set_graphs(self.ctx, 1 if enable else 0), "pf_set_graphs")

    def graph_captures(self):
        """V-cycle captures made by this context so far (pf_get_graph_captures)."""
        n = C.c_int64(0)
        _check(lib().pf_get_graph_captures(self.ctx, C.byref(n)), "pf_get_graph_captures")
        return n.value

    def set_coarse_mode(self, mode):
        """PF_COARSE_AUTO (dense matrix of the coarse solve when small), PF_COARSE_FUSED or PF_COARSE_STEPS."""
        _check(lib().pf_set_coarse_mode(self.ctx, mode), "pf_set_coarse_mode")

    def set_smoother_fusion(self, mode):
        """PF_FUSE_OFF, PF_FUSE_TUNED (default) or PF_FUSE_ALWAYS: Chebyshev steps fused into
        marching-tile block-operator applies (see pff.h)."""
        _check(lib().pf_set_smoother_fusion(self.ctx, int(mode)), "pf_set_smoother_fusion")

    def set_kernel_timing(self, enable, every=1):
        """Bracket the finest-level FP64 cell kernels with HIP events (see pff.h): True or
        PF_KTIME_JACOBIAN for G~, PF_KTIME_BLOCK for B~, or both OR-ed; False stops.
        every > 1 brackets every every-th launch of each record."""
        mask = PF_KTIME_JACOBIAN if enable is True else int(enable)
        _check(lib().pf_set_kernel_timing(self.ctx, mask, every), "pf_set_kernel_timing")

    def kernel_timing(self, op=PF_KTIME_JACOBIAN, launches=False):
        """(count, mean_s, min_s, max_s) of the bracketed launches of one record since timing
        was enabled; with launches=True, (launches seen, count, mean_s, min_s, max_s)."""
        seen, n, a, lo, hi = C.c_int64(0), I(0), D(0), D(0), D(0)
        _check(lib().pf_get_kernel_timing_op(self.ctx, op, C.byref(seen), C.byref(n), C.byref(a), C.byref(lo),
                                             C.byref(hi)), "pf_get_kernel_timing_op")
        r = (n.value, a.value, lo.value, hi.value)
        return (seen.value,) + r if launches else r

    # autotuner ---------------------------------------------------------------
    def tuning_key(self):
        m = self.mesh
        arch = self.torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        return (f"{arch}|d{m.dim}p{m.degree}|{m.n_cells[0]}x{m.n_cells[1]}x{m.n_cells[2]}|dom{m.domain}"
                f"|L{m.n_levels}|split{self.opt.stress_split}")

    def autotune(self, reps=20, cache_path=None):
        """Pick the fastest Q1 cell-loop shape per level (needs a linearization point).

        With cache_path, choices are read from / written to a JSON file keyed by
        GPU architecture and mesh shape.  Returns the tuning report.
        """
        key = self.tuning_key()
        cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        if key in cache:
            for ch in cache[key]:
                pf_set_tuning(self.ctx, ch["level"], ch["prec"], ch["mode"], ch["variant"], ch["zc"])
                if ch["mode"] == 1:
                    _check(lib().pf_set_level_fusion(self.ctx, ch["level"], ch["prec"], int(ch.get("fused", 0))),
                           "pf_set_level_fusion")
            return pf_tuning_report(self.ctx)
        pf_autotune(self.ctx, reps, _stream())
        rep = pf_tuning_report(self.ctx)
        if cache_path:
            choices = []
            for lv in rep["levels"]:
                for ch in lv["choices"]:
                    choices.append(dict(level=lv["level"], prec=PF_F64 if ch["prec"] == "f64" else PF_F32,
                                        mode=0 if ch["mode"] == "jacobian" else 1, variant=ch["variant"],
                                        zc=ch["zc"], fused=ch.get("fused", 0)))
            cache[key] = choices
            os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1)
        return rep


def solver_from_spec(s, device="cuda", **opt_overrides):
    """Build a Solver for a workload dict from the workloads module."""
    mesh = make_mesh(s["dim"], s["degree"], s["n_cells"], s["extent"], s["domain"], s["n_levels"], s["faces"])
    opt = pf_default_options()
    opt.vcycle_precision = PF_F32 if s.get("vcycle") == "f32" else PF_F64
    for k, v in opt_overrides.items():
        setattr(opt, k, v)
    return Solver(mesh, s["material"], opt, device)


# candidates of pf_batch_autotune, in its order: (shape, zc)
BATCH_CANDIDATES = [(-1, 0), (2, 0), (0, 4), (0, 8), (0, 16), (0, 32), (1, 4), (1, 8), (1, 16)]


class BatchSolver:
    """A batch context (pf_batch_*) with its torch-allocated workspace and packed-layout helpers."""

    def __init__(self, specs, opt: Options = None, device="cuda"):
        import torch
        self.torch = torch
        self.specs = list(specs)
        n = len(self.specs)
        self.n = n
        self.meshes = (Mesh * n)(*[make_mesh(s["dim"], s["degree"], s["n_cells"], s["extent"], s["domain"],
                                             s["n_levels"], s["faces"]) for s in self.specs])
        mats = []
        for s in self.specs:
            m = s["material"]
            mats += [m["E"], m["nu"], m["G_c"], m["eps"], m["kappa"], m["pressure"]]
        self.mats = (D * (6 * n))(*mats)
        self.opt = Options.from_buffer_copy(opt) if opt is not None else pf_default_options()
        splits = {s["material"].get("split", "none") for s in self.specs}
        if len(splits) > 1:
            raise ValueError("the instances of a batch share one energy split")
        if "split" in self.specs[0]["material"]:
            self.opt.stress_split = {"none": PF_SPLIT_NONE, "miehe": PF_SPLIT_MIEHE}[splits.pop()]
        nb = C.c_size_t(0)
        _check(lib().pf_batch_workspace_size(self.meshes, n, C.byref(self.opt), C.byref(nb)),
               "pf_batch_workspace_size")
        self.ws_bytes = nb.value
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        aligned = (self.ws.data_ptr() + 255) & ~255
        out = VP()
        _check(lib().pf_batch_setup(self.meshes, self.mats, n, C.byref(self.opt), aligned, self.ws_bytes,
                                    _stream(), C.byref(out)), "pf_batch_setup")
        self.b = out.value
        self.device = device
        self.L = self.specs[0]["n_levels"]
        self.dof_off, self.node_off = [], []
        for l in range(self.L):
            do, no = (I64 * (n + 1))(), (I64 * (n + 1))()
            _check(lib().pf_batch_layout(self.b, l, do, no), "pf_batch_layout")
            self.dof_off.append(list(do))
            self.node_off.append(list(no))

    def close(self):
        if self.b:
            lib().pf_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # packing -----------------------------------------------------------------
    def pack(self, arrays, level=-1, nodes=False):
        """Concatenate per-instance numpy arrays into one device tensor in the packed layout."""
        import numpy as np
        off = (self.node_off if nodes else self.dof_off)[level]
        for b, a in enumerate(arrays):
            assert a.size == off[b + 1] - off[b], (b, a.size, off[b + 1] - off[b])
        return self.torch.from_numpy(np.ascontiguousarray(np.concatenate(arrays))).to(self.device)

    def unpack(self, t, level=-1, nodes=False):
        off = (self.node_off if nodes else self.dof_off)[level]
        h = t.detach().cpu().numpy()
        return [h[off[b]:off[b + 1]] for b in range(self.n)]

    # calls -------------------------------------------------------------------
    def set_constraints(self, bits):
        _check(lib().pf_batch_set_constraints(self.b, _ptr(bits), _stream()), "pf_batch_set_constraints")

    def set_linearization(self, U, phit, active=None):
        _check(lib().pf_batch_set_linearization(self.b, _ptr(U), _ptr(phit), _ptr(active), _stream()),
               "pf_batch_set_linearization")

    def jacobian_apply(self, level, x):
        prec = PF_F64 if x.dtype == self.torch.float64 else PF_F32
        y = self.torch.empty_like(x)
        _check(lib().pf_batch_jacobian_apply(self.b, level % self.L, prec, x.data_ptr(), y.data_ptr(), _stream()),
               "pf_batch_jacobian_apply")
        return y

    def vcycle(self, r, prec=PF_F64):
        z = self.torch.empty_like(r)
        _check(lib().pf_batch_vcycle(self.b, prec, r.data_ptr(), z.data_ptr(), _stream()), "pf_batch_vcycle")
        return z

    def eig_bounds(self, level, inst):
        out = (D * 4)()
        _check(lib().pf_batch_get_eig_bounds(self.b, level % self.L, inst, out), "pf_batch_get_eig_bounds")
        return list(out)

    def set_eig_bounds(self, level, inst, bounds):
        arr = None if bounds is None else (D * 4)(*[float(v) for v in bounds])
        _check(lib().pf_batch_set_eig_bounds(self.b, level % self.L, inst, arr), "pf_batch_set_eig_bounds")

    def set_vcycle_precision(self, prec):
        _check(lib().pf_batch_set_vcycle_precision(self.b, prec), "pf_batch_set_vcycle_precision")

    def set_graphs(self, enable):
        _check(lib().pf_batch_set_graphs(self.b, 1 if enable else 0), "pf_batch_set_graphs")

    def autotune(self, reps=10):
        """pf_batch_autotune; returns the choices per level: {"level", "choices": [{prec, mode,
        shape, zc, us}]} with the candidates' times in the order of BATCH_CANDIDATES."""
        _check(lib().pf_batch_autotune(self.b, reps, _stream()), "pf_batch_autotune")
        return self.tuning()

    def tuning(self):
        out = []
        for l in range(self.L):
            ch = []
            for prec, pn in ((PF_F64, "f64"), (PF_F32, "f32")):
                for mode, mn in ((0, "jacobian"), (1, "block")):
                    sh, zc, us = I(0), I(0), (D * len(BATCH_CANDIDATES))()
                    _check(lib().pf_batch_get_tuning(self.b, l, prec, mode, C.byref(sh), C.byref(zc), us),
                           "pf_batch_get_tuning")
                    ch.append({"prec": pn, "mode": mn, "shape": sh.value, "zc": zc.value, "us": list(us)})
            out.append({"level": l, "choices": ch})
        return out

    def set_tuning(self, level, prec, mode, shape, zc):
        _check(lib().pf_batch_set_tuning(self.b, level % self.L, prec, mode, shape, zc), "pf_batch_set_tuning")

    def newton_step(self, U, Uold, phit, raise_on_error=True):
        reps = (NewtonReport * self.n)()
        st = lib().pf_batch_newton_step(self.b, U.data_ptr(), Uold.data_ptr(), phit.data_ptr(), reps, _stream())
        if raise_on_error:
            _check(st, "pf_batch_newton_step")
        return st, [r.as_dict() for r in reps]
