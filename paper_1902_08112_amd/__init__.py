"""MI355X (gfx950) matrix-free phase-field fracture Newton/GMG library.

The compute path is the HIP library libpff.so (C ABI in include/pff.h); this
package holds its sources (csrc/), the in-tree build script (build.py) and the
ctypes binding (pff.py).
"""
from . import pff  # noqa: F401
from .pff import PF_F32, PF_F64, PffError, Solver, solver_from_spec  # noqa: F401
