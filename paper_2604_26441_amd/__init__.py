"""MI355X-native matrix-free Galerkin multigrid PCG for 3D hex8 SIMP elasticity.

The solver lives in the HIP library built from csrc/ (C ABI in
include/simpgmg.h); ``simpgmg`` is its ctypes binding.
"""
from .simpgmg import (  # noqa: F401
    F64, F32, BF16, BF16X3, Options, Hierarchy, SimpGmgError, default_options, setup_hierarchy,
    update_moduli, apply_K, vcycle, pcg_solve, library_path, EXPORTS,
)
