"""MI355X-native matrix-free Galerkin multigrid PCG for 3D hex8 SIMP elasticity.

The solver lives in the HIP library built from csrc/ (C ABI in
include/simpgmg.h); ``paper_2604_26441_amd.simpgmg`` is its ctypes binding.
The binding is imported on first attribute access, so ``build`` runs without
a built library.
"""
import importlib

_BINDING = {"F64", "F32", "BF16", "BF16X3", "BF16X2", "Options", "Hierarchy", "SimpGmgError",
            "default_options", "setup_hierarchy", "update_moduli", "apply_K", "vcycle",
            "pcg_solve", "fgmres_solve", "lanczos", "autotune", "library_path", "EXPORTS", "Batch", "setup_batch",
            "pcg_solve_batch", "pcg_solve_batch_concurrent", "UNet", "unet_input", "unet_output", "unet_target",
            "warm_start_scale", "padded_grid", "set_launch_shape", "Simp", "simp_params"}


def __getattr__(name):
    if name in _BINDING:
        return getattr(importlib.import_module(".simpgmg", __name__), name)
    raise AttributeError(name)
