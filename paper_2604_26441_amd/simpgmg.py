"""ctypes binding of libsimpgmg (include/simpgmg.h).

Argument marshalling only: tensors are passed as device pointers together
with the current HIP stream of torch; every step of the solver runs in the
library's HIP kernels.  Importing this module raises if the built library is
missing; there is no fallback.
"""
import ctypes
import os

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libsimpgmg.so")

F64, F32, BF16, BF16X3, BF16X2 = 0, 1, 2, 3, 4
PRECISIONS = {"f64": F64, "f32": F32, "bf16": BF16, "bf16x3": BF16X3, "bf16x2": BF16X2}
STATUS = {0: "converged", 1: "maxit", 2: "stagnated", 3: "nonfinite", 4: "breakdown"}
PRECOND_NONE, PRECOND_JACOBI, PRECOND_VCYCLE = 0, 1, 2


class Options(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("nu", ctypes.c_double), ("E0", ctypes.c_double), ("Emin", ctypes.c_double),
        ("penal", ctypes.c_double),
        ("input_is_modulus", ctypes.c_int),
        ("n_levels", ctypes.c_int),
        ("fine_smoother", ctypes.c_int),
        ("fine_degree", ctypes.c_int),
        ("coarse_sweeps", ctypes.c_int),
        ("cheb_alpha", ctypes.c_double),
        ("jacobi_omega_max", ctypes.c_double),
        ("lambda_safety", ctypes.c_double),
        ("power_iters_fine", ctypes.c_int),
        ("power_iters_coarse", ctypes.c_int),
        ("fine_prec", ctypes.c_int),
        ("level1_prec", ctypes.c_int),
        ("dense_max", ctypes.c_int),
        ("coarse_pcg_iters", ctypes.c_int),
        ("seed", ctypes.c_uint64),
        ("flexible_beta", ctypes.c_int),
        ("stag_window", ctypes.c_int),
        ("lambda_override", ctypes.POINTER(ctypes.c_double)),
        ("use_graphs", ctypes.c_int),
        ("cycle_gamma", ctypes.c_int),
        ("stencil_form", ctypes.c_int),
        ("bf16_guard", ctypes.c_int),
        ("guard_window", ctypes.c_int),
        ("guard_drop", ctypes.c_double),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("iters", ctypes.c_int),
        ("rel_res_true", ctypes.c_double), ("rel_res_recur", ctypes.c_double),
        ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int),
        ("solve_ms", ctypes.c_double),
        ("fallback_iter", ctypes.c_int),
    ]


class SimpParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("penal", ctypes.c_double), ("E0", ctypes.c_double), ("Emin", ctypes.c_double),
        ("volfrac", ctypes.c_double), ("move", ctypes.c_double), ("rmin", ctypes.c_double),
        ("beta", ctypes.c_double), ("eta", ctypes.c_double), ("oc_tol", ctypes.c_double),
        ("oc_max_halvings", ctypes.c_int),
    ]


class SimpInfo(ctypes.Structure):
    _fields_ = [
        ("compliance", ctypes.c_double), ("volume", ctypes.c_double), ("lambda_", ctypes.c_double),
        ("max_change", ctypes.c_double), ("pcg_status", ctypes.c_int), ("pcg_iters", ctypes.c_int),
        ("rel_res_true", ctypes.c_double), ("solve_ms", ctypes.c_double),
    ]


EXPORTS = [
    "sgmg_default_options", "sgmg_setup_hierarchy", "sgmg_update_moduli", "sgmg_apply_K",
    "sgmg_vcycle", "sgmg_pcg_solve", "sgmg_fgmres_solve", "sgmg_lanczos", "sgmg_num_levels", "sgmg_level_info",
    "sgmg_copy_stencil", "sgmg_copy_diagonal", "sgmg_destroy", "sgmg_last_error",
    "sgmg_autotune", "sgmg_set_launch_shape", "sgmg_setup_batch", "sgmg_pcg_solve_batch",
    "sgmg_pcg_solve_batch_staged", "sgmg_pcg_solve_batch_graph",
    "sgmg_pcg_solve_batch_concurrent", "sgmg_batch_hierarchy",
    "sgmg_batch_block_size", "sgmg_batch_destroy", "sgmg_batch_item_layout",
    "sgmg_unet_create", "sgmg_unet_num_params", "sgmg_unet_set_params", "sgmg_unet_get_params",
    "sgmg_unet_forward", "sgmg_unet_grad", "sgmg_unet_train_step", "sgmg_unet_energy_step",
    "sgmg_unet_input",
    "sgmg_unet_output", "sgmg_unet_target", "sgmg_warm_start_scale",
    "sgmg_warm_start_scale_noalloc", "sgmg_unet_destroy",
    "sgmg_simp_default_params", "sgmg_simp_create", "sgmg_simp_destroy", "sgmg_simp_physical",
    "sgmg_simp_sensitivity", "sgmg_simp_oc_update", "sgmg_simp_step",
]


def _load():
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"libsimpgmg.so not built ({_LIB_PATH}); run __graft_entry__.build()")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    H = ctypes.c_void_p
    lib.sgmg_default_options.argtypes = [ctypes.POINTER(Options), i, i, i]
    lib.sgmg_default_options.restype = None
    lib.sgmg_setup_hierarchy.argtypes = [ctypes.POINTER(Options), vp, vp, vp, ctypes.POINTER(H)]
    lib.sgmg_update_moduli.argtypes = [H, vp, vp]
    lib.sgmg_apply_K.argtypes = [H, i, i, vp, vp, vp]
    lib.sgmg_vcycle.argtypes = [H, vp, vp, vp]
    lib.sgmg_pcg_solve.argtypes = [H, i, vp, vp, d, i, ctypes.POINTER(SolveInfo), vp]
    lib.sgmg_fgmres_solve.argtypes = [H, i, i, vp, vp, d, i, ctypes.POINTER(SolveInfo), vp]
    dp = ctypes.POINTER(ctypes.c_double)
    lib.sgmg_lanczos.argtypes = [H, i, i, vp, d, dp, dp, ctypes.POINTER(ctypes.c_int), dp, vp]
    lib.sgmg_autotune.argtypes = [H, ctypes.POINTER(ctypes.c_int), vp]
    lib.sgmg_set_launch_shape.argtypes = [H, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.sgmg_setup_batch.argtypes = [i, ctypes.POINTER(Options), ctypes.POINTER(vp),
                                     ctypes.POINTER(vp), vp, ctypes.POINTER(H)]
    lib.sgmg_pcg_solve_batch.argtypes = [H, i, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(vp),
                                         ctypes.POINTER(vp), d, i, ctypes.POINTER(SolveInfo),
                                         ctypes.POINTER(ctypes.c_double), vp]
    lib.sgmg_pcg_solve_batch_staged.argtypes = [H, i, ctypes.POINTER(ctypes.c_int),
                                                ctypes.POINTER(vp), ctypes.POINTER(vp), d, i,
                                                ctypes.POINTER(SolveInfo),
                                                ctypes.POINTER(ctypes.c_double), vp]
    lib.sgmg_pcg_solve_batch_graph.argtypes = [H, i, ctypes.POINTER(ctypes.c_int),
                                               ctypes.POINTER(vp), ctypes.POINTER(vp), d, i, i,
                                               ctypes.POINTER(SolveInfo),
                                               ctypes.POINTER(ctypes.c_int),
                                               ctypes.POINTER(ctypes.c_double), vp]
    lib.sgmg_pcg_solve_batch_concurrent.argtypes = [H, i, ctypes.POINTER(ctypes.c_int),
                                                    ctypes.POINTER(vp), ctypes.POINTER(vp), d, i, i,
                                                    ctypes.POINTER(SolveInfo),
                                                    ctypes.POINTER(ctypes.c_double), vp]
    lib.sgmg_batch_hierarchy.argtypes = [H, i]
    lib.sgmg_batch_hierarchy.restype = ctypes.c_void_p
    lib.sgmg_batch_block_size.argtypes = [H]
    lib.sgmg_batch_destroy.argtypes = [H]
    lib.sgmg_batch_destroy.restype = None
    sz = ctypes.POINTER(ctypes.c_size_t)
    lib.sgmg_batch_item_layout.argtypes = [i, ctypes.POINTER(ctypes.c_int), i, sz, sz]
    lib.sgmg_batch_item_layout.restype = ctypes.c_size_t
    fp = ctypes.POINTER(ctypes.c_float)
    lib.sgmg_unet_create.argtypes = [ctypes.c_uint64, ctypes.POINTER(H)]
    lib.sgmg_unet_num_params.argtypes = []
    lib.sgmg_unet_set_params.argtypes = [H, fp, vp]
    lib.sgmg_unet_get_params.argtypes = [H, i, fp, vp]
    lib.sgmg_unet_forward.argtypes = [H, i, i, i, i, vp, vp, vp]
    lib.sgmg_unet_grad.argtypes = [H, i, i, i, i, vp, vp, vp, fp, fp, vp]
    lib.sgmg_unet_train_step.argtypes = [H, i, i, i, i, vp, vp, vp, ctypes.c_float, fp, vp]
    lib.sgmg_unet_energy_step.argtypes = [H, H, i, i, i, i, vp, vp, vp, vp, ctypes.c_float, fp, fp, vp]
    lib.sgmg_unet_input.argtypes = [H, vp, vp, i, i, i, vp, vp]
    lib.sgmg_unet_output.argtypes = [H, vp, i, i, i, vp, vp]
    lib.sgmg_unet_target.argtypes = [H, vp, i, i, i, vp, vp, vp]
    lib.sgmg_warm_start_scale.argtypes = [H, vp, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.sgmg_warm_start_scale_noalloc.argtypes = [H, vp, vp, vp, vp]
    lib.sgmg_unet_destroy.argtypes = [H]
    lib.sgmg_unet_destroy.restype = None
    SP = ctypes.POINTER(SimpParams)
    lib.sgmg_simp_default_params.argtypes = [SP, i, i, i]
    lib.sgmg_simp_default_params.restype = None
    lib.sgmg_simp_create.argtypes = [SP, vp, ctypes.POINTER(H)]
    lib.sgmg_simp_destroy.argtypes = [H]
    lib.sgmg_simp_destroy.restype = None
    lib.sgmg_simp_physical.argtypes = [H, vp, vp, vp]
    lib.sgmg_simp_sensitivity.argtypes = [H, H, vp, dp, vp, vp, vp]
    lib.sgmg_simp_oc_update.argtypes = [H, vp, dp, dp, dp, vp]
    lib.sgmg_simp_step.argtypes = [H, H, i, vp, vp, vp, d, i, ctypes.POINTER(SimpInfo), vp]
    lib.sgmg_num_levels.argtypes = [H]
    lib.sgmg_level_info.argtypes = [H, i, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_double)]
    lib.sgmg_copy_stencil.argtypes = [H, i, ctypes.POINTER(ctypes.c_double)]
    lib.sgmg_copy_diagonal.argtypes = [H, i, ctypes.POINTER(ctypes.c_double)]
    lib.sgmg_destroy.argtypes = [H]
    lib.sgmg_destroy.restype = None
    lib.sgmg_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        getattr(lib, name)
    return lib


_lib = _load()


def library_path():
    return _LIB_PATH


class SimpGmgError(RuntimeError):
    pass


def _check(rc):
    if rc != 0:
        raise SimpGmgError(f"libsimpgmg error {rc}: {_lib.sgmg_last_error().decode()}")


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t, dtype, numel=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def default_options(nx, ny, nz, **kw):
    o = Options()
    _lib.sgmg_default_options(ctypes.byref(o), nx, ny, nz)
    for k, v in kw.items():
        if k in ("fine_prec", "level1_prec") and isinstance(v, str):
            v = PRECISIONS[v]
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def n_nodes(o):
    return (o.nx + 1) * (o.ny + 1) * (o.nz + 1)


class Hierarchy:
    """Owns an sgmg_hierarchy handle (or borrows one from a batch)."""

    def __init__(self, handle, opts, owner=None):
        self._h = handle
        self.opts = opts
        self.n_dof = 3 * n_nodes(opts)
        self._owner = owner            # a Batch keeps borrowed handles alive

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h and self._owner is None:
            _lib.sgmg_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def num_levels(self):
        return _lib.sgmg_num_levels(self._h)

    def level_info(self, level):
        dims = (ctypes.c_int * 3)()
        nf = ctypes.c_int()
        lam = ctypes.c_double()
        _check(_lib.sgmg_level_info(self._h, level, dims, ctypes.byref(nf), ctypes.byref(lam)))
        return {"dims": tuple(dims), "n_free": nf.value, "lambda": lam.value}

    def stencil(self, level):
        import numpy as np
        dims = self.level_info(level)["dims"]
        nn = (dims[0] + 1) * (dims[1] + 1) * (dims[2] + 1)
        out = np.zeros(243 * nn)
        _check(_lib.sgmg_copy_stencil(self._h, level, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out.reshape(27, 3, 3, nn)

    def diagonal(self, level):
        import numpy as np
        dims = self.level_info(level)["dims"]
        nn = (dims[0] + 1) * (dims[1] + 1) * (dims[2] + 1)
        out = np.zeros(3 * nn)
        _check(_lib.sgmg_copy_diagonal(self._h, level, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out


def setup_hierarchy(opts, rho_or_E, fixed_dof=None, lambda_override=None, stream=None):
    nel = opts.nx * opts.ny * opts.nz
    p_rho = _ptr(rho_or_E, torch.float64, nel, "rho_or_E")
    p_fix = None
    if fixed_dof is not None:
        p_fix = _ptr(fixed_dof, torch.uint8, 3 * n_nodes(opts), "fixed_dof")
    keep = None
    if lambda_override is not None:
        keep = (ctypes.c_double * len(lambda_override))(*lambda_override)
        opts.lambda_override = ctypes.cast(keep, ctypes.POINTER(ctypes.c_double))
    h = ctypes.c_void_p()
    try:
        _check(_lib.sgmg_setup_hierarchy(ctypes.byref(opts), p_rho, p_fix, _stream(stream), ctypes.byref(h)))
    finally:
        opts.lambda_override = None
    return Hierarchy(h, opts)


def autotune(h, stream=None):
    """Tune the fine operators' launch shapes for this mesh; returns
    ((rows, planes) for bf16, for bf16x3, for f64); the f64 entry may also be
    (0, 0) (node kernel) or (1, planes) (sum-factorised tiles)."""
    z = (ctypes.c_int * 6)()
    _check(_lib.sgmg_autotune(h.handle, z, _stream(stream)))
    return tuple((int(z[2 * q]), int(z[2 * q + 1])) for q in range(3))


VARIANTS = {"bf16": 0, "bf16x3": 1, "f64": 2, "level1": 3}


def set_launch_shape(h, variant, rows, planes):
    """Pin the fine operator's launch shape for variant 'bf16', 'bf16x3' or
    'f64' ((0, 0) selects the FP64 vector-ALU node kernel, (1, planes) the
    FP64 vector-ALU sum-factorised tile kernel); 'level1' chooses between the
    stored stencil (0, 0) and the element products (1, planes)."""
    _check(_lib.sgmg_set_launch_shape(h.handle, VARIANTS[variant], rows, planes))


def update_moduli(h, rho_or_E, stream=None):
    nel = h.opts.nx * h.opts.ny * h.opts.nz
    _check(_lib.sgmg_update_moduli(h.handle, _ptr(rho_or_E, torch.float64, nel, "rho_or_E"), _stream(stream)))


def apply_K(h, level, prec, u, y, stream=None):
    if isinstance(prec, str):
        prec = PRECISIONS[prec]
    dt = torch.float64 if prec == F64 else torch.float32
    info = h.level_info(level)
    d = info["dims"]
    n = 3 * (d[0] + 1) * (d[1] + 1) * (d[2] + 1)
    _check(_lib.sgmg_apply_K(h.handle, level, prec, _ptr(u, dt, n, "u"), _ptr(y, dt, n, "y"), _stream(stream)))


def vcycle(h, r, z, stream=None):
    _check(_lib.sgmg_vcycle(h.handle, _ptr(r, torch.float64, h.n_dof, "r"),
                            _ptr(z, torch.float64, h.n_dof, "z"), _stream(stream)))


def pcg_solve(h, f, u, rtol=1e-6, maxit=200, precond=PRECOND_VCYCLE, history_cap=0, stream=None):
    info = SolveInfo()
    hist = None
    if history_cap:
        hist = (ctypes.c_double * history_cap)()
        info.history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
        info.history_cap = history_cap
    _check(_lib.sgmg_pcg_solve(h.handle, precond, _ptr(f, torch.float64, h.n_dof, "f"),
                               _ptr(u, torch.float64, h.n_dof, "u"), rtol, maxit, ctypes.byref(info),
                               _stream(stream)))
    out = {"status": STATUS.get(info.status, info.status), "status_code": info.status,
           "iters": info.iters, "rel_res_true": info.rel_res_true,
           "rel_res_recur": info.rel_res_recur, "solve_ms": info.solve_ms,
           "fallback_iter": info.fallback_iter}
    if hist is not None:
        out["history"] = list(hist)[: info.iters + 1]
    return out


class Batch:
    """Owns an sgmg_batch handle (systems of possibly different meshes)."""

    def __init__(self, handle, opts_list):
        self._b = handle
        self.opts = list(opts_list)

    @property
    def handle(self):
        return self._b

    def close(self):
        if self._b:
            _lib.sgmg_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def hierarchy(self, s):
        h = _lib.sgmg_batch_hierarchy(self._b, s)
        if not h:
            raise SimpGmgError("bad system index")
        return Hierarchy(ctypes.c_void_p(h), self.opts[s], owner=self)

    def block_size(self):
        return _lib.sgmg_batch_block_size(self._b)



def fgmres_solve(h, f, u, rtol=1e-6, maxit=200, restart=32, precond=PRECOND_VCYCLE, history_cap=0,
                 stream=None):
    """Restarted right-preconditioned flexible GMRES (see sgmg_fgmres_solve);
    same return fields as pcg_solve, iters = Arnoldi steps, history = true
    relative residual at each cycle start and the estimate after each step."""
    info = SolveInfo()
    hist = None
    if history_cap:
        hist = (ctypes.c_double * history_cap)()
        info.history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
        info.history_cap = history_cap
    _check(_lib.sgmg_fgmres_solve(h.handle, precond, restart, _ptr(f, torch.float64, h.n_dof, "f"),
                                  _ptr(u, torch.float64, h.n_dof, "u"), rtol, maxit, ctypes.byref(info),
                                  _stream(stream)))
    out = {"status": STATUS.get(info.status, info.status), "status_code": info.status,
           "iters": info.iters, "rel_res_true": info.rel_res_true,
           "rel_res_recur": info.rel_res_recur, "solve_ms": info.solve_ms}
    if hist is not None:
        out["history"] = list(hist)
    return out

def lanczos(h, g, m=50, precond=PRECOND_VCYCLE, breakdown=1e-12, stream=None):
    """Preconditioned Lanczos probe of M K (see sgmg_lanczos): returns
    alpha, beta (lists of the steps taken), steps, theta_min, theta_max and
    kappa = theta_max / theta_min."""
    al = (ctypes.c_double * m)()
    be = (ctypes.c_double * m)()
    ritz = (ctypes.c_double * 2)()
    steps = ctypes.c_int()
    _check(_lib.sgmg_lanczos(h.handle, precond, m, _ptr(g, torch.float64, h.n_dof, "g"), breakdown,
                             al, be, ctypes.byref(steps), ritz, _stream(stream)))
    k = steps.value
    return {"alpha": list(al)[:k], "beta": list(be)[:k], "steps": k, "theta_min": ritz[0],
            "theta_max": ritz[1], "kappa": ritz[1] / ritz[0] if ritz[0] != 0 else float("inf")}


def setup_batch(opts_list, rho_list, fixed_list=None, stream=None):
    n = len(opts_list)
    arr = (Options * n)(*opts_list)
    rho = (ctypes.c_void_p * n)(*[_ptr(r, torch.float64, o.nx * o.ny * o.nz, "rho").value
                                  for r, o in zip(rho_list, opts_list)])
    fix = None
    if fixed_list is not None:
        fix = (ctypes.c_void_p * n)(*[None if m is None else
                                      _ptr(m, torch.uint8, 3 * n_nodes(o), "fixed").value
                                      for m, o in zip(fixed_list, opts_list)])
    b = ctypes.c_void_p()
    _check(_lib.sgmg_setup_batch(n, arr, rho, fix, _stream(stream), ctypes.byref(b)))
    return Batch(b, opts_list)


def pcg_solve_batch(batch, item_sys, f_list, u_list, rtol=1e-6, maxit=200, stream=None,
                    staged=False):
    """Solves every item (system index, f, u); returns (list of dicts, total ms).
    staged: sgmg_pcg_solve_batch_staged (one launch per stage over all items)
    instead of the persistent launch."""
    m = len(item_sys)
    sysarr = (ctypes.c_int * m)(*item_sys)
    fa = (ctypes.c_void_p * m)(*[_ptr(f, torch.float64, 3 * n_nodes(batch.opts[s]), "f").value
                                 for f, s in zip(f_list, item_sys)])
    ua = (ctypes.c_void_p * m)(*[_ptr(u, torch.float64, 3 * n_nodes(batch.opts[s]), "u").value
                                 for u, s in zip(u_list, item_sys)])
    infos = (SolveInfo * m)()
    ms = ctypes.c_double()
    fn = _lib.sgmg_pcg_solve_batch_staged if staged else _lib.sgmg_pcg_solve_batch
    _check(fn(batch.handle, m, sysarr, fa, ua, rtol, maxit, infos, ctypes.byref(ms), _stream(stream)))
    out = [{"status": STATUS.get(i.status, i.status), "iters": i.iters,
            "rel_res_true": i.rel_res_true, "rel_res_recur": i.rel_res_recur} for i in infos]
    return out, ms.value


def pcg_solve_batch_graph(batch, item_sys, f_list, u_list, rtol=1e-6, maxit=200, steps=128,
                          stream=None):
    """The staged solve with device-side iteration control (see
    sgmg_pcg_solve_batch_graph): one graph launch per `steps` iterations;
    returns (list of dicts, total ms, number of launches)."""
    m = len(item_sys)
    sysarr = (ctypes.c_int * m)(*item_sys)
    fa = (ctypes.c_void_p * m)(*[_ptr(f, torch.float64, 3 * n_nodes(batch.opts[s]), "f").value
                                 for f, s in zip(f_list, item_sys)])
    ua = (ctypes.c_void_p * m)(*[_ptr(u, torch.float64, 3 * n_nodes(batch.opts[s]), "u").value
                                 for u, s in zip(u_list, item_sys)])
    infos = (SolveInfo * m)()
    ms = ctypes.c_double()
    nl = ctypes.c_int()
    _check(_lib.sgmg_pcg_solve_batch_graph(batch.handle, m, sysarr, fa, ua, rtol, maxit, steps,
                                           infos, ctypes.byref(nl), ctypes.byref(ms),
                                           _stream(stream)))
    out = [{"status": STATUS.get(i.status, i.status), "iters": i.iters,
            "rel_res_true": i.rel_res_true, "rel_res_recur": i.rel_res_recur} for i in infos]
    return out, ms.value, nl.value


def pcg_solve_batch_concurrent(batch, item_sys, f_list, u_list, rtol=1e-6, maxit=200, workers=4,
                               stream=None):
    """The same items solved by `workers` host threads with a stream each
    (see sgmg_pcg_solve_batch_concurrent); returns (list of dicts, total ms)."""
    m = len(item_sys)
    sysarr = (ctypes.c_int * m)(*item_sys)
    fa = (ctypes.c_void_p * m)(*[_ptr(f, torch.float64, 3 * n_nodes(batch.opts[s]), "f").value
                                 for f, s in zip(f_list, item_sys)])
    ua = (ctypes.c_void_p * m)(*[_ptr(u, torch.float64, 3 * n_nodes(batch.opts[s]), "u").value
                                 for u, s in zip(u_list, item_sys)])
    infos = (SolveInfo * m)()
    ms = ctypes.c_double()
    _check(_lib.sgmg_pcg_solve_batch_concurrent(batch.handle, m, sysarr, fa, ua, rtol, maxit, workers,
                                                infos, ctypes.byref(ms), _stream(stream)))
    out = [{"status": STATUS.get(i.status, i.status), "iters": i.iters,
            "rel_res_true": i.rel_res_true, "rel_res_recur": i.rel_res_recur} for i in infos]
    return out, ms.value


def batch_item_layout(level_dofs, n_coarsest_free):
    """(allocation bytes, [(offset, size)] per sub-buffer) of one batch item's
    work memory for a hierarchy with the given full-DOF level lengths
    (host arithmetic of the library, no device work)."""
    L = len(level_dofs)
    nb = 10 + 4 * (L - 1) + 1
    dofs = (ctypes.c_int * L)(*level_dofs)
    off = (ctypes.c_size_t * nb)()
    size = (ctypes.c_size_t * nb)()
    total = _lib.sgmg_batch_item_layout(L, dofs, n_coarsest_free, off, size)
    if total == 0:
        raise SimpGmgError("bad level sizes")
    return total, list(zip(off, size))


def padded_grid(opts, multiple=8):
    """(Dp, Hp, Wp): node counts (z, y, x) rounded up to a multiple."""
    r = lambda v: (v + multiple - 1) // multiple * multiple
    return r(opts.nz + 1), r(opts.ny + 1), r(opts.nx + 1)


class UNet:
    """Owns an sgmg_unet (the warm-start network)."""

    def __init__(self, seed=0):
        self._u = ctypes.c_void_p()
        _check(_lib.sgmg_unet_create(seed, ctypes.byref(self._u)))

    def close(self):
        if self._u:
            _lib.sgmg_unet_destroy(self._u)
            self._u = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def num_params():
        return _lib.sgmg_unet_num_params()

    def set_params(self, flat, stream=None):
        import numpy as np
        a = np.ascontiguousarray(flat, dtype=np.float32)
        assert a.size == self.num_params()
        _check(_lib.sgmg_unet_set_params(self._u, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                         _stream(stream)))

    def get_params(self, quantized=False, stream=None):
        import numpy as np
        a = np.zeros(self.num_params(), dtype=np.float32)
        _check(_lib.sgmg_unet_get_params(self._u, int(quantized),
                                         a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _stream(stream)))
        return a

    def forward(self, x, stream=None):
        N, C, D, H, W = x.shape
        out = torch.empty((N, 3, D, H, W), dtype=torch.float32, device=x.device)
        _check(_lib.sgmg_unet_forward(self._u, N, D, H, W, _ptr(x, torch.float32, name="in"),
                                      _ptr(out, torch.float32, name="out"), _stream(stream)))
        return out

    def grad(self, x, t, mask=None, stream=None):
        import numpy as np
        N, C, D, H, W = x.shape
        g = np.zeros(self.num_params(), dtype=np.float32)
        loss = ctypes.c_float()
        _check(_lib.sgmg_unet_grad(self._u, N, D, H, W, _ptr(x, torch.float32), _ptr(t, torch.float32),
                                   None if mask is None else _ptr(mask, torch.float32), ctypes.byref(loss),
                                   g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _stream(stream)))
        return loss.value, g

    def train_step(self, x, t, mask=None, lr=1e-3, stream=None):
        N, C, D, H, W = x.shape
        loss = ctypes.c_float()
        _check(_lib.sgmg_unet_train_step(self._u, N, D, H, W, _ptr(x, torch.float32),
                                         _ptr(t, torch.float32),
                                         None if mask is None else _ptr(mask, torch.float32), lr,
                                         ctypes.byref(loss), _stream(stream)))
        return loss.value

    def energy_step(self, h, x, rho_or_E, f, cstar, lr=0.0, grads=False, stream=None):
        """Energy-norm score of the batch (mean over samples) and, with lr > 0,
        one Adam step; with grads=True also returns the gradients."""
        import numpy as np
        N, C, D, H, W = x.shape
        g = np.zeros(self.num_params(), dtype=np.float32) if grads else None
        loss = ctypes.c_float()
        _check(_lib.sgmg_unet_energy_step(
            self._u, h.handle, N, D, H, W, _ptr(x, torch.float32, name="in"),
            _ptr(rho_or_E, torch.float64, name="rho_or_E"), _ptr(f, torch.float64, name="f"),
            _ptr(cstar, torch.float64, name="cstar"), float(lr), ctypes.byref(loss),
            None if g is None else g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _stream(stream)))
        return (loss.value, g) if grads else loss.value


def unet_input(h, rho, f, stream=None):
    Dp, Hp, Wp = padded_grid(h.opts)
    x = torch.empty((1, 5, Dp, Hp, Wp), dtype=torch.float32, device=rho.device)
    _check(_lib.sgmg_unet_input(h.handle, _ptr(rho, torch.float64), _ptr(f, torch.float64), Dp, Hp, Wp,
                                _ptr(x, torch.float32), _stream(stream)))
    return x


def unet_target(h, u, stream=None):
    Dp, Hp, Wp = padded_grid(h.opts)
    t = torch.empty((1, 3, Dp, Hp, Wp), dtype=torch.float32, device=u.device)
    m = torch.empty((1, 1, Dp, Hp, Wp), dtype=torch.float32, device=u.device)
    _check(_lib.sgmg_unet_target(h.handle, _ptr(u, torch.float64), Dp, Hp, Wp, _ptr(t, torch.float32),
                                 _ptr(m, torch.float32), _stream(stream)))
    return t, m


def unet_output(h, y, stream=None):
    Dp, Hp, Wp = padded_grid(h.opts)
    u0 = torch.empty(h.n_dof, dtype=torch.float64, device=y.device)
    _check(_lib.sgmg_unet_output(h.handle, _ptr(y, torch.float32), Dp, Hp, Wp, _ptr(u0, torch.float64),
                                 _stream(stream)))
    return u0


def warm_start_scale(h, f, u0, stream=None):
    a = ctypes.c_double()
    _check(_lib.sgmg_warm_start_scale(h.handle, _ptr(f, torch.float64, h.n_dof), _ptr(u0, torch.float64, h.n_dof),
                                      ctypes.byref(a), _stream(stream)))
    return a.value


def warm_start_scale_noalloc(h, f, u0, alpha=None, stream=None):
    """sgmg_warm_start_scale_noalloc: u0 scaled in place, alpha (a one-element
    FP64 device tensor, optional) written on the stream; nothing allocated."""
    _check(_lib.sgmg_warm_start_scale_noalloc(
        h.handle, _ptr(f, torch.float64, h.n_dof), _ptr(u0, torch.float64, h.n_dof),
        _ptr(alpha, torch.float64, 1) if alpha is not None else None, _stream(stream)))


def simp_params(nx, ny, nz, **kw):
    p = SimpParams()
    _lib.sgmg_simp_default_params(ctypes.byref(p), nx, ny, nz)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


class Simp:
    """SIMP outer-loop state (see sgmg_simp_*): density filter row sums and
    the element work fields."""

    def __init__(self, params, stream=None):
        self.params = params
        self.n_el = params.nx * params.ny * params.nz
        self.handle = ctypes.c_void_p()
        _check(_lib.sgmg_simp_create(ctypes.byref(params), _stream(stream), ctypes.byref(self.handle)))

    def close(self):
        if self.handle:
            _lib.sgmg_simp_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def physical(self, rho, rhohat=None, stream=None):
        _check(_lib.sgmg_simp_physical(self.handle, _ptr(rho, torch.float64, self.n_el, "rho"),
                                       None if rhohat is None else
                                       _ptr(rhohat, torch.float64, self.n_el, "rhohat"),
                                       _stream(stream)))

    def sensitivity(self, h, u, dc=None, dv=None, stream=None):
        c = ctypes.c_double()
        _check(_lib.sgmg_simp_sensitivity(self.handle, h.handle, _ptr(u, torch.float64, h.n_dof, "u"),
                                          ctypes.byref(c),
                                          None if dc is None else _ptr(dc, torch.float64, self.n_el, "dc"),
                                          None if dv is None else _ptr(dv, torch.float64, self.n_el, "dv"),
                                          _stream(stream)))
        return c.value

    def oc_update(self, rho, stream=None):
        lam, vol, chg = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(_lib.sgmg_simp_oc_update(self.handle, _ptr(rho, torch.float64, self.n_el, "rho"),
                                        ctypes.byref(lam), ctypes.byref(vol), ctypes.byref(chg),
                                        _stream(stream)))
        return {"lambda": lam.value, "volume": vol.value, "max_change": chg.value}

    def step(self, h, rho, f, u, rtol=1e-6, maxit=200, precond=PRECOND_VCYCLE, stream=None):
        info = SimpInfo()
        _check(_lib.sgmg_simp_step(self.handle, h.handle, precond,
                                   _ptr(rho, torch.float64, self.n_el, "rho"),
                                   _ptr(f, torch.float64, h.n_dof, "f"), _ptr(u, torch.float64, h.n_dof, "u"),
                                   rtol, maxit, ctypes.byref(info), _stream(stream)))
        return {"compliance": info.compliance, "volume": info.volume, "lambda": info.lambda_,
                "max_change": info.max_change, "pcg_status": STATUS.get(info.pcg_status, info.pcg_status),
                "pcg_iters": info.pcg_iters, "rel_res_true": info.rel_res_true, "solve_ms": info.solve_ms}
