"""ctypes declarations of libddgmres.so (the C ABI in include/ddgmres.h).

The library is the product: every step of the solver and the predictor runs in
its HIP kernels.  There is no fallback; importing this module without the
built library raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddgmres.so")

DD_OK, DD_NOT_CONVERGED, DD_EINVAL, DD_ENOMEM, DD_EHIP, DD_ENONFINITE = 0, 1, -1, -2, -3, -4
DD_C64, DD_C128 = 0, 1
STATUS_NAMES = {0: "DD_OK", 1: "DD_NOT_CONVERGED", -1: "DD_EINVAL", -2: "DD_ENOMEM",
                -3: "DD_EHIP", -4: "DD_ENONFINITE"}


class DDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class dd_pml(C.Structure):
    _fields_ = [("npml_x", C.c_int), ("npml_y", C.c_int), ("grade_m", C.c_int),
                ("ln_R", C.c_double)]


class dd_solver_opts(C.Structure):
    _fields_ = [("inner", C.c_int), ("cgs_passes", C.c_int), ("restart", C.c_int),
                ("kmax", C.c_int), ("elems_per_thread", C.c_int), ("hist_cap", C.c_int),
                ("check_every", C.c_int), ("select_reorth", C.c_int), ("use_graph", C.c_int),
                ("precond", C.c_int), ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("fused", C.c_int)]


class dd_info(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int), ("matvecs", C.c_int),
                ("restarts", C.c_int), ("k_used", C.c_int), ("fallback_plain", C.c_int),
                ("reorth_steps", C.c_int),
                ("rel_res_true", C.c_double), ("rel_res_est", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class dd_kernel_stats(C.Structure):
    _fields_ = [("ms", C.c_double * 4), ("launches", C.c_longlong * 4),
                ("bytes", C.c_double * 4)]


P = C.c_void_p
PP = C.POINTER(C.c_void_p)
I = C.c_int
D = C.c_double

_SIGS = {
    "dd_last_error": (C.c_char_p, []),
    "fdfd_op_create": (I, [C.POINTER(C.c_float), I, I, D, D, C.POINTER(dd_pml), P, PP]),
    "fdfd_op_apply": (I, [P, P, P, I, P]),
    "fdfd_op_dims": (I, [P, C.POINTER(I), C.POINTER(I)]),
    "fdfd_op_destroy": (None, [P]),
    "dd_solver_opts_default": (None, [C.POINTER(dd_solver_opts)]),
    "dd_solver_create": (I, [PP, I, C.POINTER(dd_solver_opts), PP]),
    "dd_solver_workspace_bytes": (I, [PP, I, C.POINTER(dd_solver_opts), C.POINTER(C.c_size_t)]),
    "gmres_workspace_bytes": (C.c_size_t, [P, I, I, I]),
    "dd_solver_bind": (I, [P, PP]),
    "dd_solver_set_subspace": (I, [P, PP, C.POINTER(I), P]),
    "dd_solver_solve": (I, [P, PP, PP, D, I, PP, C.POINTER(dd_info), P]),
    "dd_solver_history": (I, [P, I, C.POINTER(D), I, C.POINTER(I)]),
    "dd_solver_recycle": (I, [P, I, PP, C.POINTER(I), C.POINTER(D), P]),
    "dd_harmonic_ritz_host": (I, [I, I, C.POINTER(D), C.POINTER(D), I, C.POINTER(D), C.POINTER(D)]),
    "dd_solver_debug_copy": (I, [P, I, I, P, C.c_size_t]),
    "dd_solver_device_bytes": (C.c_size_t, [P]),
    "dd_solver_elems_per_thread": (I, [P]),
    "dd_solver_profile": (I, [P, I]),
    "dd_solver_autotune": (I, [PP, I, C.POINTER(dd_solver_opts), C.POINTER(I), C.POINTER(D)]),
    "dd_solver_kernel_stats": (I, [P, C.POINTER(dd_kernel_stats)]),
    "dd_solver_destroy": (None, [P]),
    "gmres_solve": (I, [P, P, P, P, I, D, I, I, C.POINTER(dd_solver_opts), P,
                        C.POINTER(dd_info), P]),
    "gmres_solve_batched": (I, [PP, I, PP, PP, PP, C.POINTER(I), D, I, I,
                                C.POINTER(dd_solver_opts), PP, C.POINTER(dd_info), P]),
    "pca_build": (I, [P, I, I, I, P, C.POINTER(D), P]),
    "proj_loss_batched": (I, [P, P, I, I, I, C.POINTER(D), P]),
    "local_pca_targets": (I, [P, I, I, I, I, P, P]),
    "eim_field": (I, [PP, I, PP, PP, P]),
    "eim_field_noalloc": (I, [PP, I, PP, PP, P]),
    "res_loss_batched": (I, [PP, PP, PP, I, I, C.POINTER(D), P]),
    "res_loss_grad_batched": (I, [PP, PP, PP, I, I, C.POINTER(D), PP, P]),
    "dd_cnn_train_step_res": (I, [P, P, P, PP, PP, I, C.c_float, C.c_float, C.c_float,
                                  C.POINTER(C.c_float), P]),
    "dd_cnn_grad_res": (I, [P, P, P, PP, PP, I, C.POINTER(C.c_float), C.POINTER(C.c_float),
                            C.c_size_t, P]),
    "dd_cnn_create": (I, [I, I, I, I, I, C.c_ulonglong, PP]),
    "dd_cnn_destroy": (None, [P]),
    "dd_cnn_layer_info": (I, [P, I, C.POINTER(I), C.POINTER(I), C.POINTER(I),
                              C.POINTER(I), C.POINTER(I)]),
    "dd_cnn_num_params": (C.c_size_t, [P]),
    "dd_cnn_get_params": (I, [P, C.POINTER(C.c_float), C.c_size_t]),
    "dd_cnn_set_params": (I, [P, C.POINTER(C.c_float), C.c_size_t]),
    "dd_cnn_predict": (I, [P, P, I, P, P]),
    "dd_cnn_predict_eim": (I, [P, P, P, I, P, P]),
    "dd_cnn_dims": (I, [P, C.POINTER(I), C.POINTER(I), C.POINTER(I), C.POINTER(I), C.POINTER(I)]),
    "dd_cnn_save": (I, [P, C.c_char_p]),
    "dd_cnn_load": (I, [C.c_char_p, I, PP]),
    "predictor_save_pca": (I, [C.c_char_p, P, I, I, I, P]),
    "predictor_load": (I, [C.c_char_p, I, PP]),
    "predictor_info": (I, [P, C.POINTER(I), C.POINTER(I), C.POINTER(I), C.POINTER(I),
                           C.POINTER(I)]),
    "predict_subspace": (I, [P, PP, PP, P, I, P, P]),
    "predictor_destroy": (None, [P]),
    "dd_cnn_train_step": (I, [P, P, P, P, I, C.c_float, C.c_float, C.c_float,
                              C.POINTER(C.c_float), P]),
    "dd_cnn_grad": (I, [P, P, P, P, I, C.POINTER(C.c_float), C.POINTER(C.c_float),
                        C.c_size_t, P]),
    "dd_cnn_debug_activation": (I, [P, I, I, C.POINTER(C.c_float), C.c_size_t]),
}


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it first (python -m paper_1902_00090_amd.build)")
    # torch ships its own HIP runtime with the same soname (libamdhip64.so.7);
    # importing torch first makes the dynamic loader reuse that runtime for this
    # library, so the process holds one HIP runtime and device pointers and
    # streams from torch are valid here.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        try:
            fn = getattr(lib, name)
        except AttributeError:
            continue
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def check(status: int, what: str = "") -> int:
    """Raise DDError for negative statuses; return the status otherwise."""
    if status < 0:
        msg = lib().dd_last_error().decode(errors="replace")
        raise DDError(status, f"{what}: {msg}" if what else msg)
    return status


def ptr_array(ptrs):
    arr = (C.c_void_p * len(ptrs))()
    for i, p in enumerate(ptrs):
        arr[i] = p
    return arr
