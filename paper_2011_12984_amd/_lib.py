"""ctypes binding of libbdfgpu.so (the C ABI in include/bdfgpu.h).

Argument marshalling only: torch tensors supply device memory and the
current HIP stream; every computation happens in the library's kernels.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# BDFGPU_LIB selects another build of the same library (for A/B timing)
LIB_PATH = os.environ.get("BDFGPU_LIB") or os.path.join(HERE, "libbdfgpu.so")

_lib = None

vp = C.c_void_p
dp = C.POINTER(C.c_double)
ip = C.POINTER(C.c_int)


class BdfProblem(C.Structure):
    _fields_ = [("ntopo", C.c_int), ("topo_n", ip), ("topo_R", ip), ("topo_off", ip),
                ("nu_all", ip), ("mu_all", ip), ("ncells", C.c_long), ("cell_topo", ip),
                ("rates", vp), ("y0", vp), ("t0", C.c_double)]


class BdfOptions(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("qmax", C.c_int),
                ("maxcor", C.c_int), ("h0", C.c_double), ("hmin", C.c_double),
                ("linsol", C.c_int), ("refine_max_it", C.c_int), ("max_steps", C.c_long),
                ("mode", C.c_int), ("attempts_per_sync", C.c_int), ("launch", C.c_int),
                ("precond", vp), ("nonneg", C.c_int), ("map_small", C.c_int),
                ("jit", C.c_int), ("no_defer", C.c_int), ("per_cell", C.c_int),
                ("vc", C.c_int), ("lazy", C.c_int), ("newton_per_launch", C.c_int)]


class BdfStats(C.Structure):
    _fields_ = [(k, C.c_long) for k in (
        "nsteps", "nattempts", "nfevals", "nsetups", "nniters", "nncfails", "netfails",
        "nlinsolves", "refine_sweeps", "refine_fallbacks", "nprojections", "hist_reads",
        "lp_cell_solves", "lp_fallback_cells", "lp_step_fallbacks")] + [
        ("order_hist", C.c_long * 6), ("t", C.c_double), ("h", C.c_double),
        ("hu", C.c_double), ("err_last", C.c_double), ("q", C.c_int), ("qu", C.c_int),
        ("qwait", C.c_int), ("status", C.c_int), ("nstale_retries", C.c_long),
        ("nliters", C.c_long), ("ncont", C.c_long)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "order_hist"}
        d["order_hist"] = list(self.order_hist)
        return d


# name -> (restype, argtypes)
SIGNATURES = {
    "bdfgpu_last_error": (C.c_char_p, []),
    "bdfgpu_version": (C.c_char_p, []),
    "nvec_linear_sum": (C.c_int, [C.c_long, C.c_double, vp, C.c_double, vp, vp, vp]),
    "nvec_linear_combination": (C.c_int, [C.c_int, dp, C.POINTER(vp), vp, C.c_long, vp]),
    "nvec_scale_add_multi": (C.c_int, [C.c_int, dp, vp, C.POINTER(vp), C.POINTER(vp), C.c_long, vp]),
    "nvec_dot_prod_multi": (C.c_int, [C.c_int, vp, C.POINTER(vp), vp, C.c_long, C.c_int, vp]),
    "nvec_dot_prod_multi_noalloc": (C.c_int, [C.c_int, vp, C.POINTER(vp), vp, C.c_long, vp]),
    "nvec_wrms_norm": (C.c_int, [C.c_long, vp, vp, vp, C.c_int, vp]),
    "nvec_wrms_norm_multi": (C.c_int, [C.c_int, C.POINTER(vp), C.POINTER(vp), vp, C.c_long, C.c_int, vp]),
    "nvec_max_norm": (C.c_int, [C.c_long, vp, vp, C.c_int, vp]),
    "nvec_ewt": (C.c_int, [C.c_long, C.c_double, C.c_double, vp, vp, vp]),
    "nvec_scale": (C.c_int, [C.c_long, C.c_double, vp, vp, vp]),
    "nvec_const": (C.c_int, [C.c_long, C.c_double, vp, vp]),
    "batched_lu_factor_f64": (C.c_int, [C.c_int, C.c_int, vp, vp, vp, vp]),
    "batched_lu_solve_f64": (C.c_int, [C.c_int, C.c_int, vp, vp, vp, vp]),
    "batched_lu_factor_f32": (C.c_int, [C.c_int, C.c_int, vp, vp, vp, vp]),
    "batched_lu_solve_f32": (C.c_int, [C.c_int, C.c_int, vp, vp, vp, vp]),
    "batched_lu_factor_f64_var": (C.c_int, [C.c_int, C.c_int, vp, vp, vp, vp, vp, vp, vp]),
    "batched_lu_solve_f64_var": (C.c_int, [C.c_int, C.c_int, vp, vp, vp, vp, vp, vp, vp]),
    "batched_lu_factor_f32_var": (C.c_int, [C.c_int, C.c_int, vp, vp, vp, vp, vp, vp, vp]),
    "batched_lu_solve_f32_var": (C.c_int, [C.c_int, C.c_int, vp, vp, vp, vp, vp, vp, vp]),
    "batched_lu_solve_refine": (C.c_int, [C.c_int, C.c_int, vp, vp, vp, vp, vp, C.c_int, vp, vp, vp]),
    "bdf_create": (C.c_int, [C.POINTER(BdfProblem), C.POINTER(BdfOptions), vp, C.POINTER(vp)]),
    "bdf_workspace_bytes": (C.c_size_t, [C.POINTER(BdfProblem), C.POINTER(BdfOptions)]),
    "bdf_create_ws": (C.c_int, [C.POINTER(BdfProblem), C.POINTER(BdfOptions), vp, C.c_size_t, vp,
                                C.POINTER(vp)]),
    "bdf_destroy": (C.c_int, [vp]),
    "bdf_get_tuning": (C.c_int, [vp, ip, ip, dp]),
    "bdf_step": (C.c_int, [vp, C.c_double, dp]),
    "bdf_integrate": (C.c_int, [vp, C.c_double, dp]),
    "bdf_advance": (C.c_int, [vp, C.c_double, C.c_long, dp, C.POINTER(C.c_long)]),
    "bdf_set_profiling": (C.c_int, [vp, C.c_int]),
    "bdf_get_kernel_times": (C.c_int, [vp, dp, C.POINTER(C.c_long)]),
    "bdf_get_y": (C.c_int, [vp, vp]),
    "bdf_get_stats": (C.c_int, [vp, C.POINTER(BdfStats)]),
    "bdf_get_N": (C.c_long, [vp]),
    "bdf_get_cell_stats": (C.c_int, [vp, vp, vp, vp]),
    "bdf_get_state": (C.c_int, [vp, dp, ip, vp, vp]),
    "bdf_set_state": (C.c_int, [vp, dp, ip, vp, vp]),
    "bdf_eval_rhs_jac": (C.c_int, [vp, vp, vp, vp]),
    "bdf_capture_blocks": (C.c_int, [vp, C.c_int, C.c_long, C.c_long, vp, vp, C.POINTER(C.c_long)]),
    "precond_create": (C.c_int, [C.c_int, C.c_int, C.c_int, C.POINTER(vp)]),
    "precond_destroy": (C.c_int, [vp]),
    "precond_num_params": (C.c_long, [vp]),
    "precond_set_params": (C.c_int, [vp, vp]),
    "precond_get_params": (C.c_int, [vp, vp, vp]),
    "precond_set_normalization": (C.c_int, [vp, dp, dp]),
    "precond_get_normalization": (C.c_int, [vp, dp, dp]),
    "precond_fit_normalization": (C.c_int, [vp, vp, C.c_long, vp]),
    "precond_loss_grad": (C.c_int, [vp, C.c_int, vp, vp, dp, vp]),
    "precond_adam": (C.c_int, [vp, C.c_double, C.c_double, C.c_double, C.c_double, vp]),
    "precond_train_epoch": (C.c_int, [vp, C.c_long, vp, vp, vp, C.c_int, C.c_double, dp, vp]),
    "precond_eval_loss": (C.c_int, [vp, C.c_long, vp, vp, dp, vp]),
    "precond_forward": (C.c_int, [vp, C.c_long, vp, vp, C.c_int, vp]),
}


def lib():
    """Load libbdfgpu.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2011_12984_amd.build` "
                "(the GPU path has no fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class BdfGpuError(RuntimeError):
    def __init__(self, fn, code):
        msg = lib().bdfgpu_last_error()
        super().__init__(f"{fn} returned {code}: {msg.decode() if msg else ''}")
        self.code = code


def check(fn, code):
    if code < 0:
        raise BdfGpuError(fn, code)
    return code


def check_status(fn, code):
    """Integrator calls: a positive status is a recoverable failure of the
    step (the handle stops at its last accepted state), also raised."""
    if code != 0:
        raise BdfGpuError(fn, code)
    return code
