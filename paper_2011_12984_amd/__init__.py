"""Batched stiff-ODE BDF-Newton on AMD MI355X (gfx950).

Python binding of the C ABI declared in include/bdfgpu.h.  Every function
keeps the C name and only marshals arguments: torch tensors provide device
memory and the current HIP stream.  Dense blocks are passed as contiguous
tensors of shape (nb, n, n) holding column-major blocks, i.e. element (i, j)
of block b is ``A[b, j, i]``.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from ._lib import (BdfGpuError, BdfOptions, BdfProblem, BdfStats, check, check_status, dp, ip,
                   lib, vp)

__all__ = [
    "nvec_linear_sum", "nvec_linear_combination", "nvec_scale_add_multi",
    "nvec_dot_prod_multi", "nvec_dot_prod_multi_noalloc", "nvec_wrms_norm", "nvec_wrms_norm_multi", "nvec_max_norm", "nvec_ewt", "nvec_scale",
    "nvec_const", "batched_lu_factor_f64", "batched_lu_solve_f64", "batched_lu_factor_f32",
    "batched_lu_solve_f32", "batched_lu_solve_refine", "batched_lu_factor_var",
    "batched_lu_solve_var", "Bdf", "BdfGpuError", "lib",
    "LS_LU64", "LS_LU32REF", "LS_LEARNED", "LS_GJ", "MODE_STREAM", "MODE_GRAPH", "RESULT_DEVICE",
    "LAUNCH_PER_CLASS", "LAUNCH_FUSED", "LAUNCH_AUTO", "capture_training_set", "train_precond",
    "Precond",
]

LS_LU64, LS_LU32REF, LS_LEARNED, LS_GJ, LS_GMRES = 0, 1, 2, 3, 4
MODE_STREAM, MODE_GRAPH = 0, 1
LAUNCH_PER_CLASS, LAUNCH_FUSED, LAUNCH_AUTO = 0, 1, 2
RESULT_DEVICE = 1


def _torch():
    import torch
    return torch


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype):
    torch = _torch()
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} device tensor")
    return t


def _ptr_array(ts):
    arr = (vp * len(ts))()
    for j, t in enumerate(ts):
        arr[j] = t.data_ptr()
    return arr


def _dbl_array(vals):
    vals = [float(v) for v in vals]
    return (C.c_double * len(vals))(*vals)


# ---------------------------------------------------------------------------
# vector operations
# ---------------------------------------------------------------------------

def nvec_linear_sum(a, x, b, y, z):
    torch = _torch()
    for t in (x, y, z):
        _dev(t, torch.float64)
    check("nvec_linear_sum", lib().nvec_linear_sum(x.numel(), a, _p(x), b, _p(y), _p(z), _stream()))
    return z


def nvec_linear_combination(c, X, z):
    torch = _torch()
    for t in list(X) + [z]:
        _dev(t, torch.float64)
    cc = _dbl_array(c)
    check("nvec_linear_combination",
          lib().nvec_linear_combination(len(X), C.cast(cc, dp), _ptr_array(X), _p(z), z.numel(),
                                        _stream()))
    return z


def nvec_scale_add_multi(a, x, Y, Z):
    torch = _torch()
    for t in [x] + list(Y) + list(Z):
        _dev(t, torch.float64)
    aa = _dbl_array(a)
    check("nvec_scale_add_multi",
          lib().nvec_scale_add_multi(len(Y), C.cast(aa, dp), _p(x), _ptr_array(Y), _ptr_array(Z),
                                     x.numel(), _stream()))
    return Z


def nvec_dot_prod_multi(x, Y, out=None):
    """Host list of dots (synchronising), or into device tensor `out`."""
    torch = _torch()
    for t in [x] + list(Y):
        _dev(t, torch.float64)
    if out is None:
        d = (C.c_double * len(Y))()
        check("nvec_dot_prod_multi",
              lib().nvec_dot_prod_multi(len(Y), _p(x), _ptr_array(Y), C.cast(d, vp), x.numel(), 0,
                                        _stream()))
        return list(d)
    check("nvec_dot_prod_multi",
          lib().nvec_dot_prod_multi(len(Y), _p(x), _ptr_array(Y), _p(out), x.numel(), RESULT_DEVICE,
                                    _stream()))
    return out


def nvec_dot_prod_multi_noalloc(x, Y, out):
    """Dots into the device tensor `out` without any allocation by the
    library (static per-device scratch; overlapping calls on one GPU race)."""
    torch = _torch()
    for t in [x, out] + list(Y):
        _dev(t, torch.float64)
    check("nvec_dot_prod_multi_noalloc",
          lib().nvec_dot_prod_multi_noalloc(len(Y), _p(x), _ptr_array(Y), _p(out), x.numel(),
                                            _stream()))
    return out


def nvec_wrms_norm(x, w, out=None):
    torch = _torch()
    _dev(x, torch.float64)
    _dev(w, torch.float64)
    if out is None:
        r = C.c_double(0.0)
        check("nvec_wrms_norm", lib().nvec_wrms_norm(x.numel(), _p(x), _p(w), C.cast(C.pointer(r), vp),
                                                     0, _stream()))
        return r.value
    check("nvec_wrms_norm", lib().nvec_wrms_norm(x.numel(), _p(x), _p(w), _p(out), RESULT_DEVICE,
                                                 _stream()))
    return out


def nvec_wrms_norm_multi(X, Wt, out=None):
    """WRMS norms of the vectors X[j] with weights Wt[j] (Wt may repeat one
    tensor): host list (synchronising), or into device tensor `out`."""
    torch = _torch()
    for t in list(X) + list(Wt):
        _dev(t, torch.float64)
    if len(X) != len(Wt):
        raise ValueError("one weight vector per vector")
    n = X[0].numel()
    if out is None:
        d = (C.c_double * len(X))()
        check("nvec_wrms_norm_multi",
              lib().nvec_wrms_norm_multi(len(X), _ptr_array(X), _ptr_array(Wt), C.cast(d, vp), n,
                                         0, _stream()))
        return list(d)
    check("nvec_wrms_norm_multi",
          lib().nvec_wrms_norm_multi(len(X), _ptr_array(X), _ptr_array(Wt), _p(out), n,
                                     RESULT_DEVICE, _stream()))
    return out


def nvec_max_norm(x, out=None):
    torch = _torch()
    _dev(x, torch.float64)
    if out is None:
        r = C.c_double(0.0)
        check("nvec_max_norm", lib().nvec_max_norm(x.numel(), _p(x), C.cast(C.pointer(r), vp), 0,
                                                   _stream()))
        return r.value
    check("nvec_max_norm", lib().nvec_max_norm(x.numel(), _p(x), _p(out), RESULT_DEVICE, _stream()))
    return out


def nvec_ewt(y, rtol, atol, w):
    check("nvec_ewt", lib().nvec_ewt(y.numel(), rtol, atol, _p(y), _p(w), _stream()))
    return w


def nvec_scale(c, x, z):
    check("nvec_scale", lib().nvec_scale(x.numel(), c, _p(x), _p(z), _stream()))
    return z


def nvec_const(c, z):
    check("nvec_const", lib().nvec_const(z.numel(), c, _p(z), _stream()))
    return z


# ---------------------------------------------------------------------------
# batched LU
# ---------------------------------------------------------------------------

def _blocks(A, dtype):
    torch = _torch()
    _dev(A, dtype)
    if A.dim() != 3 or A.shape[1] != A.shape[2]:
        raise ValueError("expected (nb, n, n) blocks")
    return A.shape[0], A.shape[1]


def batched_lu_factor_f64(A, piv, info):
    nb, n = _blocks(A, _torch().float64)
    check("batched_lu_factor_f64",
          lib().batched_lu_factor_f64(nb, n, _p(A), _p(piv), _p(info), _stream()))
    return A, piv, info


def batched_lu_solve_f64(LU, piv, B):
    nb, n = _blocks(LU, _torch().float64)
    check("batched_lu_solve_f64", lib().batched_lu_solve_f64(nb, n, _p(LU), _p(piv), _p(B), _stream()))
    return B


def batched_lu_factor_f32(A, piv, info):
    nb, n = _blocks(A, _torch().float32)
    check("batched_lu_factor_f32",
          lib().batched_lu_factor_f32(nb, n, _p(A), _p(piv), _p(info), _stream()))
    return A, piv, info


def batched_lu_solve_f32(LU, piv, B):
    nb, n = _blocks(LU, _torch().float32)
    check("batched_lu_solve_f32", lib().batched_lu_solve_f32(nb, n, _p(LU), _p(piv), _p(B), _stream()))
    return B


def _var_layout(sizes, device):
    """Device arrays (sizes int32, moff int64, voff int64) of packed blocks."""
    torch = _torch()
    sz = np.asarray(sizes, np.int64)
    moff = np.concatenate([[0], np.cumsum(sz * sz)[:-1]]).astype(np.int64)
    voff = np.concatenate([[0], np.cumsum(sz)[:-1]]).astype(np.int64)
    return (torch.tensor(sz.astype(np.int32), device=device), torch.tensor(moff, device=device),
            torch.tensor(voff, device=device))


def batched_lu_factor_var(A, piv, info, sizes, layout=None, nmax=None):
    """Blocks of uneven sizes packed in A (column-major, block after block);
    float64 or float32.  layout: (sizes, moff, voff) device tensors, else
    the packed layout of `sizes` (host ints)."""
    torch = _torch()
    f64 = A.dtype == torch.float64
    _dev(A, torch.float64 if f64 else torch.float32)
    sz, mo, vo = layout if layout is not None else _var_layout(sizes, A.device)
    nmax = int(max(sizes)) if nmax is None else nmax
    fn = "batched_lu_factor_f64_var" if f64 else "batched_lu_factor_f32_var"
    check(fn, getattr(lib(), fn)(len(sizes), nmax, _p(sz), _p(mo), _p(vo), _p(A), _p(piv),
                                 _p(info), _stream()))
    return A, piv, info


def batched_lu_solve_var(LU, piv, B, sizes, layout=None, nmax=None):
    torch = _torch()
    f64 = LU.dtype == torch.float64
    _dev(LU, torch.float64 if f64 else torch.float32)
    sz, mo, vo = layout if layout is not None else _var_layout(sizes, LU.device)
    nmax = int(max(sizes)) if nmax is None else nmax
    fn = "batched_lu_solve_f64_var" if f64 else "batched_lu_solve_f32_var"
    check(fn, getattr(lib(), fn)(len(sizes), nmax, _p(sz), _p(mo), _p(vo), _p(LU), _p(piv),
                                 _p(B), _stream()))
    return B


def batched_lu_solve_refine(M, LU32, piv32, B, X, max_it, sweeps, status):
    nb, n = _blocks(M, _torch().float64)
    check("batched_lu_solve_refine",
          lib().batched_lu_solve_refine(nb, n, _p(M), _p(LU32), _p(piv32), _p(B), _p(X), max_it,
                                        _p(sweeps), _p(status), _stream()))
    return X


# ---------------------------------------------------------------------------
# BDF integrator
# ---------------------------------------------------------------------------

class Bdf:
    """Handle on a grouped BDF integrator (bdf_create ... bdf_destroy).

    topologies: list of (nu, mu) integer arrays of shape (R, n);
    cell_topo: int array (ncells,); rates, y0: float64 device tensors
    (concatenated per cell).  jit: compile network-specialised Newton
    kernels for the one-lane-per-cell classes (bitwise the same results).
    defer: apply each accepted step's history update in the next attempt's
    Newton kernel (where the classes allow it) instead of a separate pass.
    newton_per_launch: Newton iterations per launch of the fused kernel
    (0: 2); the results do not depend on it."""

    def __init__(self, topologies, cell_topo, rates, y0, t0=0.0, rtol=1e-6, atol=1e-10,
                 qmax=5, maxcor=3, h0=0.0, hmin=0.0, linsol=LS_LU64, refine_max_it=5,
                 max_steps=0, mode=MODE_STREAM, attempts_per_sync=8, nonneg=False,
                 precond=None, launch=LAUNCH_PER_CLASS, map_small=0, jit=False, defer=True,
                 workspace=None, per_cell=False, vc=False, lazy=False, newton_per_launch=0):
        torch = _torch()
        _dev(rates, torch.float64)
        _dev(y0, torch.float64)
        self._keep = []
        topo_n = np.array([nu.shape[1] for nu, _ in topologies], np.int32)
        topo_R = np.array([nu.shape[0] for nu, _ in topologies], np.int32)
        off = np.concatenate([[0], np.cumsum(topo_n * topo_R)[:-1]]).astype(np.int32)
        nu_all = np.concatenate([np.ascontiguousarray(nu, np.int32).ravel() for nu, _ in topologies]).astype(np.int32)
        mu_all = np.concatenate([np.ascontiguousarray(mu, np.int32).ravel() for _, mu in topologies]).astype(np.int32)
        ct = np.ascontiguousarray(cell_topo, np.int32)
        self._keep += [topo_n, topo_R, off, nu_all, mu_all, ct, rates, y0]
        ipt = lambda a: a.ctypes.data_as(ip)
        prob = BdfProblem(len(topo_n), ipt(topo_n), ipt(topo_R), ipt(off), ipt(nu_all),
                          ipt(mu_all), len(ct), ipt(ct), _p(rates), _p(y0), float(t0))
        self._precond = precond
        opts = BdfOptions(rtol, atol, qmax, maxcor, h0, hmin, linsol, refine_max_it, max_steps,
                          mode, attempts_per_sync, launch,
                          precond.h if precond is not None else None, int(bool(nonneg)),
                          int(map_small), int(bool(jit)), int(not defer), int(bool(per_cell)),
                          int(bool(vc)), int(bool(lazy)), int(newton_per_launch))
        h = vp()
        if workspace is None:
            check("bdf_create", lib().bdf_create(C.byref(prob), C.byref(opts), _stream(),
                                                 C.byref(h)))
        else:
            # caller-owned device workspace (a uint8 tensor kept alive by
            # the handle), sized with workspace_bytes
            if not workspace.is_cuda or not workspace.is_contiguous():
                raise ValueError("workspace must be a contiguous device tensor")
            self._keep.append(workspace)
            check("bdf_create_ws", lib().bdf_create_ws(
                C.byref(prob), C.byref(opts), _p(workspace),
                workspace.numel() * workspace.element_size(), _stream(), C.byref(h)))
        self.h = h
        self.N = lib().bdf_get_N(h)
        self.device = y0.device

    @staticmethod
    def workspace_bytes(prob, **kw):
        """Device bytes a handle of this problem and these options needs
        (bdf_workspace_bytes); options as for the constructor."""
        return Bdf._sizing(prob, **kw)

    @staticmethod
    def _sizing(prob, rtol=None, atol=None, qmax=None, maxcor=3, h0=0.0, hmin=0.0, linsol=LS_LU64,
                refine_max_it=5, max_steps=0, mode=MODE_STREAM, attempts_per_sync=8,
                nonneg=None, launch=LAUNCH_PER_CLASS, map_small=0, jit=False, defer=True,
                precond=None, per_cell=False, vc=False, lazy=False, newton_per_launch=0):
        topologies = prob["topologies"]
        topo_n = np.array([nu.shape[1] for nu, _ in topologies], np.int32)
        topo_R = np.array([nu.shape[0] for nu, _ in topologies], np.int32)
        off = np.concatenate([[0], np.cumsum(topo_n * topo_R)[:-1]]).astype(np.int32)
        nu_all = np.concatenate([np.ascontiguousarray(nu, np.int32).ravel() for nu, _ in topologies]).astype(np.int32)
        mu_all = np.concatenate([np.ascontiguousarray(mu, np.int32).ravel() for _, mu in topologies]).astype(np.int32)
        ct = np.ascontiguousarray(prob["cell_topo"], np.int32)
        ipt = lambda a: a.ctypes.data_as(ip)
        pr = BdfProblem(len(topo_n), ipt(topo_n), ipt(topo_R), ipt(off), ipt(nu_all), ipt(mu_all),
                        len(ct), ipt(ct), None, None, float(prob["t0"]))
        opts = BdfOptions(prob["rtol"] if rtol is None else rtol, prob["atol"] if atol is None else atol,
                          prob["qmax"] if qmax is None else qmax, maxcor, h0, hmin, linsol,
                          refine_max_it, max_steps, mode, attempts_per_sync, launch,
                          precond.h if precond is not None else None,
                          int(bool(prob.get("nonneg", False) if nonneg is None else nonneg)),
                          int(map_small), int(bool(jit)), int(not defer), int(bool(per_cell)),
                          int(bool(vc)), int(bool(lazy)), int(newton_per_launch))
        return int(lib().bdf_workspace_bytes(C.byref(pr), C.byref(opts)))

    @classmethod
    def from_problem(cls, prob, device="cuda", **kw):
        torch = _torch()
        rates = torch.tensor(np.asarray(prob["rates"], np.float64), device=device)
        y0 = torch.tensor(np.asarray(prob["y0"], np.float64), device=device)
        kw.setdefault("rtol", prob["rtol"])
        kw.setdefault("atol", prob["atol"])
        kw.setdefault("qmax", prob["qmax"])
        kw.setdefault("nonneg", bool(prob.get("nonneg", False)))
        return cls(prob["topologies"], prob["cell_topo"], rates, y0, t0=prob["t0"], **kw)

    def close(self):
        if getattr(self, "h", None):
            lib().bdf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, t_end):
        t = C.c_double(0.0)
        check_status("bdf_step", lib().bdf_step(self.h, t_end, C.byref(t)))
        return t.value

    def integrate(self, t_end):
        t = C.c_double(0.0)
        check_status("bdf_integrate", lib().bdf_integrate(self.h, t_end, C.byref(t)))
        return t.value

    def advance(self, t_end, nsteps):
        """At most nsteps accepted steps towards t_end; returns (t, taken)."""
        t = C.c_double(0.0)
        taken = C.c_long(0)
        check_status("bdf_advance",
                     lib().bdf_advance(self.h, t_end, nsteps, C.byref(t), C.byref(taken)))
        return t.value, taken.value

    def set_profiling(self, on=True):
        check("bdf_set_profiling", lib().bdf_set_profiling(self.h, 1 if on else 0))

    def tuning(self):
        """{"launch": 0/1, "map_small": 0/1, "ms_per_step": {(launch, map_small): ms}}"""
        la, ms = C.c_int(0), C.c_int(0)
        t = (C.c_double * 4)()
        check("bdf_get_tuning", lib().bdf_get_tuning(self.h, C.byref(la), C.byref(ms),
                                                     C.cast(t, dp)))
        return {"launch": la.value, "map_small": ms.value,
                "ms_per_step": {(k // 2, k % 2): t[k] for k in range(4) if t[k] >= 0}}

    def kernel_times(self):
        """{group: (total_ms, launches)}: "newton" (predictor, factorisation
        and all Newton iterations), "learned" (predictor and MLP inference,
        learned mode only), "accept" (history update)."""
        ms = (C.c_double * 3)()
        cnt = (C.c_long * 3)()
        check("bdf_get_kernel_times", lib().bdf_get_kernel_times(self.h, C.cast(ms, dp),
                                                                 C.cast(cnt, C.POINTER(C.c_long))))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(("newton", "learned", "accept"))}

    def cell_stats(self, with_hu=False):
        """Per-cell stepping: (counts (ncells, 5): steps, attempts, Newton
        iterations, error-test and convergence failures; t (ncells,)), and
        the last accepted step sizes (ncells,) when with_hu."""
        nc = len(self._keep[5])
        counts = np.zeros((nc, 5), np.int32)
        t = np.zeros(nc)
        hu = np.zeros(nc)
        check("bdf_get_cell_stats", lib().bdf_get_cell_stats(
            self.h, C.c_void_p(counts.ctypes.data), C.c_void_p(t.ctypes.data),
            C.c_void_p(hu.ctypes.data)))
        return (counts, t, hu) if with_hu else (counts, t)

    def y(self):
        torch = _torch()
        y = torch.empty(self.N, dtype=torch.float64, device=self.device)
        check("bdf_get_y", lib().bdf_get_y(self.h, _p(y)))
        torch.cuda.current_stream().synchronize()
        return y

    def stats(self):
        s = BdfStats()
        check("bdf_get_stats", lib().bdf_get_stats(self.h, C.byref(s)))
        return s.as_dict()

    def get_state(self):
        torch = _torch()
        dv = (C.c_double * 2)()
        iv = (C.c_int * 2)()
        z6 = torch.empty(6 * self.N, dtype=torch.float64, device=self.device)
        dpv = torch.empty(self.N, dtype=torch.float64, device=self.device)
        check("bdf_get_state", lib().bdf_get_state(self.h, C.cast(dv, dp), C.cast(iv, ip), _p(z6), _p(dpv)))
        return dict(t=dv[0], h=dv[1], q=iv[0], qwait=iv[1], z=z6.view(6, self.N), dprev=dpv)

    def set_state(self, t, h, q, qwait, z6, dprev):
        dv = (C.c_double * 2)(t, h)
        iv = (C.c_int * 2)(q, qwait)
        z6 = z6.contiguous().view(-1)
        check("bdf_set_state", lib().bdf_set_state(self.h, C.cast(dv, dp), C.cast(iv, ip), _p(z6),
                                                   _p(dprev.contiguous())))

    def capture_blocks(self, n, stride, max_blocks):
        """(X_raw (k, n+1), M (k, n*n) column-major) device tensors."""
        torch = _torch()
        X = torch.empty(max(1, max_blocks) * (n + 1), dtype=torch.float64, device=self.device)
        M = torch.empty(max(1, max_blocks) * n * n, dtype=torch.float64, device=self.device)
        got = C.c_long(0)
        check("bdf_capture_blocks", lib().bdf_capture_blocks(self.h, n, stride, max_blocks, _p(X),
                                                             _p(M), C.byref(got)))
        k = got.value
        return X[: k * (n + 1)].view(k, n + 1), M[: k * n * n].view(k, n * n)

    def eval_rhs_jac(self, y, jac_entries):
        torch = _torch()
        f = torch.empty(self.N, dtype=torch.float64, device=self.device)
        J = torch.empty(jac_entries, dtype=torch.float64, device=self.device)
        check("bdf_eval_rhs_jac", lib().bdf_eval_rhs_jac(self.h, _p(y.contiguous()), _p(f), _p(J)))
        return f, J


class Precond:
    """Learned block preconditioner (precond_create ... precond_destroy)."""

    def __init__(self, n, hid=256, batch_cap=1024):
        h = vp()
        check("precond_create", lib().precond_create(n, hid, batch_cap, C.byref(h)))
        self.h = h
        self.n, self.hid, self.batch_cap = n, hid, batch_cap
        self.np = lib().precond_num_params(h)

    def close(self):
        if getattr(self, "h", None):
            lib().precond_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        p = np.ascontiguousarray(params, np.float32)
        assert p.size == self.np
        check("precond_set_params", lib().precond_set_params(self.h, C.c_void_p(p.ctypes.data)))

    def get_params(self, with_grads=False):
        p = np.empty(self.np, np.float32)
        g = np.empty(self.np, np.float32) if with_grads else None
        check("precond_get_params", lib().precond_get_params(
            self.h, C.c_void_p(p.ctypes.data), C.c_void_p(g.ctypes.data) if g is not None else None))
        return (p, g) if with_grads else p

    def set_normalization(self, mean, std):
        m = np.ascontiguousarray(mean, np.float64)
        sd = np.ascontiguousarray(std, np.float64)
        check("precond_set_normalization", lib().precond_set_normalization(
            self.h, m.ctypes.data_as(dp), sd.ctypes.data_as(dp)))

    def get_normalization(self):
        m = np.empty(self.n + 1)
        sd = np.empty(self.n + 1)
        check("precond_get_normalization", lib().precond_get_normalization(
            self.h, m.ctypes.data_as(dp), sd.ctypes.data_as(dp)))
        return m, sd

    def fit_normalization(self, X):
        check("precond_fit_normalization", lib().precond_fit_normalization(
            self.h, _p(X), X.shape[0], _stream()))

    def loss_grad(self, X, M):
        loss = C.c_double(0.0)
        check("precond_loss_grad", lib().precond_loss_grad(self.h, X.shape[0], _p(X), _p(M),
                                                           C.byref(loss), _stream()))
        return loss.value

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        check("precond_adam", lib().precond_adam(self.h, lr, b1, b2, eps, _stream()))

    def train_epoch(self, X, M, perm, batch=1024, lr=1e-3):
        loss = C.c_double(0.0)
        check("precond_train_epoch", lib().precond_train_epoch(
            self.h, X.shape[0], _p(X), _p(M), _p(perm), batch, lr, C.byref(loss), _stream()))
        return loss.value

    def eval_loss(self, X, M):
        loss = C.c_double(0.0)
        check("precond_eval_loss", lib().precond_eval_loss(self.h, X.shape[0], _p(X), _p(M),
                                                           C.byref(loss), _stream()))
        return loss.value

    def forward(self, X, use_mfma=True):
        torch = _torch()
        out = torch.empty(X.shape[0], self.n * self.n, dtype=torch.float32, device=X.device)
        check("precond_forward", lib().precond_forward(self.h, X.shape[0], _p(X), _p(out),
                                                       1 if use_mfma else 0, _stream()))
        return out


# ---------------------------------------------------------------------------
# Training pipeline of the learned preconditioner (host orchestration of the
# C ABI: every step runs in the library's kernels)
# ---------------------------------------------------------------------------

def capture_training_set(bdf, n, nblocks, per_capture=4096, steps_between=8, t_end=None):
    """Advance a plain integrator and capture blocks M = I - gamma J(y) with
    their MLP inputs [y, log gamma] until `nblocks` are collected.  Each
    capture takes every stride-th cell so that one capture yields at most
    `per_capture` blocks.  Returns device tensors (X (k, n+1), M (k, n*n))."""
    torch = _torch()
    ncells = bdf.N // n
    stride = max(1, ncells // per_capture)
    Xs, Ms, got = [], [], 0
    t_end = float("inf") if t_end is None else t_end
    while got < nblocks:
        X, M = bdf.capture_blocks(n, stride, min(per_capture, nblocks - got))
        Xs.append(X.clone())
        Ms.append(M.clone())
        got += X.shape[0]
        t, taken = bdf.advance(t_end, steps_between)
        if taken == 0:
            break
    return torch.cat(Xs), torch.cat(Ms)


def train_precond(pc, X, M, epochs=30, batch=1024, lr=1e-3, val_frac=0.1, seed=0):
    """Split off a seeded random `val_frac` for validation, fit the input
    normalisation on the training part, then `epochs` passes of mini-batch
    Adam over seeded permutations.  Returns
    {"train": [mean loss per epoch], "val": [held-out loss per epoch],
    "val0": held-out loss before training}."""
    torch = _torch()
    ns = X.shape[0]
    nval = int(ns * val_frac)
    gen = torch.Generator(device=X.device)
    gen.manual_seed(seed)
    split = torch.randperm(ns, generator=gen, device=X.device)
    iva, itr = split[:nval], split[nval:]
    Xva, Mva = X.index_select(0, iva).contiguous(), M.index_select(0, iva).contiguous()
    Xtr, Mtr = X.index_select(0, itr).contiguous(), M.index_select(0, itr).contiguous()
    pc.fit_normalization(Xtr)
    hist = {"train": [], "val": [], "val0": pc.eval_loss(Xva, Mva) if nval else None}
    for _ in range(epochs):
        perm = torch.randperm(Xtr.shape[0], generator=gen, device=X.device).to(torch.int32)
        hist["train"].append(pc.train_epoch(Xtr, Mtr, perm, batch=batch, lr=lr))
        if nval:
            hist["val"].append(pc.eval_loss(Xva, Mva))
    return hist
