"""Python handle on the serial FP64 CPU oracle (``oracle/orc.c``).

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this module.  The product library
never loads it and shares no code with it.

Every function here is argument marshalling around the C routines; the
arithmetic lives in ``orc.c``.  Dense blocks cross this boundary as numpy
arrays of shape (nb, n, n) in mathematical (row, column) order and are
handed to C column-major.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "orc.c")
LIB = os.path.join(HERE, "liborc.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = C.CDLL(LIB)
        _declare(_lib)
    return _lib


dp = C.POINTER(C.c_double)
fp = C.POINTER(C.c_float)
ip = C.POINTER(C.c_int)


class OrcMLP(C.Structure):
    _fields_ = [("nin", C.c_int), ("hid", C.c_int), ("nout", C.c_int),
                ("W1", fp), ("b1", fp), ("W2", fp), ("b2", fp),
                ("W3", fp), ("b3", fp), ("in_mean", dp), ("in_std", dp)]


class OrcProblem(C.Structure):
    _fields_ = [("ntopo", C.c_int), ("topo_n", ip), ("topo_R", ip),
                ("topo_off", ip), ("nu_all", ip), ("mu_all", ip),
                ("ncells", C.c_long), ("cell_topo", ip), ("rates", dp),
                ("y0", dp), ("t0", C.c_double)]


class OrcOptions(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("qmax", C.c_int),
                ("maxcor", C.c_int), ("h0", C.c_double), ("linsol", C.c_int),
                ("refine_max_it", C.c_int), ("max_steps", C.c_long),
                ("hmin", C.c_double), ("mlp", C.POINTER(OrcMLP)), ("nonneg", C.c_int),
                ("fixed_step", C.c_int), ("vc", C.c_int), ("lazy", C.c_int)]


class OrcStats(C.Structure):
    _fields_ = [(k, C.c_long) for k in (
        "nsteps", "nattempts", "nfevals", "nsetups", "nniters", "nncfails",
        "netfails", "nlinsolves", "refine_sweeps", "refine_fallbacks",
        "lp_cell_solves", "lp_fallback_cells", "lp_step_fallbacks")] + [
        ("order_hist", C.c_long * 6), ("nprojections", C.c_long), ("nstale_retries", C.c_long),
        ("nliters", C.c_long), ("lp_unconverged", C.c_long)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "order_hist"}
        d["order_hist"] = list(self.order_hist)
        return d


class OrcScalars(C.Structure):
    _fields_ = [("t", C.c_double), ("h", C.c_double), ("err_last", C.c_double),
                ("q", C.c_int), ("qwait", C.c_int), ("qprime_pending", C.c_int),
                ("initialized", C.c_int), ("hu", C.c_double), ("qu", C.c_int),
                ("err_qm1", C.c_double), ("err_qp1", C.c_double),
                ("eta_proposed", C.c_double), ("q_proposed", C.c_int)]


def _declare(L):
    L.orc_nv_wrms_norm.restype = C.c_double
    L.orc_nv_wrms_norm.argtypes = [C.c_long, dp, dp]
    L.orc_nv_max_norm.restype = C.c_double
    L.orc_nv_max_norm.argtypes = [C.c_long, dp]
    L.orc_nv_linear_sum.argtypes = [C.c_long, C.c_double, dp, C.c_double, dp, dp]
    L.orc_nv_linear_combination.argtypes = [C.c_int, dp, C.POINTER(dp), dp, C.c_long]
    L.orc_nv_scale_add_multi.argtypes = [C.c_int, dp, dp, C.POINTER(dp), C.POINTER(dp), C.c_long]
    L.orc_nv_dot_prod_multi.argtypes = [C.c_int, dp, C.POINTER(dp), dp, C.c_long]
    L.orc_nv_ewt.argtypes = [C.c_long, C.c_double, C.c_double, dp, dp]
    L.orc_nv_scale.argtypes = [C.c_long, C.c_double, dp, dp]
    L.orc_nv_const.argtypes = [C.c_long, C.c_double, dp]
    L.orc_lu_factor.restype = C.c_int
    L.orc_lu_factor.argtypes = [C.c_int, dp, ip]
    L.orc_lu_solve.argtypes = [C.c_int, dp, ip, dp]
    L.orc_lu_factor_f32.restype = C.c_int
    L.orc_lu_factor_f32.argtypes = [C.c_int, fp, ip]
    L.orc_lu_solve_f32.argtypes = [C.c_int, fp, ip, fp]
    L.orc_lu_refine_solve.restype = C.c_int
    L.orc_lu_refine_solve.argtypes = [C.c_int, dp, fp, ip, dp, dp, C.c_int, ip]
    L.orc_gj_inverse.restype = C.c_int
    L.orc_gj_inverse.argtypes = [C.c_int, dp, dp]
    L.orc_ma_rhs.argtypes = [C.c_int, C.c_int, ip, ip, dp, dp, dp]
    L.orc_ma_jac.argtypes = [C.c_int, C.c_int, ip, ip, dp, dp, dp]
    L.orc_set_bf16.argtypes = [C.c_int]
    L.orc_bf16_round.restype = C.c_float
    L.orc_bf16_round.argtypes = [C.c_float]
    L.orc_mlp_forward.argtypes = [C.POINTER(OrcMLP), dp, dp]
    L.orc_mlp_loss_grad.restype = C.c_double
    L.orc_mlp_loss_grad.argtypes = [C.POINTER(OrcMLP), C.c_int, dp, dp, dp, dp, dp, dp, dp, dp]
    L.orc_adam_step.argtypes = [C.c_long, fp, dp, dp, dp, C.c_long, C.c_double,
                                C.c_double, C.c_double, C.c_double]
    L.orc_bdf_create.restype = C.c_void_p
    L.orc_bdf_create.argtypes = [C.POINTER(OrcProblem), C.POINTER(OrcOptions)]
    L.orc_bdf_destroy.argtypes = [C.c_void_p]
    L.orc_bdf_N.restype = C.c_long
    L.orc_bdf_N.argtypes = [C.c_void_p]
    L.orc_bdf_step.restype = C.c_int
    L.orc_bdf_step.argtypes = [C.c_void_p, C.c_double]
    L.orc_bdf_integrate.restype = C.c_int
    L.orc_bdf_integrate.argtypes = [C.c_void_p, C.c_double]
    L.orc_bdf_init.argtypes = [C.c_void_p, C.c_double]
    L.orc_bdf_get_y.argtypes = [C.c_void_p, dp]
    L.orc_bdf_get_stats.argtypes = [C.c_void_p, C.POINTER(OrcStats)]
    L.orc_bdf_get_scalars.argtypes = [C.c_void_p, C.POINTER(OrcScalars)]
    L.orc_bdf_set_scalars.argtypes = [C.c_void_p, C.POINTER(OrcScalars)]
    L.orc_bdf_get_history.argtypes = [C.c_void_p, dp, dp]
    L.orc_bdf_set_history.argtypes = [C.c_void_p, dp, dp]
    L.orc_bdf_coeffs.argtypes = [C.c_int, dp, dp]
    L.orc_bdf_set_past_steps.argtypes = [C.c_void_p, C.c_int, dp, C.c_double, C.c_double]
    L.orc_bdf_get_past_steps.restype = C.c_int
    L.orc_bdf_get_past_steps.argtypes = [C.c_void_p, dp, dp, dp]
    L.orc_bdf_get_lazy.argtypes = [C.c_void_p, dp, C.POINTER(C.c_long), dp]
    L.orc_gmres_solve.restype = C.c_int
    L.orc_gmres_solve.argtypes = [C.c_long, ip, dp, dp, ip, dp, dp, C.c_double, dp]


def _d(a):
    return a.ctypes.data_as(dp)


def _f(a):
    return a.ctypes.data_as(fp)


def _i(a):
    return a.ctypes.data_as(ip)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptrs(arrs):
    P = (dp * len(arrs))()
    for j, a in enumerate(arrs):
        P[j] = _d(a)
    return P


# ----------------------------------------------------------------------------
# Vector operations
# ----------------------------------------------------------------------------

def linear_sum(a, x, b, y):
    x, y = _c64(x), _c64(y)
    z = np.empty_like(x)
    lib().orc_nv_linear_sum(len(x), a, _d(x), b, _d(y), _d(z))
    return z


def linear_combination(c, X):
    X = [_c64(x) for x in X]
    c = _c64(c)
    z = np.empty_like(X[0])
    lib().orc_nv_linear_combination(len(X), _d(c), _ptrs(X), _d(z), len(z))
    return z


def scale_add_multi(a, x, Y):
    x = _c64(x)
    Y = [_c64(v) for v in Y]
    a = _c64(a)
    Z = [np.empty_like(x) for _ in Y]
    lib().orc_nv_scale_add_multi(len(Y), _d(a), _d(x), _ptrs(Y), _ptrs(Z), len(x))
    return Z


def dot_prod_multi(x, Y):
    x = _c64(x)
    Y = [_c64(v) for v in Y]
    d = np.empty(len(Y))
    lib().orc_nv_dot_prod_multi(len(Y), _d(x), _ptrs(Y), _d(d), len(x))
    return d


def wrms_norm(x, w):
    x, w = _c64(x), _c64(w)
    return lib().orc_nv_wrms_norm(len(x), _d(x), _d(w))


def max_norm(x):
    x = _c64(x)
    return lib().orc_nv_max_norm(len(x), _d(x))


def ewt(y, rtol, atol):
    y = _c64(y)
    w = np.empty_like(y)
    lib().orc_nv_ewt(len(y), rtol, atol, _d(y), _d(w))
    return w


def scale(c, x):
    x = _c64(x)
    z = np.empty_like(x)
    lib().orc_nv_scale(len(x), c, _d(x), _d(z))
    return z


def const(c, n):
    z = np.empty(n)
    lib().orc_nv_const(n, c, _d(z))
    return z


# ----------------------------------------------------------------------------
# Dense LU per block
# ----------------------------------------------------------------------------

def lu_factor(A):
    """A: (nb, n, n).  Returns (LU (nb, n, n), piv (nb, n) 0-based, info (nb,))."""
    A = np.asarray(A, dtype=np.float64)
    nb, n, _ = A.shape
    LU = np.empty_like(A)
    piv = np.zeros((nb, n), dtype=np.int32)
    info = np.zeros(nb, dtype=np.int32)
    for b in range(nb):
        cm = np.asfortranarray(A[b]).ravel(order="F").copy()
        pv = np.zeros(n, dtype=np.int32)
        info[b] = lib().orc_lu_factor(n, _d(cm), _i(pv))
        LU[b] = cm.reshape(n, n, order="F")
        piv[b] = pv
    return LU, piv, info


def gj_inverse(A):
    """A: (nb, n, n).  Returns (inverses (nb, n, n), info (nb,)) by
    Gauss-Jordan elimination with partial pivoting."""
    A = np.asarray(A, dtype=np.float64)
    nb, n, _ = A.shape
    Xs = np.zeros_like(A)
    info = np.zeros(nb, dtype=np.int32)
    for b in range(nb):
        cm = np.asfortranarray(A[b]).ravel(order="F").copy()
        X = np.zeros(n * n)
        info[b] = lib().orc_gj_inverse(n, _d(cm), _d(X))
        Xs[b] = X.reshape(n, n)
    return Xs, info


def lu_solve(LU, piv, B):
    LU = np.asarray(LU, dtype=np.float64)
    nb, n, _ = LU.shape
    X = _c64(B).reshape(nb, n).copy()
    for b in range(nb):
        cm = LU[b].ravel(order="F").copy()
        pv = np.ascontiguousarray(piv[b], dtype=np.int32)
        xb = X[b].copy()
        lib().orc_lu_solve(n, _d(cm), _i(pv), _d(xb))
        X[b] = xb
    return X


def lu_factor_f32(A):
    A = np.asarray(A, dtype=np.float32)
    nb, n, _ = A.shape
    LU = np.empty_like(A)
    piv = np.zeros((nb, n), dtype=np.int32)
    info = np.zeros(nb, dtype=np.int32)
    for b in range(nb):
        cm = A[b].ravel(order="F").astype(np.float32).copy()
        pv = np.zeros(n, dtype=np.int32)
        info[b] = lib().orc_lu_factor_f32(n, _f(cm), _i(pv))
        LU[b] = cm.reshape(n, n, order="F")
        piv[b] = pv
    return LU, piv, info


def lu_solve_f32(LU, piv, B):
    LU = np.asarray(LU, dtype=np.float32)
    nb, n, _ = LU.shape
    X = np.asarray(B, dtype=np.float32).reshape(nb, n).copy()
    for b in range(nb):
        cm = LU[b].ravel(order="F").copy()
        pv = np.ascontiguousarray(piv[b], dtype=np.int32)
        xb = X[b].copy()
        lib().orc_lu_solve_f32(n, _f(cm), _i(pv), _f(xb))
        X[b] = xb
    return X


def refine_solve(M, B, max_it=5):
    """FP32 LU + FP64 refinement with per-block FP64 fallback.
    Returns (X, status (0 converged / 1 fell back), sweeps)."""
    M = np.asarray(M, dtype=np.float64)
    nb, n, _ = M.shape
    LU32, piv32, info = lu_factor_f32(M.astype(np.float32))
    X = np.zeros((nb, n))
    status = np.zeros(nb, dtype=np.int32)
    sweeps = np.zeros(nb, dtype=np.int32)
    Bv = _c64(B).reshape(nb, n)
    for b in range(nb):
        cm = M[b].ravel(order="F").copy()
        lu = LU32[b].ravel(order="F").astype(np.float32).copy()
        pv = np.ascontiguousarray(piv32[b], dtype=np.int32)
        bb = Bv[b].copy()
        xb = np.zeros(n)
        sw = C.c_int(0)
        if info[b]:
            st = 1
        else:
            st = lib().orc_lu_refine_solve(n, _d(cm), _f(lu), _i(pv), _d(bb), _d(xb),
                                           max_it, C.byref(sw))
        if st:
            LU, pv64, inf64 = lu_factor(M[b:b + 1])
            xb = lu_solve(LU, pv64, bb[None])[0]
        X[b] = xb
        status[b] = st
        sweeps[b] = sw.value
    return X, status, sweeps


# ----------------------------------------------------------------------------
# Mass action
# ----------------------------------------------------------------------------

def ma_rhs(nu, mu, kappa, y):
    nu = np.ascontiguousarray(nu, dtype=np.int32)
    mu = np.ascontiguousarray(mu, dtype=np.int32)
    R, n = nu.shape
    kappa, y = _c64(kappa), _c64(y)
    f = np.empty(n)
    lib().orc_ma_rhs(n, R, _i(nu), _i(mu), _d(kappa), _d(y), _d(f))
    return f


def ma_jac(nu, mu, kappa, y):
    nu = np.ascontiguousarray(nu, dtype=np.int32)
    mu = np.ascontiguousarray(mu, dtype=np.int32)
    R, n = nu.shape
    kappa, y = _c64(kappa), _c64(y)
    J = np.empty(n * n)
    lib().orc_ma_jac(n, R, _i(nu), _i(mu), _d(kappa), _d(y), _d(J))
    return J.reshape(n, n, order="F")


# ----------------------------------------------------------------------------
# MLP
# ----------------------------------------------------------------------------

def bf16_round(x):
    return lib().orc_bf16_round(float(x))


def set_bf16(on: bool):
    lib().orc_set_bf16(1 if on else 0)


class MLP:
    """FP32 master weights + input standardisation for the oracle MLP."""

    def __init__(self, W1, b1, W2, b2, W3, b3, in_mean, in_std):
        self.W1 = np.ascontiguousarray(W1, np.float32)
        self.b1 = np.ascontiguousarray(b1, np.float32)
        self.W2 = np.ascontiguousarray(W2, np.float32)
        self.b2 = np.ascontiguousarray(b2, np.float32)
        self.W3 = np.ascontiguousarray(W3, np.float32)
        self.b3 = np.ascontiguousarray(b3, np.float32)
        self.in_mean = _c64(in_mean)
        self.in_std = _c64(in_std)
        self.s = OrcMLP(self.W1.shape[1], self.W1.shape[0], self.W3.shape[0],
                        _f(self.W1), _f(self.b1), _f(self.W2), _f(self.b2),
                        _f(self.W3), _f(self.b3), _d(self.in_mean), _d(self.in_std))

    def forward(self, x_raw):
        x_raw = np.atleast_2d(_c64(x_raw))
        out = np.empty((x_raw.shape[0], self.s.nout))
        for b in range(x_raw.shape[0]):
            xb = x_raw[b].copy()
            ob = np.empty(self.s.nout)
            lib().orc_mlp_forward(C.byref(self.s), _d(xb), _d(ob))
            out[b] = ob
        return out

    def loss_grad(self, X_raw, Mb):
        """Mb: (B, n, n) mathematical order."""
        X_raw = _c64(X_raw)
        B = X_raw.shape[0]
        Mc = np.stack([np.asarray(m).ravel(order="F") for m in Mb]).astype(np.float64)
        Mc = np.ascontiguousarray(Mc)
        g = [np.zeros(a.shape) for a in (self.W1, self.b1, self.W2, self.b2, self.W3, self.b3)]
        L = lib().orc_mlp_loss_grad(C.byref(self.s), B, _d(X_raw), _d(Mc),
                                    *[_d(x) for x in g])
        return L, g


def adam_step(p, g, m1, m2, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In place on float32 p and float64 m1, m2."""
    lib().orc_adam_step(p.size, _f(p), _d(_c64(g)), _d(m1), _d(m2), t, lr, b1, b2, eps)


# ----------------------------------------------------------------------------
# BDF integrator
# ----------------------------------------------------------------------------

LS_LU64, LS_LU32REF, LS_LEARNED, LS_GJ, LS_GMRES = 0, 1, 2, 3, 4


def gmres_solve(Ms, Ps, w, r, tol):
    """The Newton-Krylov GMRES on blocks Ms (list of n x n) preconditioned
    by the LU factors of the blocks Ps; returns (del, iterations)."""
    ns = np.array([m.shape[0] for m in Ms], np.int32)
    M = np.concatenate([np.asarray(m, float).T.ravel() for m in Ms])
    LUs, pivs = [], []
    for P in Ps:
        lu, pv, _ = lu_factor(np.asarray(P, float)[None])
        LUs.append(lu[0].T.ravel())
        pivs.append(pv[0])
    LU = np.concatenate(LUs)
    piv = np.concatenate(pivs).astype(np.int32)
    w, r = _c64(w), _c64(r)
    d = np.zeros_like(r)
    it = lib().orc_gmres_solve(len(ns), _i(ns), _d(M), _d(LU), _i(piv), _d(w), _d(r), tol, _d(d))
    return d, it


def bdf_coeffs(q):
    l = np.zeros(q + 1)
    tq = C.c_double(0.0)
    lib().orc_bdf_coeffs(q, _d(l), C.byref(tq))
    return l, tq.value


class Bdf:
    """Oracle integrator over a workloads.Problem."""

    def __init__(self, prob, rtol=None, atol=None, qmax=None, maxcor=3, h0=0.0,
                 linsol=LS_LU64, refine_max_it=5, max_steps=0, hmin=0.0,
                 mlp: MLP | None = None, nonneg=None, fixed_step=False, vc=False,
                 lazy=False):
        self._keep = []
        topo_n = np.array([nu.shape[1] for nu, _ in prob.topologies], np.int32)
        topo_R = np.array([nu.shape[0] for nu, _ in prob.topologies], np.int32)
        sizes = topo_n * topo_R
        topo_off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int32)
        nu_all = np.concatenate([np.ascontiguousarray(nu, np.int32).ravel()
                                 for nu, _ in prob.topologies]).astype(np.int32)
        mu_all = np.concatenate([np.ascontiguousarray(mu, np.int32).ravel()
                                 for _, mu in prob.topologies]).astype(np.int32)
        cell_topo = np.ascontiguousarray(prob.cell_topo, np.int32)
        rates = _c64(prob.rates)
        y0 = _c64(prob.y0)
        self._keep += [topo_n, topo_R, topo_off, nu_all, mu_all, cell_topo, rates, y0]
        self.prob = OrcProblem(len(topo_n), _i(topo_n), _i(topo_R), _i(topo_off),
                               _i(nu_all), _i(mu_all), len(cell_topo), _i(cell_topo),
                               _d(rates), _d(y0), float(prob.t0))
        self.mlp = mlp
        self.opts = OrcOptions(prob.rtol if rtol is None else rtol,
                               prob.atol if atol is None else atol,
                               prob.qmax if qmax is None else qmax, maxcor, h0,
                               linsol, refine_max_it, max_steps, hmin,
                               C.pointer(mlp.s) if mlp is not None else None,
                               int(prob.get("nonneg", False) if nonneg is None else nonneg),
                               int(bool(fixed_step)), int(bool(vc)), int(bool(lazy)))
        self.h = lib().orc_bdf_create(C.byref(self.prob), C.byref(self.opts))
        if not self.h:
            raise ValueError("orc_bdf_create refused the options (lazy needs LU64, GJ or GMRES)")
        self.N = lib().orc_bdf_N(self.h)

    def __del__(self):
        try:
            if self.h:
                lib().orc_bdf_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def step(self, t_end):
        return lib().orc_bdf_step(self.h, t_end)

    def integrate(self, t_end):
        return lib().orc_bdf_integrate(self.h, t_end)

    def init(self, t_end):
        """Starting step and history, as the first step computes them."""
        lib().orc_bdf_init(self.h, t_end)

    def y(self):
        y = np.empty(self.N)
        lib().orc_bdf_get_y(self.h, _d(y))
        return y

    def stats(self):
        s = OrcStats()
        lib().orc_bdf_get_stats(self.h, C.byref(s))
        return s.as_dict()

    def scalars(self):
        s = OrcScalars()
        lib().orc_bdf_get_scalars(self.h, C.byref(s))
        return {k: getattr(s, k) for k, _ in s._fields_}

    def set_scalars(self, d):
        s = OrcScalars(**d)
        lib().orc_bdf_set_scalars(self.h, C.byref(s))

    def history(self):
        z = np.empty(6 * self.N)
        dp_ = np.empty(self.N)
        lib().orc_bdf_get_history(self.h, _d(z), _d(dp_))
        return z.reshape(6, self.N), dp_

    def past_steps(self):
        """(accepted step sizes, most recent first; scale and step of the
        saved correction) of the variable-coefficient form."""
        tau = np.zeros(6)
        c, h = C.c_double(), C.c_double()
        k = lib().orc_bdf_get_past_steps(self.h, _d(tau), C.byref(c), C.byref(h))
        return tau[:k].copy(), c.value, h.value

    def set_past_steps(self, tau, dprev_c=1.0, dprev_h=1.0):
        tau = _c64(tau)
        lib().orc_bdf_set_past_steps(self.h, len(tau), _d(tau) if len(tau) else None,
                                     dprev_c, dprev_h)

    def lazy_state(self):
        g, c = C.c_double(), C.c_double()
        n = C.c_long()
        lib().orc_bdf_get_lazy(self.h, C.byref(g), C.byref(n), C.byref(c))
        return {"gamma_s": g.value, "nst_s": n.value, "crate": c.value}

    def set_history(self, z, dprev):
        z = _c64(z).reshape(-1)
        dprev = _c64(dprev)
        lib().orc_bdf_set_history(self.h, _d(z), _d(dprev))
