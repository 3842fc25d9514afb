"""Pins for the oracle's Newton-Krylov solve (linsol GMRES).

The paper's demonstration offers a global Newton iteration whose linear
systems GMRES solves with the task-local block solver as preconditioner
(Section 7; Krylov solvers, Section 5).  The oracle solves each Newton
system with right-preconditioned GMRES scaled by the error weights, the
block-Jacobi preconditioner being the cells' LU factors at the last setup.
Pinned against independent facts:

 * with a preconditioner from another gamma and a tight tolerance the
   GMRES correction equals numpy's direct solution of the block system,
   and with the integrator's tolerance its scaled residual meets it;
 * GMRES converges in as many iterations as the preconditioned operator
   has distinct eigenvalues: one when the preconditioner is the matrix
   itself (or a scalar multiple), one per distinct decay rate for decay
   cells with a stale preconditioner;
 * a whole integration with a fresh preconditioner takes one Krylov
   iteration per solve and ends where the direct solve ends; with the lazy
   preconditioner it ends as accurate against a tight-tolerance run.
The Krylov dimension (5), the tolerance factor (0.05 of the Newton
tolerance) and classical Gram-Schmidt are readings, parity-unpinned.
"""
import math

import numpy as np
import pytest

import workloads as W

LS_GMRES = 4


@pytest.mark.parametrize("n,ncells", [(3, 40), (4, 25), (5, 9)])
def test_gmres_with_a_stale_preconditioner_is_exact_in_n_iterations(orc, n, ncells):
    """Every cell has the same Jacobian J (n distinct eigenvalues) and the
    preconditioner is the block of another gamma: the preconditioned
    operator (I - g J)(I - g_s J)^{-1} has the n eigenvalues
    (1 - g lam)/(1 - g_s lam), so GMRES is exact after n iterations and
    equals numpy's direct solve; with the integrator's loose tolerance the
    scaled residual meets it."""
    rng = W.rng_for(1800 + n)
    J = rng.uniform(-1.0, 1.0, (n, n)) * 50.0 - np.eye(n) * 50.0 * n
    g, gs = 0.02, 0.016
    Ms = [np.eye(n) - g * J] * ncells
    Ps = [np.eye(n) - gs * J] * ncells
    N = n * ncells
    w = 10.0 ** rng.uniform(2, 6, N)
    r = rng.uniform(-1.0, 1.0, N) / w
    tol = 1e-11 * np.linalg.norm(w * r)
    d, it = orc.gmres_solve(Ms, Ps, w, r, tol)
    exact = np.concatenate([np.linalg.solve(Ms[c], r[c * n:(c + 1) * n]) for c in range(ncells)])
    res = np.concatenate([Ms[c] @ d[c * n:(c + 1) * n] for c in range(ncells)])
    print(n, ncells, "iterations", it)
    assert it == n
    assert np.allclose(d, exact, rtol=1e-8, atol=1e-9 * np.abs(exact).max())
    assert np.linalg.norm(w * (r - res)) <= 10 * tol
    tol2 = 0.005 * math.sqrt(N)
    d2, it2 = orc.gmres_solve(Ms, Ps, w, r * 1e3, tol2)
    res2 = np.concatenate([Ms[c] @ d2[c * n:(c + 1) * n] for c in range(ncells)])
    assert 1 <= it2 <= n
    assert np.linalg.norm(w * (r * 1e3 - res2)) <= tol2 * (1 + 1e-9)


@pytest.mark.parametrize("rates", [[40.0] * 6, [3.0, 3.0, 70.0, 70.0, 900.0, 900.0],
                                   [1.0, 8.0, 60.0, 500.0]])
def test_iterations_equal_distinct_eigenvalues(orc, rates):
    """Scalar decay cells: M = 1 + gamma kappa, preconditioner 1 + gamma_s
    kappa, so the preconditioned operator is diagonal with one eigenvalue
    per distinct rate, and GMRES is exact after that many iterations."""
    kap = np.array(rates)
    g, gs = 0.013, 0.011
    Ms = [np.array([[1.0 + g * k]]) for k in kap]
    Ps = [np.array([[1.0 + gs * k]]) for k in kap]
    w = np.ones(kap.size)
    r = np.linspace(1.0, 2.0, kap.size)
    d, it = orc.gmres_solve(Ms, Ps, w, r, 1e-13)
    assert it == len(set(rates))
    assert np.allclose(d, r / (1.0 + g * kap), rtol=1e-11)
    # the matrix itself as preconditioner: one iteration
    d1, it1 = orc.gmres_solve(Ms, Ms, w, r, 1e-13)
    assert it1 == 1 and np.allclose(d1, r / (1.0 + g * kap), rtol=1e-13)


def test_fresh_preconditioner_run_matches_direct(orc):
    """Without lazy reuse the preconditioner is M itself at every attempt,
    so each Krylov solve that starts above the tolerance takes one iteration
    and the run ends where the direct solve's run ends."""
    p = W.random_network_batch(16, n=10, seed=1701, t_end=1e-3)
    b = orc.Bdf(p, linsol=LS_GMRES)
    a = orc.Bdf(p)
    assert b.integrate(p.t_end) == 0 and a.integrate(p.t_end) == 0
    sb, sa = b.stats(), a.stats()
    assert 0 < sb["nliters"] <= sb["nniters"]
    w = 1.0 / (p.rtol * np.abs(a.y()) + p.atol)
    d = math.sqrt(np.mean(((b.y() - a.y()) * w) ** 2))
    print("GMRES(P = M) vs LU:", sb["nsteps"], sa["nsteps"], f"wrms {d:.2e}")
    assert d <= 1.0


def test_lazy_krylov_run_is_as_accurate(orc):
    p = W.random_network_batch(32, n=10, seed=1601, t_end=1.0)
    ref = orc.Bdf(p, rtol=p.rtol * 1e-3, atol=p.atol * 1e-3)
    assert ref.integrate(p.t_end) == 0
    yr = ref.y()

    def err(y):
        w = 1.0 / (p.rtol * np.abs(yr) + p.atol)
        return math.sqrt(np.mean(((y - yr) * w) ** 2))

    a = orc.Bdf(p)
    k = orc.Bdf(p, linsol=LS_GMRES, lazy=True)
    assert a.integrate(p.t_end) == 0 and k.integrate(p.t_end) == 0
    ea, ek = err(a.y()), err(k.y())
    sa, sk = a.stats(), k.stats()
    print(f"LU error {ea:.3e}, {sa['nsetups']} setups; Krylov + lazy error {ek:.3e}, "
          f"{sk['nsetups']} setups, {sk['nliters']} Krylov iterations over {sk['nniters']} "
          f"Newton iterations")
    assert ek <= 3.0 * ea + 1.0
    assert sk["nsetups"] * 3 < sa["nsetups"]
    assert sk["nliters"] > sk["nniters"] // 2
