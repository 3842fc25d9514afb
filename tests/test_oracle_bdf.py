"""Pins for the oracle's grouped BDF integrator.

The paper only names CVODE (Section 1) and gives the grouped Newton with a
block-diagonal solve and whole-step retry (Section 7); the integrator is a
fixed-coefficient Nordsieck BDF of orders 1..5.  Its arithmetic is pinned
here independently of its own formulas:

 * one step from a polynomial history reproduces the textbook BDF_q
   recurrence  sum_{j=1..q} (1/j) nabla^j y_n = h f(y_n)  (pins the l vector);
 * for a solution that is a polynomial of degree q+1 the step's local error
   estimate equals the true one-step error (pins the error constant), and
   lower-degree components are exact;
 * linear systems y' = A y against expm(A t); Robertson against scipy Radau;
 * count conservation of sum(y); grouping identical cells.
The step-size and order heuristics' constants are readings, not pinned.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import workloads as W


def one_cell_problem(nu, mu, rates, y0, ncells=1, rtol=1.0, atol=1.0, qmax=5):
    nu = np.asarray(nu, np.int32)
    mu = np.asarray(mu, np.int32)
    return W.Problem(topologies=[(nu, mu)], cell_topo=np.zeros(ncells, np.int32),
                     rates=np.asarray(rates, float).ravel().copy(),
                     y0=np.asarray(y0, float).ravel().copy(), rtol=rtol, atol=atol,
                     t0=0.0, t_end=1e9, qmax=qmax, label="pin")


def set_state(b, z, q, h, t=0.0, qwait=50):
    N = b.N
    z6 = np.zeros((6, N))
    z6[: len(z)] = z
    b.set_history(z6, np.zeros(N))
    b.set_scalars(dict(t=t, h=h, err_last=0.0, q=q, qwait=qwait,
                       qprime_pending=0, initialized=1, hu=h, qu=q))


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5])
def test_step_is_textbook_bdf_recurrence(orc, q):
    rng = W.rng_for(200 + q)
    ncells = 6
    kap = rng.uniform(0.5, 50.0, ncells)
    # A -> 0 : y' = -kappa y, one species per cell
    p = one_cell_problem([[1]], [[0]], kap, np.ones(ncells), ncells=ncells,
                         rtol=1e3, atol=1e3)
    b = orc.Bdf(p, qmax=5)
    h = 0.07
    z = rng.uniform(-0.5, 0.5, (q + 1, ncells))
    z[0] += 2.0
    set_state(b, z, q, h)
    assert b.step(1e9) == 0
    yn = b.history()[0][0]
    # past values of the history polynomial p(s) = sum_k z_k s^k at s = -j
    past = np.array([sum(z[k] * (-j) ** k for k in range(q + 1)) for j in range(q)])
    seq = np.vstack([yn[None], past])          # y_n, y_{n-1}, ..., y_{n-q}
    lhs = np.zeros(ncells)
    d = seq.copy()
    for j in range(1, q + 1):
        d = d[:-1] - d[1:]                     # nabla^j y_n is d[0]
        lhs += d[0] / j
    rhs = h * (-kap * yn)
    assert np.allclose(lhs, rhs, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5])
def test_error_estimate_exact_for_degree_q_plus_1(orc, q):
    """Catalytic chain 0 -> X0, X_{k-1} -> X_{k-1} + X_k has polynomial
    solutions: X_k has degree k+1.  With species up to degree q+1 and an
    interpolating history, species of degree <= q are reproduced exactly and
    the step's error estimate equals the true error of the top species."""
    m = q + 1
    nu = np.zeros((m, m), np.int32)
    mu = np.zeros((m, m), np.int32)
    mu[0, 0] = 1
    for k in range(1, m):
        nu[k, k - 1] = 1
        mu[k, k - 1] = 1
        mu[k, k] = 1
    rng = W.rng_for(300 + q)
    c = rng.uniform(0.2, 1.0, m)
    P = np.polynomial.Polynomial
    sols = [P([c[0], 1.0])]
    for k in range(1, m):
        sols.append(P([c[k]]) + sols[-1].integ())
    t1, h = 1.0, 0.05
    p = one_cell_problem(nu, mu, np.ones(m), np.zeros(m), rtol=1.0, atol=1.0)
    b = orc.Bdf(p, qmax=5)
    # interpolating history through t1, t1 - h, ..., t1 - q h
    V = np.array([[(-j) ** k for k in range(q + 1)] for j in range(q + 1)], float)
    vals = np.array([[s(t1 - j * h) for s in sols] for j in range(q + 1)])
    z = np.linalg.solve(V, vals)
    set_state(b, z, q, h, t=t1)
    assert b.step(1e9) == 0
    yn = b.history()[0][0]
    yex = np.array([s(t1 + h) for s in sols])
    err = yn - yex
    assert np.abs(err[:-1]).max() <= 1e-12
    assert abs(err[-1]) > 1e-12
    yprev = vals[0]
    w = 1.0 / (np.abs(yprev) + 1.0)
    true_wrms = math.sqrt(np.mean((err * w) ** 2))
    assert b.scalars()["err_last"] == pytest.approx(true_wrms, rel=1e-7)


def test_linear_chain_against_expm(orc):
    n, ncells = 5, 8
    p = W.linear_chain_batch(ncells, n, seed=41)
    nu, mu = p.topologies[0]
    errs = {}
    for rtol in (1e-4, 1e-6, 1e-8):
        b = orc.Bdf(p, rtol=rtol, atol=rtol * 1e-4)
        assert b.integrate(p.t_end) == 0
        y = b.y().reshape(ncells, n)
        e = []
        for c in range(ncells):
            A = orc.ma_jac(nu, mu, p.rates[c * n:(c + 1) * n], np.zeros(n))
            ye = sl.expm(A * p.t_end) @ p.y0[c * n:(c + 1) * n]
            w = 1.0 / (rtol * np.abs(ye) + rtol * 1e-4)
            e.append(np.sqrt(np.mean(((y[c] - ye) * w) ** 2)))
        errs[rtol] = max(e)
    # global error within a modest multiple of the tolerance ...
    assert errs[1e-6] <= 10.0
    # ... and the absolute error falls as the tolerance tightens
    assert errs[1e-8] * 1e-8 < errs[1e-6] * 1e-6 < errs[1e-4] * 1e-4


def test_robertson_against_radau(orc):
    from scipy.integrate import solve_ivp
    nu, mu = W.robertson_topology()
    k = W.ROBERTSON_RATES
    p = one_cell_problem(nu, mu, k, [1.0, 0.0, 0.0], rtol=1e-8, atol=1e-12)
    b = orc.Bdf(p)
    assert b.integrate(40.0) == 0
    ref = solve_ivp(lambda t, y: orc.ma_rhs(nu, mu, k, y), (0, 40), [1.0, 0.0, 0.0],
                    method="Radau", rtol=1e-12, atol=1e-16,
                    jac=lambda t, y: orc.ma_jac(nu, mu, k, y)).y[:, -1]
    y = b.y()
    assert np.allclose(y, ref, rtol=2e-6, atol=1e-12)
    assert b.scalars()["t"] == 40.0


def test_conservation_and_exact_end_time(orc):
    # the method itself (no projection) keeps sum(y) to rounding
    p = W.random_network_batch(16, n=10, seed=77)
    b = orc.Bdf(p, nonneg=False)
    assert b.integrate(p.t_end) == 0
    y = b.y().reshape(16, 10)
    y0 = p.y0.reshape(16, 10)
    assert np.abs(y.sum(1) - y0.sum(1)).max() <= 1e-12
    assert b.scalars()["t"] == p.t_end
    st = b.stats()
    assert st["nsteps"] == sum(st["order_hist"])
    assert st["nattempts"] == st["nsteps"] + st["netfails"] + st["nncfails"]


def test_grouping_identical_cells(orc):
    one = W.random_network_batch(1, n=10, seed=5)
    many = W.Problem(dict(one))
    many["cell_topo"] = np.zeros(4, np.int32)
    many["rates"] = np.tile(one.rates, 4)
    many["y0"] = np.tile(one.y0, 4)
    b1, b4 = orc.Bdf(one), orc.Bdf(many)
    assert b1.integrate(one.t_end) == 0 and b4.integrate(one.t_end) == 0
    assert b1.stats()["nsteps"] == b4.stats()["nsteps"]
    assert np.allclose(b4.y().reshape(4, 10), b1.y()[None], rtol=1e-12, atol=1e-15)


def test_fp32_refined_matches_fp64(orc):
    p = W.random_network_batch(32, n=10, seed=90)
    b64 = orc.Bdf(p)
    b32 = orc.Bdf(p, linsol=orc.LS_LU32REF)
    assert b64.integrate(p.t_end) == 0 and b32.integrate(p.t_end) == 0
    s64, s32 = b64.stats(), b32.stats()
    assert abs(s64["nsteps"] - s32["nsteps"]) <= max(2, s64["nsteps"] // 50)
    w = 1.0 / (p.rtol * np.abs(b64.y()) + p.atol)
    assert np.sqrt(np.mean(((b32.y() - b64.y()) * w) ** 2)) <= 1.0


def test_learned_identity_network_falls_back_to_lu(orc):
    """An MLP whose output is zero gives X = I (plain fixed-point form);
    on a stiff problem the per-cell test must move cells to exact LU and the
    result must agree with the LU integrator."""
    n = 6
    p = W.random_network_batch(8, n=n, seed=12, shared_rates=True)
    hid = 16
    nin, nout = n + 1, n * n
    z = np.zeros
    mlp = orc.MLP(z((hid, nin)), z(hid), z((hid, hid)), z(hid), z((nout, hid)), z(nout),
                  z(nin), np.ones(nin))
    bl = orc.Bdf(p, linsol=orc.LS_LEARNED, mlp=mlp, nonneg=False)
    b64 = orc.Bdf(p, nonneg=False)
    bref = orc.Bdf(p, rtol=1e-10, atol=1e-14, nonneg=False)
    for b in (bl, b64, bref):
        assert b.integrate(p.t_end) == 0
    st = bl.stats()
    assert st["lp_fallback_cells"] > 0 or st["lp_step_fallbacks"] > 0
    # two valid step sequences differ by about the global error: compare both
    # against a tight-tolerance run, in units of the requested tolerance
    ref = bref.y()
    w = 1.0 / (p.rtol * np.abs(ref) + p.atol)
    for b in (bl, b64):
        assert np.sqrt(np.mean(((b.y() - ref) * w) ** 2)) <= 10.0


def test_learned_underestimating_inverse_keeps_every_cell_accurate(orc):
    """X = 0.2 I underestimates M^{-1} for the non-stiff species: its
    corrections are small, so the grouped Newton test alone could accept
    an attempt after one iteration with cells far from the Newton solution.
    The guard (no acceptance at the first iteration; a cell that does not
    contract by 0.9 moves to LU and blocks acceptance at that iteration)
    keeps every cell within 3x (+1 WRMS) of the LU run's error against a
    tight-tolerance run."""
    n = 6
    p = W.random_network_batch(16, n=n, seed=13, shared_rates=True, t_end=1e-3)
    hid = 16
    nin, nout = n + 1, n * n
    z = np.zeros
    b3 = z(nout)
    b3[:: n + 1] = 0.2 - 1.0            # X = I + diag(b3) = 0.2 I
    mlp = orc.MLP(z((hid, nin)), z(hid), z((hid, hid)), z(hid), z((nout, hid)), b3,
                  z(nin), np.ones(nin))
    bl = orc.Bdf(p, linsol=orc.LS_LEARNED, mlp=mlp, nonneg=False)
    b64 = orc.Bdf(p, nonneg=False)
    bref = orc.Bdf(p, rtol=p.rtol * 1e-3, atol=p.atol * 1e-3, nonneg=False)
    for b in (bl, b64, bref):
        assert b.integrate(p.t_end) == 0
    st = bl.stats()
    assert st["lp_unconverged"] > st["nattempts"] // 2
    ref = bref.y()
    w = 1.0 / (p.rtol * np.abs(ref) + p.atol)
    cell = lambda y: np.sqrt(np.mean((((y - ref) * w) ** 2).reshape(-1, n), 1))
    el, e64 = cell(bl.y()), cell(b64.y())
    print(f"per-cell error vs tight run: learned max {el.max():.3e} median {np.median(el):.3e}; "
          f"LU max {e64.max():.3e}; {st['lp_unconverged']} unconverged-cell events, "
          f"{st['lp_fallback_cells']} LU switches, {st['lp_step_fallbacks']} LU retries")
    assert el.max() <= 3.0 * e64.max() + 1.0
    # one step from the same state: every cell's accepted value is the
    # Newton solution the LU step reaches, to a fraction of the tolerance
    b64 = orc.Bdf(p, nonneg=False)
    for _ in range(25):
        assert b64.step(p.t_end) == 0
    sc = b64.scalars()
    z6, dprev = b64.history()
    bl = orc.Bdf(p, linsol=orc.LS_LEARNED, mlp=mlp, nonneg=False)
    for b in (b64, bl):
        b.set_history(z6, dprev)
        b.set_scalars(sc)
        assert b.step(p.t_end) == 0
    assert bl.scalars()["t"] == b64.scalars()["t"]
    w = 1.0 / (p.rtol * np.abs(z6[0]) + p.atol)
    dc = np.sqrt(np.mean((((bl.y() - b64.y()) * w) ** 2).reshape(-1, n), 1))
    print(f"one step: per-cell difference learned vs LU max {dc.max():.3e}")
    assert dc.max() <= 0.5


def test_tstop_and_max_steps(orc):
    p = W.robertson_batch(4)
    b = orc.Bdf(p, max_steps=5)
    assert b.integrate(10.0) == -6
    b = orc.Bdf(p)
    assert b.integrate(1e-3) == 0 and b.scalars()["t"] == 1e-3
    assert b.integrate(2e-3) == 0 and b.scalars()["t"] == 2e-3


def test_nonnegativity_projection(orc):
    """With the y >= 0 projection every accepted solution is non-negative, the
    projected mass stays at the absolute-tolerance level, and the run agrees
    with the unprojected one within the tolerance."""
    p = W.random_network_batch(64, n=10, seed=77)
    bp = orc.Bdf(p, nonneg=True)
    bu = orc.Bdf(p, nonneg=False)
    assert bp.integrate(p.t_end) == 0 and bu.integrate(p.t_end) == 0
    y = bp.y()
    assert y.min() >= 0.0
    assert bp.stats()["nprojections"] > 0
    drift = np.abs(y.reshape(64, 10).sum(1) - p.y0.reshape(64, 10).sum(1)).max()
    assert drift <= 1e3 * p.atol
    w = 1.0 / (p.rtol * np.abs(bu.y()) + p.atol)
    assert np.sqrt(np.mean(((y - bu.y()) * w) ** 2)) <= 10.0


def test_bimolecular_blowup_closed_form(orc):
    """2A -> 2B with A < 0: dA/dt = -2 k A^2 has the closed form
    A(t) = A0 / (1 + 2 k A0 t), which runs away to -infinity at
    t* = 1 / (2 k |A0|).  The unprojected integrator follows the closed
    form before t* and cannot pass it; this is why mass-action workloads use
    the y >= 0 projection."""
    nu = np.array([[2, 0]], np.int32)
    mu = np.array([[0, 2]], np.int32)
    k, A0 = 1e8, -1e-9
    tstar = 1.0 / (2 * k * abs(A0))
    p = one_cell_problem(nu, mu, [k], [A0, 1.0], rtol=1e-8, atol=1e-14)
    b = orc.Bdf(p, nonneg=False)
    assert b.integrate(0.5 * tstar) == 0
    exact = A0 / (1 + 2 * k * A0 * 0.5 * tstar)
    assert b.y()[0] == pytest.approx(exact, rel=1e-5)
    assert b.y().sum() == pytest.approx(1.0 + A0, rel=1e-12)
    b2 = orc.Bdf(p, nonneg=False, max_steps=3000)
    st = b2.integrate(2 * tstar)
    assert st != 0 and abs(b2.y()[0]) > 1e3 * abs(A0)
