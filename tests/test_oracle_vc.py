"""Pins for the oracle's variable-coefficient BDF and lazy Newton matrix.

The paper names CVODE (Section 1), whose BDF takes its coefficients from
the actual step sizes.  The variable-coefficient option (vc) reads that as
the BDF formula on the actual past grid, carried in Nordsieck form, and
derives every constant from one model: the history is the polynomial
through the last q + 1 accepted values.  Each part is pinned against an
independent computation (Lagrange polynomials on the irregular grid, exact
polynomial solutions), never against its own formula:

 * one step from an arbitrary history is the variable-step BDF_q formula
   through the history's values at the actual past times (pins l);
 * for a degree-(q+1) solution with an exact interpolating history on an
   irregular grid, the error estimate is the true one-step error (pins the
   error constant), and D = c acor is h^{q+1} y^{(q+1)} / (q+1)! (pins the
   scale of the order-(q+1) estimate);
 * err_{q-1} is the true error of the variable-step order-(q-1) step;
 * along a whole integration with step-size changes, order raises and
   lowerings and error-test failures, the history interpolates the last
   q + 1 accepted values after every step (pins the past-step bookkeeping
   and the order-change adjustments); the fixed-coefficient form does not;
 * at constant steps the form reduces to the fixed-coefficient one.

Lazy Newton matrix: on a linear problem at a fixed step the stored factors
are the fresh ones, so the lazy run equals the eager run and sets up every
20 steps.  Its reuse rules (20 steps, |gamma ratio - 1| <= 0.3, the
2 / (1 + gamma ratio) scaling, the carried convergence rate) are readings
and parity-unpinned.
"""
import math

import numpy as np
import pytest

import workloads as W
from test_oracle_bdf_order import chain, chain_solutions, problem

P = np.polynomial.Polynomial


def set_state(b, z, dprev, q, h, t, qwait, tau, dprev_c=1.0, dprev_h=1.0):
    N = b.N
    z6 = np.zeros((6, N))
    z6[: len(z)] = z
    b.set_history(z6, dprev)
    b.set_scalars(dict(t=t, h=h, err_last=0.0, q=q, qwait=qwait, qprime_pending=0,
                       initialized=1, hu=h, qu=q, err_qm1=-1.0, err_qp1=-1.0,
                       eta_proposed=1.0, q_proposed=q))
    b.set_past_steps(tau, dprev_c, dprev_h)


def past_times(t1, tau, k):
    """t1 and the k - 1 accepted points before it (tau: most recent step
    first)."""
    ts = [t1]
    for i in range(k - 1):
        ts.append(ts[-1] - tau[i])
    return np.array(ts)


def history_through(sols, ts, t1, h, q):
    """Nordsieck vector z[0..q] (units of h around t1) of the degree-q
    polynomial through the exact values at the q + 1 times ts."""
    s = (ts - t1) / h
    V = np.array([[sj ** k for k in range(q + 1)] for sj in s])
    vals = np.array([[f(t) for f in sols] for t in ts])
    return np.linalg.solve(V, vals)


def lagrange_deriv_at(ts, x):
    """d/dt of every Lagrange basis polynomial of the nodes ts, at x."""
    out = []
    for j, tj in enumerate(ts):
        others = [tm for m, tm in enumerate(ts) if m != j]
        num = P.fromroots(others)
        out.append(num.deriv()(x) / num(tj))
    return np.array(out)


def vs_bdf_value(k, ts_past, y_past, tn, fn_lin=None, g=None):
    """y_n of the variable-step BDF_k: the polynomial through (tn, y_n) and
    the k past points has slope f(tn, y_n) at tn; f = -kappa y (fn_lin =
    kappa) or f = g(t)."""
    d = lagrange_deriv_at(np.concatenate([[tn], ts_past[:k]]), tn)
    rest = sum(d[j + 1] * y_past[j] for j in range(k))
    if fn_lin is not None:
        return -rest / (d[0] + fn_lin)
    return (g - rest) / d[0]


def irregular_steps(rng, h, k):
    return h * rng.uniform(0.3, 3.0, k)


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5])
def test_vc_step_is_variable_step_bdf(orc, q):
    rng = W.rng_for(1200 + q)
    ncells = 6
    kap = rng.uniform(0.5, 50.0, ncells)
    nu, mu = np.array([[1]], np.int32), np.array([[0]], np.int32)
    p = W.Problem(topologies=[(nu, mu)], cell_topo=np.zeros(ncells, np.int32), rates=kap,
                  y0=np.ones(ncells), rtol=1e3, atol=1e3, t0=0.0, t_end=1e9, qmax=5,
                  label="pin")
    b = orc.Bdf(p, qmax=5, vc=True)
    h = 0.07
    tau = irregular_steps(rng, h, 6)
    z = rng.uniform(-0.5, 0.5, (q + 1, ncells))
    z[0] += 2.0
    set_state(b, z, np.zeros(ncells), q, h, 0.0, 50, tau)
    assert b.step(1e9) == 0
    yn = b.history()[0][0]
    ts = past_times(0.0, tau, q)                    # t_{n-1}, ..., t_{n-q}
    s = ts / h
    y_past = np.array([sum(z[k] * sj ** k for k in range(q + 1)) for sj in s])
    expect = np.array([vs_bdf_value(q, ts, y_past[:, c], h, fn_lin=kap[c])
                       for c in range(ncells)])
    assert np.allclose(yn, expect, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5])
def test_vc_error_estimate_exact_on_irregular_grid(orc, q):
    m = q + 1                                        # top species of degree q+1
    rng = W.rng_for(1300 + q)
    sols = chain_solutions(m, rng.uniform(0.2, 1.0, m))
    nu, mu = chain(m)
    t1, h = 1.0, 0.05
    tau = irregular_steps(rng, h, 6)
    b = orc.Bdf(problem(nu, mu, np.zeros(m)), qmax=5, vc=True)
    ts = past_times(t1, tau, q + 1)
    set_state(b, history_through(sols, ts, t1, h, q), np.zeros(m), q, h, t1, 50, tau)
    assert b.step(1e9) == 0
    yn = b.history()[0][0]
    yex = np.array([f(t1 + h) for f in sols])
    err = yn - yex
    assert np.abs(err[:-1]).max() <= 1e-12
    assert abs(err[-1]) > 1e-10
    w = 1.0 / (np.abs([f(t1) for f in sols]) + 1.0)
    true = math.sqrt(np.mean((err * w) ** 2))
    assert b.scalars()["err_last"] == pytest.approx(true, rel=1e-7)
    # D = c acor is the Nordsieck top component h^{q+1} y^{(q+1)} / (q+1)!
    _, acor = b.history()
    _, c, hprev = b.past_steps()
    assert hprev == h
    top = sols[-1].coef[q + 1] * h ** (q + 1)
    assert c * acor[-1] == pytest.approx(top, rel=1e-8)


@pytest.mark.parametrize("q", [2, 3, 4, 5])
def test_vc_err_qm1_is_true_error_of_order_q_minus_1_step(orc, q):
    m = q                                            # X_{q-1} has degree q
    rng = W.rng_for(1400 + q)
    sols = chain_solutions(m, rng.uniform(0.2, 1.0, m))
    nu, mu = chain(m)
    t1, h = 1.0, 0.04
    tau = irregular_steps(rng, h, 6)
    b = orc.Bdf(problem(nu, mu, np.zeros(m)), qmax=5, vc=True)
    ts = past_times(t1, tau, q + 1)
    set_state(b, history_through(sols, ts, t1, h, q), np.zeros(m), q, h, t1, 1, tau)
    assert b.step(1e9) == 0
    est = b.scalars()["err_qm1"]
    top, g = sols[-1], sols[-2]
    yn = vs_bdf_value(q - 1, ts, np.array([top(t) for t in ts]), t1 + h, g=g(t1 + h))
    err_top = yn - top(t1 + h)
    w_top = 1.0 / (abs(top(t1)) + 1.0)
    true = math.sqrt(err_top ** 2 * w_top ** 2 / m)
    assert est == pytest.approx(true, rel=1e-8)


def history_poly_error(b, tys, rtol, atol):
    """Largest WRMS difference between the stored history polynomial and
    the last q + 1 accepted values (tys: list of (t, y), newest last)."""
    sc = b.scalars()
    z, _ = b.history()
    q, h, tn = sc["q"], sc["h"], sc["t"]
    worst = 0.0
    for i in range(q + 1):
        t, y = tys[-1 - i]
        s = (t - tn) / h
        v = sum(z[j] * s ** j for j in range(q + 1))
        w = 1.0 / (rtol * np.abs(y) + atol)
        worst = max(worst, math.sqrt(np.mean(((v - y) * w) ** 2)))
    return worst


def run_recording(orc, p, steps, **kw):
    b = orc.Bdf(p, **kw)
    b.init(p.t_end)
    tys = [(p.t0, p.y0.copy())]
    worst = 0.0
    for _ in range(steps):
        assert b.step(p.t_end) == 0
        tys.append((b.scalars()["t"], b.y()))
        if len(tys) > b.scalars()["q"] + 1:
            worst = max(worst, history_poly_error(b, tys, p.rtol, p.atol))
        if b.scalars()["t"] >= p.t_end:
            break
    return b, worst


def test_vc_history_interpolates_last_accepted_values(orc):
    p = W.random_network_batch(8, n=6, seed=1501, t_end=1.0)
    b, worst = run_recording(orc, p, 600, vc=True)
    st = b.stats()
    # the run exercised what the invariant has to survive
    assert st["netfails"] > 0 and st["nsteps"] >= 200
    assert sum(1 for k in st["order_hist"][1:] if k > 0) >= 4
    print(f"vc: {st['nsteps']} steps, orders {st['order_hist']}, error-test failures "
          f"{st['netfails']}; worst interpolation residual {worst:.2e} WRMS")
    assert worst <= 1e-6
    # the fixed-coefficient form does not keep it across step-size changes
    _, worst_fixed = run_recording(orc, p, 600)
    print(f"fixed coefficients: worst interpolation residual {worst_fixed:.2e} WRMS")
    assert worst_fixed >= 1e-2


@pytest.mark.parametrize("q", [1, 3, 5])
def test_vc_equals_fixed_at_constant_steps(orc, q):
    p = problem([[1], [0]], [[0], [1]], [1.0], rtol=1e30, atol=1e30)   # y' = 1 - y
    p["rates"] = np.array([1.0, 1.0])
    outs = []
    for vc in (False, True):
        b = orc.Bdf(p, qmax=5, fixed_step=True, vc=vc)
        h = 0.01
        z = np.array([[(-h) ** j / math.factorial(j) * (1 if j == 0 else -1)] for j in
                      range(q + 1)])
        z[0] = 0.0
        set_state(b, z, np.zeros(1), q, h, 0.0, 10 ** 6, [h] * 6)
        for _ in range(100):
            assert b.step(1e9) == 0
        outs.append(b.y()[0])
    assert outs[1] == pytest.approx(outs[0], rel=1e-13)


@pytest.mark.parametrize("q", [1, 2, 3, 4])
def test_vc_err_qp1_at_constant_steps_is_the_fixed_estimate(orc, q):
    """With equal past steps the order-(q+1) estimate of the variable form
    is the fixed form's (itself pinned exact in test_oracle_bdf_order)."""
    m = q
    top = (q - 1, 0)
    rng = W.rng_for(500 + q)
    sols = chain_solutions(m, rng.uniform(0.2, 1.0, m + 1), top)
    nu, mu = chain(m, top)
    N = m + 1
    t1, h = 1.0, 0.05
    ests = []
    for vc in (False, True):
        b = orc.Bdf(problem(nu, mu, np.zeros(N)), qmax=5, vc=vc)
        ts = past_times(t1, [h] * 6, q + 1)
        set_state(b, history_through(sols, ts, t1, h, q), np.zeros(N), q, h, t1, 50, [h] * 6)
        assert b.step(1e9) == 0
        _, acor1 = b.history()
        _, c1, h1 = b.past_steps()
        ts = past_times(t1 + h, [h] * 6, q + 1)
        set_state(b, history_through(sols, ts, t1 + h, h, q), acor1, q, h, t1 + h, 1,
                  [h] * 6, c1, h1)
        assert b.step(1e9) == 0
        ests.append(b.scalars()["err_qp1"])
    assert ests[1] == pytest.approx(ests[0], rel=1e-12)


def test_lazy_equals_eager_on_a_linear_problem_at_fixed_step(orc):
    """y' = A y with A constant: J never changes, and at a fixed step gamma
    does not either, so the stored factors are the fresh ones; the lazy
    run sets up once every 20 steps and ends where the eager run ends."""
    n = 4
    nu = np.zeros((n, n), np.int32)
    mu = np.zeros((n, n), np.int32)
    for k in range(n):                       # X_k -> X_{k+1} (last: -> 0)
        nu[k, k] = 1
        if k + 1 < n:
            mu[k, k + 1] = 1
    rates = np.array([50.0, 3.0, 0.7, 1e3])
    p = W.Problem(topologies=[(nu, mu)], cell_topo=np.zeros(3, np.int32),
                  rates=np.tile(rates, 3), y0=np.tile([1.0, 0, 0, 0], 3),
                  rtol=1e-3, atol=1e-3, t0=0.0, t_end=1e9, qmax=5, label="lin")
    h = 2e-4
    z1 = h * np.tile(orc.ma_rhs(nu, mu, rates, np.array([1.0, 0, 0, 0])), 3)
    outs, stats = [], []
    for lazy in (False, True):
        b = orc.Bdf(p, fixed_step=True, lazy=lazy)
        set_state(b, np.array([p.y0, z1]), np.zeros(3 * n), 1, h, 0.0, 10 ** 6, [h] * 6)
        for _ in range(95):
            assert b.step(1e9) == 0
        outs.append(b.y())
        stats.append(b.stats())
    assert np.allclose(outs[1], outs[0], rtol=1e-12, atol=1e-15)
    print({k: (stats[0][k], stats[1][k]) for k in ("nattempts", "netfails", "nsetups")})
    assert stats[0]["nattempts"] == stats[1]["nattempts"] == 95
    assert stats[0]["nsetups"] == 95
    assert stats[1]["nsetups"] == 5 and stats[1]["nstale_retries"] == 0


@pytest.mark.parametrize("case", ["network", "brusselator_gj"])
def test_lazy_run_is_as_accurate(orc, case):
    """Lazy reuse changes the Newton iteration, not the method: against a
    tight-tolerance run, the lazy run's error stays within 3x (+1 WRMS) of
    the eager run's, with a fraction of the setups."""
    if case == "network":
        p, lin = W.random_network_batch(32, n=10, seed=1601, t_end=1.0), 0
    else:
        p, lin = W.brusselator_batch(64), 3
    ref = orc.Bdf(p, rtol=p.rtol * 1e-3, atol=p.atol * 1e-3)
    assert ref.integrate(p.t_end) == 0
    yr = ref.y()

    def err(y):
        w = 1.0 / (p.rtol * np.abs(yr) + p.atol)
        return math.sqrt(np.mean(((y - yr) * w) ** 2))

    out = {}
    for name, kw in (("eager", {}), ("lazy", dict(lazy=True)),
                     ("vc_lazy", dict(vc=True, lazy=True))):
        b = orc.Bdf(p, linsol=lin, **kw)
        assert b.integrate(p.t_end) == 0
        out[name] = (err(b.y()), b.stats())
    e0, s0 = out["eager"]
    for name, (e, s) in out.items():
        print(case, name, f"error {e:.3e}", {k: s[k] for k in
              ("nsteps", "nattempts", "nsetups", "nniters", "nstale_retries")})
        assert e <= 3.0 * e0 + 1.0
    assert out["lazy"][1]["nsetups"] * 3 < s0["nsetups"]
