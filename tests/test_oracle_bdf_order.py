"""Pins for the oracle's order-selection arithmetic, starting step and
convergence order.

The paper names CVODE as the integrator (Section 1) without stating its
method, so the integrator is the fixed-coefficient Nordsieck BDF reading.
The order-change quantities it uses are derived from the same reading as
the local error estimate, so each is pinned here against an independent
computation, never against its own formula:

 * err_{q-1} (from the new history's z[q]) equals the true local error of
   the textbook order-(q-1) BDF step, solved directly from exact past values,
   on a solution whose top species is a degree-q polynomial;
 * err_{q+1} (from the difference of two successive corrections) equals the
   true local error of the textbook order-(q+1) step on a degree-(q+2)
   polynomial, when both steps start from exact interpolating histories;
 * an order raise sets z[q+1] to h^{q+1} y^{(q+1)} / (q+1)!, the Nordsieck
   component of the exact solution (degree q+1, so y^{(q+1)} is constant);
 * with the step size and order held fixed, the global error of BDF_q on
   y' = -y falls as h^q (q = 1..5);
 * the starting step equals scipy's independent implementation of the
   same published algorithm (Hairer, Norsett and Wanner, Solving ODEs I,
   Sec. II.4, with weighted RMS norms and p = 1).

Test problems are mass-action networks with polynomial solutions: the
reaction 0 -> X0 gives X0' = 1, and a catalytic reaction
X_a + X_b -> X_a + X_b + X_c gives X_c' = X_a X_b.
"""
import math

import numpy as np
import pytest

import workloads as W

P = np.polynomial.Polynomial


def problem(nu, mu, y0, rtol=1.0, atol=1.0, qmax=5, t_end=1e9):
    nu = np.asarray(nu, np.int32)
    mu = np.asarray(mu, np.int32)
    return W.Problem(topologies=[(nu, mu)], cell_topo=np.zeros(1, np.int32),
                     rates=np.ones(nu.shape[0]), y0=np.asarray(y0, float).copy(),
                     rtol=rtol, atol=atol, t0=0.0, t_end=t_end, qmax=qmax, label="pin")


def chain(m, top_product=None):
    """Species X0..X_{m-1}: 0 -> X0 and X_{k-1} -> X_{k-1} + X_k.  With
    top_product = (a, b) one more species T is added with T' = X_a X_b."""
    ns = m + (1 if top_product else 0)
    R = ns
    nu = np.zeros((R, ns), np.int32)
    mu = np.zeros((R, ns), np.int32)
    mu[0, 0] = 1
    for k in range(1, m):
        nu[k, k - 1] = 1
        mu[k, k - 1] = 1
        mu[k, k] = 1
    if top_product:
        a, b = top_product
        nu[m, a] += 1
        nu[m, b] += 1
        mu[m, a] += 1
        mu[m, b] += 1
        mu[m, m] += 1
    return nu, mu


def chain_solutions(m, consts, top_product=None):
    sols = [P([consts[0], 1.0])]
    for k in range(1, m):
        sols.append(P([consts[k]]) + sols[-1].integ())
    if top_product:
        a, b = top_product
        sols.append(P([consts[m]]) + (sols[a] * sols[b]).integ())
    return sols


def interpolating_history(sols, t1, h, q):
    """Nordsieck vector (z[0..q]) of the degree-q polynomial through the
    exact values at t1, t1 - h, ..., t1 - q h."""
    V = np.array([[(-j) ** k for k in range(q + 1)] for j in range(q + 1)], float)
    vals = np.array([[s(t1 - j * h) for s in sols] for j in range(q + 1)])
    return np.linalg.solve(V, vals)


def set_state(b, z, dprev, q, h, t, qwait):
    N = b.N
    z6 = np.zeros((6, N))
    z6[: len(z)] = z
    b.set_history(z6, dprev)
    b.set_scalars(dict(t=t, h=h, err_last=0.0, q=q, qwait=qwait, qprime_pending=0,
                       initialized=1, hu=h, qu=q, err_qm1=-1.0, err_qp1=-1.0,
                       eta_proposed=1.0, q_proposed=q))


def textbook_bdf_value(k, past, h, g_n):
    """y_n of the order-k BDF formula sum_{j=1..k} (1/j) nabla^j y_n = h g_n
    for a right-hand side g that does not depend on y, past = [y_{n-1}, ...,
    y_{n-k}] exact.  Solved directly: the coefficient of y_n is H_k."""
    Hk = sum(1.0 / j for j in range(1, k + 1))
    rest = 0.0
    for j in range(1, k + 1):
        for i in range(1, j + 1):
            rest += (1.0 / j) * (-1) ** i * math.comb(j, i) * past[i - 1]
    return (h * g_n - rest) / Hk


@pytest.mark.parametrize("q", [2, 3, 4, 5])
def test_err_qm1_is_true_error_of_order_q_minus_1_step(orc, q):
    m = q                                    # X_{q-1} has degree q
    rng = W.rng_for(400 + q)
    consts = rng.uniform(0.2, 1.0, m)
    sols = chain_solutions(m, consts)
    nu, mu = chain(m)
    t1, h = 1.0, 0.04
    b = orc.Bdf(problem(nu, mu, np.zeros(m)), qmax=5)
    z = interpolating_history(sols, t1, h, q)
    set_state(b, z, np.zeros(m), q, h, t1, qwait=1)
    assert b.step(1e9) == 0
    est = b.scalars()["err_qm1"]
    # true order-(q-1) step: only the top species (degree q) has an error
    top = sols[-1]
    g = sols[-2]
    past = [top(t1 - i * h) for i in range(q - 1)]
    yn = textbook_bdf_value(q - 1, past, h, g(t1 + h))
    err_top = yn - top(t1 + h)
    w_top = 1.0 / (abs(top(t1)) + 1.0)
    true = math.sqrt(err_top ** 2 * w_top ** 2 / m)
    assert est == pytest.approx(true, rel=1e-8)


@pytest.mark.parametrize("q", [1, 2, 3, 4])
def test_err_qp1_is_true_error_of_order_q_plus_1_step(orc, q):
    # X0..X_{q-1} of degrees 1..q (exact at order q); T' = X_{q-1} X0 has
    # degree q+2 and its step is a plain quadrature of exactly reproduced data
    m = q
    top = (q - 1, 0)
    rng = W.rng_for(500 + q)
    consts = rng.uniform(0.2, 1.0, m + 1)
    sols = chain_solutions(m, consts, top)
    nu, mu = chain(m, top)
    N = m + 1
    t1, h = 1.0, 0.05
    b = orc.Bdf(problem(nu, mu, np.zeros(N)), qmax=5)
    # first step from the exact history at t1: its correction becomes dprev
    set_state(b, interpolating_history(sols, t1, h, q), np.zeros(N), q, h, t1, qwait=50)
    assert b.step(1e9) == 0
    _, acor1 = b.history()
    # second step, same h, again from the exact history (now at t1 + h)
    set_state(b, interpolating_history(sols, t1 + h, h, q), acor1, q, h, t1 + h, qwait=1)
    assert b.step(1e9) == 0
    est = b.scalars()["err_qp1"]
    T = sols[-1]
    g = sols[top[0]] * sols[top[1]]
    tn = t1 + 2 * h
    past = [T(tn - i * h) for i in range(1, q + 2)]
    yn = textbook_bdf_value(q + 1, past, h, g(tn))
    err_T = yn - T(tn)
    w_T = 1.0 / (abs(T(t1 + h)) + 1.0)
    true = math.sqrt(err_T ** 2 * w_T ** 2 / N)
    assert est == pytest.approx(true, rel=1e-7)


@pytest.mark.parametrize("q", [1, 2, 3, 4])
def test_order_raise_sets_exact_nordsieck_component(orc, q):
    m = q + 1                                # top species X_q has degree q+1
    rng = W.rng_for(600 + q)
    consts = rng.uniform(0.2, 1.0, m)
    sols = chain_solutions(m, consts)
    nu, mu = chain(m)
    t1, h = 1.0, 0.05
    b = orc.Bdf(problem(nu, mu, np.zeros(m)), qmax=5)
    set_state(b, interpolating_history(sols, t1, h, q), np.zeros(m), q, h, t1, qwait=50)
    assert b.step(1e9) == 0
    _, acor1 = b.history()
    # the same step again one h later: the two corrections agree, so the
    # order-(q+1) estimate vanishes and the raise is selected
    set_state(b, interpolating_history(sols, t1 + h, h, q), acor1, q, h, t1 + h, qwait=1)
    assert b.step(1e9) == 0
    sc = b.scalars()
    assert sc["q"] == q + 1
    hn = sc["h"]
    assert hn == pytest.approx(10.0 * h, rel=1e-14)      # growth clamped at 10
    z, _ = b.history()
    lead = [s.coef[q + 1] if len(s.coef) > q + 1 else 0.0 for s in sols]
    expect = np.array(lead) * hn ** (q + 1)
    assert z[q + 1][-1] == pytest.approx(expect[-1], rel=1e-9)
    # lower species are reproduced exactly: their corrections are rounding,
    # scaled by the raise coefficient and the rescale by 10^{q+1}
    assert np.abs(z[q + 1][:-1]).max() <= 100 * 2.2e-16 * 10.0 ** (q + 1)


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5])
def test_fixed_step_global_error_order(orc, q):
    """y' = -y on [0, 1] with h and q held fixed and an exact Taylor
    starting history: the global error of BDF_q is O(h^q)."""
    p = problem([[1]], [[0]], [1.0], rtol=1e30, atol=1e30)
    errs = []
    Ns = (40, 80) if q <= 2 else (20, 40)
    for nsteps in Ns:
        h = 1.0 / nsteps
        b = orc.Bdf(p, qmax=5, fixed_step=True)
        z = np.array([[(-h) ** j / math.factorial(j)] for j in range(q + 1)])
        set_state(b, z, np.zeros(1), q, h, 0.0, qwait=10 ** 6)
        for _ in range(nsteps):
            assert b.step(1e9) == 0
        sc = b.scalars()
        assert sc["q"] == q and sc["h"] == h
        assert sc["t"] == pytest.approx(1.0, rel=1e-13)
        errs.append(abs(b.y()[0] - math.exp(-1.0)))
    slope = math.log2(errs[0] / errs[1])
    assert abs(slope - q) <= 0.25, (q, errs, slope)


@pytest.mark.parametrize("seed,t_end", [(1, 1e9), (2, 1e9), (3, 1e-9), (4, 1e9)])
def test_starting_step_matches_scipy(orc, seed, t_end):
    from scipy.integrate._ivp.common import select_initial_step
    p = W.random_network_batch(6, n=10, seed=900 + seed)
    p["t_end"] = t_end
    if seed == 4:          # no reactions fire: both derivatives vanish
        p["rates"] = np.zeros_like(p.rates)
    b = orc.Bdf(p)
    b.init(t_end)
    h = b.scalars()["h"]
    nu, mu = p.topologies[0]
    n, R = 10, nu.shape[0]

    def fun(t, y):
        return np.concatenate([orc.ma_rhs(nu, mu, p.rates[c * R:(c + 1) * R], y[c * n:(c + 1) * n])
                               for c in range(p.ncells)])

    y0 = p.y0.copy()
    ref = select_initial_step(fun, 0.0, y0, t_end, np.inf, fun(0.0, y0), 1, 1, p.rtol, p.atol)
    assert h == pytest.approx(ref, rel=1e-12)
