"""Oracle pins for the paper's demonstration reaction and the Gauss-Jordan
block inverse (Section 7: the task-local solver applies the inverse of
each 3 x 3 block, generated with a symbolic Gauss-Jordan method).

* The mass-action network of workloads.brusselator_topology reproduces the
  paper's three reaction equations and their Jacobian exactly as written.
* orc_gj_inverse equals the exact rational inverse (fractions) of integer
  matrices, numpy's inverse on random well-conditioned blocks, a
  permutation's transpose, and flags the first zero pivot.
* The integrator with the Gauss-Jordan solve takes the same steps as with
  LU on the demonstration reaction and ends within 1e-6 WRMS of it.
"""
from fractions import Fraction

import numpy as np
import pytest

import workloads as W


def paper_rhs(y, A=1.0, B=3.5, eps=5e-6):
    u, v, w = y
    return np.array([A - (w + 1.0) * u + v * u * u, w * u - v * u * u, (B - w) / eps - w * u])


def paper_jac(y, A=1.0, B=3.5, eps=5e-6):
    u, v, w = y
    return np.array([[-(w + 1.0) + 2.0 * u * v, u * u, -u],
                     [w - 2.0 * u * v, -u * u, u],
                     [-w, 0.0, -1.0 / eps - u]])


def test_network_is_the_paper_reaction(orc):
    nu, mu = W.brusselator_topology()
    k = W.brusselator_rates()
    rng = W.rng_for(5)
    for _ in range(20):
        y = rng.uniform(0.1, 5.0, 3)
        f = orc.ma_rhs(nu, mu, k, y)
        ref = paper_rhs(y)
        assert np.allclose(f, ref, rtol=1e-13, atol=1e-13 * np.abs(k).max())
        J = orc.ma_jac(nu, mu, k, y)
        assert np.allclose(J, paper_jac(y), rtol=1e-13, atol=1e-13 * np.abs(k).max())


def test_initial_profile_matches_the_paper():
    p = W.brusselator_batch(101, length=10.0)
    y = p.y0.reshape(-1, 3)
    mid = y[50]    # x = 5 = length / 2: the Gaussian's peak, p = 0.1 at the centre cell
    assert mid[0] == pytest.approx(1.1, abs=1e-4)
    assert mid[1] == pytest.approx(3.6, abs=1e-4)
    assert mid[2] == pytest.approx(3.1, abs=1e-4)
    assert np.all(y[:, 0] > 1.0) and np.all(np.diff(y[:51, 0]) > 0)


def exact_inverse(M):
    n = len(M)
    a = [[Fraction(int(M[i][j])) for j in range(n)] + [Fraction(int(i == j)) for j in range(n)]
         for i in range(n)]
    for k in range(n):
        p = max(range(k, n), key=lambda i: (abs(a[i][k]), -i))
        a[k], a[p] = a[p], a[k]
        d = a[k][k]
        a[k] = [x / d for x in a[k]]
        for i in range(n):
            if i != k:
                f = a[i][k]
                a[i] = [x - f * y for x, y in zip(a[i], a[k])]
    return np.array([[float(x) for x in row[n:]] for row in a])


@pytest.mark.parametrize("n", [2, 3, 4])
def test_gj_inverse_exact_on_integer_blocks(orc, n):
    rng = W.rng_for(100 + n)
    for _ in range(30):
        M = rng.integers(-9, 10, size=(n, n)).astype(np.float64)
        if abs(np.linalg.det(M)) < 0.5:
            continue
        X, info = orc.gj_inverse(M[None])
        assert info[0] == 0
        Xe = exact_inverse(M)
        assert np.allclose(X[0], Xe, rtol=1e-13, atol=1e-15 * np.abs(Xe).max())


def test_gj_inverse_random_permutation_singular(orc):
    rng = W.rng_for(7)
    A = W.random_blocks(40, 8, seed=8, diag_shift=3.0)
    X, info = orc.gj_inverse(A)
    assert np.all(info == 0)
    assert np.allclose(np.einsum("bij,bjk->bik", X, A), np.eye(8)[None], atol=1e-12)
    P = np.eye(4)[[2, 0, 3, 1]]
    X, info = orc.gj_inverse(P[None])
    assert info[0] == 0 and np.array_equal(X[0], P.T)
    S = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [0.0, 1.0, 1.0]])
    _, info = orc.gj_inverse(S[None])
    assert info[0] == 3     # columns 1 and 2 are eliminated, the third pivot is exactly zero


def test_integrator_gj_equals_lu_on_the_reaction(orc):
    p = W.brusselator_batch(24, t_end=2.0)
    a = orc.Bdf(p, linsol=orc.LS_GJ)
    b = orc.Bdf(p)
    assert a.integrate(p.t_end) == 0 and b.integrate(p.t_end) == 0
    sa, sb = a.stats(), b.stats()
    assert sa["nsteps"] == sb["nsteps"] and sa["nattempts"] == sb["nattempts"]
    w = 1.0 / (p.rtol * np.abs(b.y()) + p.atol)
    assert np.sqrt(np.mean(((a.y() - b.y()) * w) ** 2)) <= 1e-6
    assert sa["lp_cell_solves"] == 0
