"""Pins for the oracle's vector operations.

The paper splits vector operations into streaming operations and reductions
that return one scalar (Section 2; Section 4.1).  The fused operations are not
defined there, so the oracle writes their plain definitions out; these tests
pin them with exact integer arithmetic, closed forms and exact rationals.
"""
from fractions import Fraction

import numpy as np
import pytest

import workloads as W


def _ints(rng, shape, lo=-1000, hi=1000):
    return rng.integers(lo, hi, size=shape).astype(np.float64)


def test_linear_sum_exact_on_integers(orc):
    rng = W.rng_for(1)
    x, y = _ints(rng, 1001), _ints(rng, 1001)
    z = orc.linear_sum(3.0, x, -2.0, y)
    assert np.array_equal(z, 3 * x - 2 * y)


def test_linear_combination_exact_on_integers(orc):
    rng = W.rng_for(2)
    X = _ints(rng, (16, 777))
    c = rng.integers(-8, 8, size=16).astype(np.float64)
    z = orc.linear_combination(c, list(X))
    ref = np.array([sum(int(c[j]) * int(X[j, i]) for j in range(16)) for i in range(777)], dtype=np.float64)
    assert np.array_equal(z, ref)


def test_linear_combination_identities(orc):
    rng = W.rng_for(3)
    x = rng.uniform(-1, 1, 500)
    # (x, -x) with equal coefficients cancels exactly
    assert np.array_equal(orc.linear_combination([0.7, 0.7], [x, -x]), np.zeros(500))
    # all X_j = 1 gives sum(c) (exact for dyadic coefficients)
    c = np.array([0.5, -0.25, 2.0, 1.125])
    ones = [np.ones(10)] * 4
    assert np.array_equal(orc.linear_combination(c, ones), np.full(10, c.sum()))
    # one vector: plain scaling
    assert np.array_equal(orc.linear_combination([2.0], [x]), 2.0 * x)


def test_scale_add_multi(orc):
    rng = W.rng_for(4)
    x = _ints(rng, 300)
    Y = [_ints(rng, 300) for _ in range(6)]
    a = np.array([0.0, 1.0, -1.0, 2.0, 3.0, -4.0])
    Z = orc.scale_add_multi(a, x, Y)
    for j in range(6):
        assert np.array_equal(Z[j], a[j] * x + Y[j])
    assert np.array_equal(Z[0], Y[0])  # a_j = 0 gives Y_j


def test_dot_prod_multi_exact_rationals(orc):
    rng = W.rng_for(5)
    x = rng.uniform(-1, 1, 4000)
    Y = [rng.uniform(-1, 1, 4000) for _ in range(8)]
    d = orc.dot_prod_multi(x, Y)
    for j in range(8):
        exact = sum(Fraction(a) * Fraction(b) for a, b in zip(x, Y[j]))
        # compensated summation: within a couple of ulps of the exact value
        assert abs(Fraction(d[j]) - exact) <= Fraction(4e-16) * max(abs(exact), Fraction(1e-300)) + Fraction(1e-300)


def test_dot_prod_unit_basis(orc):
    rng = W.rng_for(6)
    x = rng.uniform(-1, 1, 9)
    E = list(np.eye(9)[:8])
    assert np.array_equal(orc.dot_prod_multi(x, E), x[:8])


def test_wrms_constant_vectors(orc):
    for n in (1, 7, 1000):
        for c, w in ((3.0, 0.5), (-2.5, 4.0), (1e-3, 1e8)):
            v = orc.wrms_norm(np.full(n, c), np.full(n, w))
            assert v == pytest.approx(abs(c * w), rel=2e-16, abs=0)


def test_wrms_exact_rational(orc):
    rng = W.rng_for(7)
    x = rng.uniform(-1, 1, 3000)
    w = rng.uniform(1e2, 1e8, 3000)
    v = orc.wrms_norm(x, w)
    s = sum((Fraction(a) * Fraction(b)) ** 2 for a, b in zip(x, w)) / len(x)
    exact = float(s) ** 0.5
    assert v == pytest.approx(exact, rel=4e-16)


def test_empty_and_single(orc):
    assert orc.wrms_norm(np.zeros(0), np.zeros(0)) == 0.0
    assert orc.wrms_norm(np.array([-3.0]), np.array([2.0])) == 6.0
    assert orc.max_norm(np.array([1.0, -5.0, 2.0])) == 5.0


def test_ewt(orc):
    y = np.array([0.0, 1.0, -2.0, 1e-4])
    w = orc.ewt(y, 1e-6, 1e-10)
    assert w[0] == 1e10                       # pure absolute tolerance
    assert w[1] == pytest.approx(1.0 / (1e-6 + 1e-10), rel=1e-15)
    assert w[2] == w[2] and w[2] < w[1]       # sign of y does not matter
    # weighted value of one tolerance unit is 1
    tol = 1e-6 * np.abs(y) + 1e-10
    assert np.allclose(w * tol, 1.0, rtol=1e-15, atol=0)
