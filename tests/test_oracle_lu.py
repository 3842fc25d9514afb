"""Pins for the oracle's per-block dense LU (getrf semantics) and solves.

The batched block-diagonal direct solve is the paper's Section 5 (one
dense block per cell, one shared pattern); the per-block algorithm is
right-looking LU with partial pivoting.  Pins: exact rational elimination
on small integer blocks, scipy's LAPACK getrf pivots, permutation matrices,
backward error and the singular-pivot report.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sl

import workloads as W


def rational_lu(A):
    """Exact partial-pivot LU over the rationals (first maximal pivot)."""
    n = len(A)
    M = [[Fraction(int(v)) for v in row] for row in A]
    piv = []
    info = 0
    for k in range(n):
        p = max(range(k, n), key=lambda i: (abs(M[i][k]), -i))
        piv.append(p)
        M[k], M[p] = M[p], M[k]
        if M[k][k] == 0:
            info = info or k + 1
            continue
        for i in range(k + 1, n):
            M[i][k] = M[i][k] / M[k][k]
            for j in range(k + 1, n):
                M[i][j] -= M[i][k] * M[k][j]
    return M, piv, info


@pytest.mark.parametrize("n", [2, 3, 4])
def test_lu_matches_exact_rationals(orc, n):
    rng = W.rng_for(100 + n)
    A = rng.integers(-9, 10, size=(40, n, n)).astype(np.float64)
    LU, piv, info = orc.lu_factor(A)
    for b in range(40):
        M, p, inf = rational_lu(A[b])
        assert list(piv[b]) == p
        assert info[b] == inf
        for i in range(n):
            for j in range(n):
                ex = M[i][j]
                assert abs(Fraction(LU[b, i, j]) - ex) <= Fraction(1e-13) * max(1, abs(ex))


def test_lu_pivots_match_lapack_on_separated_pivots(orc):
    rng = W.rng_for(7)
    A = rng.uniform(-1, 1, size=(50, 8, 8))
    LU, piv, info = orc.lu_factor(A)
    # continuous random entries: pivot ties have probability zero, so
    # LAPACK (which scales by the reciprocal pivot) must choose the same rows
    for b in range(50):
        lu, pv = sl.lu_factor(A[b])
        assert info[b] == 0
        assert np.array_equal(piv[b], pv)
        assert np.allclose(LU[b], lu, rtol=1e-12, atol=1e-13)


def test_permutation_matrix(orc):
    P = np.eye(6)[[3, 0, 5, 1, 4, 2]]
    LU, piv, info = orc.lu_factor(P[None])
    assert info[0] == 0
    assert np.array_equal(np.abs(np.diag(LU[0])), np.ones(6))
    x = orc.lu_solve(LU, piv, np.arange(6.0)[None])
    assert np.array_equal(P @ x[0], np.arange(6.0))


@pytest.mark.parametrize("n", [3, 10, 21, 64])
def test_backward_error(orc, n):
    A = W.random_blocks(20, n, seed=n)
    B = W.rng_for(n + 1).uniform(-1, 1, (20, n))
    LU, piv, info = orc.lu_factor(A)
    X = orc.lu_solve(LU, piv, B)
    u = 2.0 ** -53
    for b in range(20):
        r = A[b] @ X[b] - B[b]
        berr = np.abs(r).max() / (np.abs(A[b]).sum(1).max() * np.abs(X[b]).max())
        assert berr <= 10 * n * u
        # the factors reproduce PA
        L = np.tril(LU[b], -1) + np.eye(n)
        U = np.triu(LU[b])
        PA = A[b].copy()
        for k in range(n):
            PA[[k, piv[b, k]]] = PA[[piv[b, k], k]]
        assert np.allclose(L @ U, PA, atol=20 * n * u * np.abs(A[b]).max())


def test_singular_pivot_reports_info(orc):
    A = np.array([[[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [1.0, 0.0, 1.0]]])
    _, _, info = orc.lu_factor(A)
    assert info[0] == 3
    Z = np.zeros((1, 4, 4))
    _, piv, info = orc.lu_factor(Z)
    assert info[0] == 1 and list(piv[0]) == [0, 1, 2, 3]


def test_f32_lu_is_float_arithmetic(orc):
    A = W.random_blocks(10, 6, seed=3).astype(np.float32)
    LU, piv, info = orc.lu_factor_f32(A)
    LU64, piv64, _ = orc.lu_factor(A.astype(np.float64))
    assert np.array_equal(piv, piv64)
    assert np.allclose(LU, LU64, rtol=1e-4, atol=1e-5)
    assert LU.dtype == np.float32


def test_refinement_reaches_fp64(orc):
    n = 10
    A = W.random_blocks(30, n, seed=11, diag_shift=3.0)
    B = W.rng_for(12).uniform(-1, 1, (30, n))
    X, st, sw = orc.refine_solve(A, B, max_it=5)
    LU, piv, _ = orc.lu_factor(A)
    X64 = orc.lu_solve(LU, piv, B)
    u = 2.0 ** -53
    assert np.all(st == 0)
    for b in range(30):
        kappa = np.linalg.cond(A[b], np.inf)
        assert np.abs(X[b] - X64[b]).max() <= 10 * n * u * kappa * np.abs(X64[b]).max()


def test_refinement_falls_back_on_ill_conditioned_block(orc):
    n = 6
    rng = W.rng_for(13)
    Q1, _ = np.linalg.qr(rng.normal(size=(n, n)))
    Q2, _ = np.linalg.qr(rng.normal(size=(n, n)))
    s = np.logspace(0, -9, n)           # cond ~ 1e9 >> 1/eps32
    A = (Q1 * s) @ Q2.T
    b = rng.uniform(-1, 1, n)
    X, st, sw = orc.refine_solve(A[None], b[None], max_it=5)
    assert st[0] == 1
    LU, piv, _ = orc.lu_factor(A[None])
    assert np.allclose(X[0], orc.lu_solve(LU, piv, b[None])[0], rtol=0, atol=0)
