"""Pins for the oracle's mass-action right-hand side and Jacobian.

Per-cell chemistry of the paper's submodel use case (Section 2): every cell
carries the same small network; the integrator groups the cells.  Pins: the
textbook Robertson equations, count conservation, the analytic Jacobian
against central differences, and a zero-order source.
"""
import numpy as np
import pytest

import workloads as W


def test_robertson_textbook_equations(orc):
    nu, mu = W.robertson_topology()
    k = W.ROBERTSON_RATES
    rng = W.rng_for(21)
    for _ in range(20):
        y = rng.uniform(0, 1, 3)
        A, B, Cc = y
        ref = np.array([-0.04 * A + 1e4 * B * Cc,
                        0.04 * A - 1e4 * B * Cc - 3e7 * B * B,
                        3e7 * B * B])
        f = orc.ma_rhs(nu, mu, k, y)
        assert np.allclose(f, ref, rtol=1e-14, atol=1e-14 * np.abs(ref).max())
        J = orc.ma_jac(nu, mu, k, y)
        Jref = np.array([[-0.04, 1e4 * Cc, 1e4 * B],
                         [0.04, -1e4 * Cc - 6e7 * B, -1e4 * B],
                         [0.0, 6e7 * B, 0.0]])
        assert np.allclose(J, Jref, rtol=1e-14, atol=1e-6)


@pytest.mark.parametrize("n", [3, 10, 21, 64])
def test_conservation_and_fd_jacobian(orc, n):
    rng = W.rng_for(30 + n)
    nu, mu = W.random_network(n, 2 * n, rng)
    # every reaction consumes and produces the same number of molecules
    assert np.array_equal(nu.sum(1), mu.sum(1))
    k = W.log_uniform(rng, -3, 3, 2 * n)
    y = rng.uniform(0.1, 1.0, n)
    f = orc.ma_rhs(nu, mu, k, y)
    J = orc.ma_jac(nu, mu, k, y)
    scale = np.abs(k).max() * 10
    assert abs(f.sum()) <= 1e-13 * scale
    assert np.abs(J.sum(0)).max() <= 1e-13 * scale
    eps = 1e-6
    for j in range(n):
        e = np.zeros(n)
        e[j] = eps
        fd = (orc.ma_rhs(nu, mu, k, y + e) - orc.ma_rhs(nu, mu, k, y - e)) / (2 * eps)
        # second-order networks: central difference is exact up to rounding
        assert np.allclose(J[:, j], fd, rtol=1e-7, atol=1e-7 * scale)


def test_zero_order_source_and_catalysis(orc):
    # 0 -> X1 (rate 2), X1 -> X1 + X2 (rate 3)
    nu = np.array([[0, 0], [1, 0]], np.int32)
    mu = np.array([[1, 0], [1, 1]], np.int32)
    y = np.array([0.5, 7.0])
    f = orc.ma_rhs(nu, mu, [2.0, 3.0], y)
    assert np.array_equal(f, [2.0, 1.5])
    J = orc.ma_jac(nu, mu, [2.0, 3.0], y)
    assert np.array_equal(J, [[0.0, 0.0], [3.0, 0.0]])


def test_network_generator_properties():
    rng = W.rng_for(5)
    nu, mu = W.random_network(10, 20, rng)
    assert nu.shape == (20, 10)
    order = nu.sum(1)
    assert set(order.tolist()) <= {1, 2}
    for k in range(20):
        assert not np.array_equal(nu[k], mu[k])
