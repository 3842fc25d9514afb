"""Pins for the oracle's MLP (learned block preconditioner) pieces.

Not from the paper: the learned preconditioner is an addition on top of the
paper's block-diagonal direct solve (Section 5).  Pins: BF16 round-to-nearest-
even against torch's independent conversion, the backward pass against central
finite differences (rounding points off), the loss of an exact inverse, and
Adam's first step in closed form.
"""
import numpy as np
import pytest
import torch

import workloads as W


def test_bf16_rounding_matches_torch(orc):
    rng = W.rng_for(1)
    vals = np.concatenate([rng.normal(size=2000).astype(np.float32),
                           np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.5 - 2 ** -8,
                                     65504.0, 1e-40, 0.0, -0.0, 3.0e38], np.float32)])
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float32).numpy()
    got = np.array([orc.bf16_round(v) for v in vals], np.float32)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def small_net(orc, n=3, hid=8, seed=3):
    rng = W.rng_for(seed)
    nin, nout = n + 1, n * n
    W1 = rng.normal(0, 0.5, (hid, nin)).astype(np.float32)
    b1 = rng.normal(0, 0.1, hid).astype(np.float32)
    W2 = rng.normal(0, 0.5, (hid, hid)).astype(np.float32)
    b2 = rng.normal(0, 0.1, hid).astype(np.float32)
    W3 = rng.normal(0, 0.5, (nout, hid)).astype(np.float32)
    b3 = rng.normal(0, 0.1, nout).astype(np.float32)
    mean = rng.normal(0, 0.1, nin)
    std = rng.uniform(0.5, 2.0, nin)
    return orc.MLP(W1, b1, W2, b2, W3, b3, mean, std)


def test_backward_against_finite_differences(orc):
    n = 3
    net = small_net(orc, n)
    rng = W.rng_for(4)
    X = rng.normal(size=(5, n + 1))
    M = np.eye(n)[None] + 0.3 * rng.normal(size=(5, n, n))
    orc.set_bf16(False)
    try:
        L, g = net.loss_grad(X, M)
        params = [net.W1, net.b1, net.W2, net.b2, net.W3, net.b3]
        for p, gp in zip(params, g):
            flat = p.reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                h = 1e-2 * max(1.0, abs(float(old)))
                # FP32 weights: perturb by an exactly representable step
                flat[idx] = np.float32(old + h)
                hp = float(flat[idx]) - float(old)
                Lp, _ = net.loss_grad(X, M)
                flat[idx] = np.float32(old - h)
                hm = float(old) - float(flat[idx])
                Lm, _ = net.loss_grad(X, M)
                flat[idx] = old
                fd = (Lp - Lm) / (hp + hm)
                gv = gp.reshape(-1)[idx]
                # loss is piecewise quadratic in each weight: central
                # differences are exact unless a ReLU switches
                assert fd == pytest.approx(gv, rel=1e-6, abs=1e-9)
    finally:
        orc.set_bf16(True)


def test_exact_inverse_has_zero_loss(orc):
    """With W3 = 0 and b3 = vec(M^-1 - I) the net outputs the exact inverse."""
    n = 3
    net = small_net(orc, n)
    rng = W.rng_for(6)
    M = np.eye(n) + 0.2 * rng.normal(size=(n, n))
    Xinv = np.linalg.inv(M)
    net.W3[:] = 0
    net.b3[:] = (Xinv - np.eye(n)).reshape(-1).astype(np.float32)
    L, g = net.loss_grad(rng.normal(size=(1, n + 1)), M[None])
    assert L <= 1e-12       # only the FP32 rounding of b3 remains
    out = net.forward(rng.normal(size=(1, n + 1)))[0]
    assert np.allclose(out.reshape(n, n) + np.eye(n), Xinv, atol=1e-6)


def test_adam_first_step_closed_form(orc):
    rng = W.rng_for(7)
    p = rng.normal(size=50).astype(np.float32)
    g = rng.normal(size=50)
    m1, m2 = np.zeros(50), np.zeros(50)
    p0 = p.copy()
    orc.adam_step(p, g, m1, m2, 1, lr=1e-3)
    # bias-corrected first step is lr * g / (|g| + eps) = lr * sign(g)
    expect = p0.astype(np.float64) - 1e-3 * g / (np.abs(g) + 1e-8)
    assert np.allclose(p, expect.astype(np.float32), rtol=0, atol=1e-7)
