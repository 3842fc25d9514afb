"""GPU parity of the N_Vector operations against the CPU oracle.

Streaming and reduction operations of Section 2 / Section 4.1.  Bar:
componentwise |z - z_ref| <= 1e-12 * sum_j |c_j x_ji| for streaming
operations, |d - d_ref| <= 1e-12 * sum_i |x_i y_i| for dot products,
1e-12 relative for the WRMS norm; exact for max norm, ewt-free ops on
integers.  Sizes span several launch tiles, a ragged tail, length 0 and 1,
and misaligned (odd-offset) vectors.
"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 17, 4099, 1 << 18 | 3]


def T(a, dev):
    return torch.tensor(np.asarray(a, np.float64), device=dev)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("nv", [1, 2, 7, 16])
def test_linear_combination(orc, dev, G, n, nv):
    X = W.uniform_vectors(nv, n, seed=11 + n)
    c = W.uniform_coefficients(nv, seed=3 + nv)
    Xd = [T(x, dev) for x in X]
    z = torch.empty(n, dtype=torch.float64, device=dev)
    G.nvec_linear_combination(c, Xd, z)
    if n == 0:
        return
    ref = orc.linear_combination(c, list(X))
    bound = 1e-12 * (np.abs(c[:, None] * X).sum(0)) + 1e-300
    assert np.all(np.abs(z.cpu().numpy() - ref) <= bound)


# From 12 vectors, whole chunks of 8192 16-byte units (16384 doubles) take the long-run kernel and
# the rest the tile kernel on advanced pointers: one unit short of a chunk, exactly one chunk, and
# three chunks plus 2048 units plus an odd element.
CHUNK = 16384


@pytest.mark.parametrize("n", [CHUNK - 2, CHUNK, 3 * CHUNK + 4096 + 1])
@pytest.mark.parametrize("nv", [12, 13, 16])
@pytest.mark.parametrize("alias", [False, True])
def test_linear_combination_long_runs(orc, dev, G, n, nv, alias):
    X = W.uniform_vectors(nv, n, seed=31 + n + nv)
    c = W.uniform_coefficients(nv, seed=7 + nv)
    Xd = [T(x, dev) for x in X]
    z = Xd[0] if alias else torch.empty(n, dtype=torch.float64, device=dev)
    G.nvec_linear_combination(c, Xd, z)
    ref = orc.linear_combination(c, list(X))
    bound = 1e-12 * (np.abs(c[:, None] * X).sum(0))
    assert np.all(np.abs(z.cpu().numpy() - ref) <= bound)


def test_linear_combination_misaligned_and_aliased(orc, dev, G):
    n = 10001
    X = W.uniform_vectors(3, n + 1, seed=5)
    base = [T(x, dev) for x in X]
    Xd = [b[1:] for b in base]               # 8-byte offset: scalar path
    c = [0.5, -1.25, 2.0]
    out = Xd[0]                              # z aliases X[0]
    ref = orc.linear_combination(c, [x[1:] for x in X])
    G.nvec_linear_combination(c, Xd, out)
    bound = 1e-12 * np.abs(np.array(c)[:, None] * X[:, 1:]).sum(0)
    assert np.all(np.abs(out.cpu().numpy() - ref) <= bound)


@pytest.mark.parametrize("n", SIZES)
def test_linear_sum_scale_const_ewt(orc, dev, G, n):
    rng = W.rng_for(40 + n)
    x, y = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    xd, yd = T(x, dev), T(y, dev)
    z = torch.empty(n, dtype=torch.float64, device=dev)
    G.nvec_linear_sum(0.3, xd, -1.7, yd, z)
    ref = orc.linear_sum(0.3, x, -1.7, y)
    assert np.all(np.abs(z.cpu().numpy() - ref) <= 1e-12 * (0.3 * np.abs(x) + 1.7 * np.abs(y)) + 1e-300)
    G.nvec_scale(2.5, xd, z)
    assert np.array_equal(z.cpu().numpy(), orc.scale(2.5, x))
    G.nvec_const(-3.0, z)
    assert np.array_equal(z.cpu().numpy(), orc.const(-3.0, n))
    G.nvec_ewt(xd, 1e-6, 1e-10, z)
    assert np.allclose(z.cpu().numpy(), orc.ewt(x, 1e-6, 1e-10), rtol=1e-15, atol=0)


@pytest.mark.parametrize("n", [1, 2, 4099, 1 << 18 | 3])
def test_scale_const_ewt_misaligned_and_in_place(orc, dev, G, n):
    """8-byte offset views (element-by-element kernels), then the aligned
    16-byte-unit kernels in place (z aliases x) with an odd tail."""
    rng = W.rng_for(90 + n)
    x = rng.uniform(-1, 1, n + 1)
    base = T(x, dev)
    xd = base[1:]
    z = torch.empty(n + 1, dtype=torch.float64, device=dev)[1:]
    G.nvec_scale(-0.75, xd, z)
    assert np.array_equal(z.cpu().numpy(), orc.scale(-0.75, x[1:]))
    G.nvec_ewt(xd, 1e-6, 1e-10, z)
    assert np.allclose(z.cpu().numpy(), orc.ewt(x[1:], 1e-6, 1e-10), rtol=1e-15, atol=0)
    G.nvec_const(7.5, z)
    assert np.array_equal(z.cpu().numpy(), orc.const(7.5, n))
    y = T(x[1:], dev)
    G.nvec_scale(3.0, y, y)
    assert np.array_equal(y.cpu().numpy(), orc.scale(3.0, x[1:]))


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("nv", [1, 3, 6])
def test_scale_add_multi(orc, dev, G, n, nv):
    rng = W.rng_for(60 + n + nv)
    x = rng.uniform(-1, 1, n)
    Y = [rng.uniform(-1, 1, n) for _ in range(nv)]
    a = rng.uniform(-1, 1, nv)
    Zd = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(nv)]
    G.nvec_scale_add_multi(a, T(x, dev), [T(v, dev) for v in Y], Zd)
    ref = orc.scale_add_multi(a, x, Y)
    for j in range(nv):
        b = 1e-12 * (np.abs(a[j] * x) + np.abs(Y[j])) + 1e-300
        assert np.all(np.abs(Zd[j].cpu().numpy() - ref[j]) <= b)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("nv", [1, 8])
def test_dot_prod_multi(orc, dev, G, n, nv):
    rng = W.rng_for(80 + n)
    x = rng.uniform(-1, 1, n)
    Y = [rng.uniform(-1, 1, n) for _ in range(nv)]
    d = G.nvec_dot_prod_multi(T(x, dev), [T(v, dev) for v in Y])
    if n == 0:
        assert d == [0.0] * nv
        return
    ref = orc.dot_prod_multi(x, Y)
    for j in range(nv):
        assert abs(d[j] - ref[j]) <= 1e-12 * np.abs(x * Y[j]).sum()
    # device-result variant is asynchronous and gives the same numbers
    out = torch.empty(nv, dtype=torch.float64, device=dev)
    G.nvec_dot_prod_multi(T(x, dev), [T(v, dev) for v in Y], out=out)
    assert np.array_equal(out.cpu().numpy(), np.array(d))


@pytest.mark.parametrize("n", SIZES)
def test_wrms_and_max(orc, dev, G, n):
    x = W.uniform_vectors(1, n, seed=90 + n)[0]
    w = W.weight_vector(n, seed=91 + n)
    v = G.nvec_wrms_norm(T(x, dev), T(w, dev))
    ref = orc.wrms_norm(x, w)
    assert v == pytest.approx(ref, rel=1e-12, abs=0)
    m = G.nvec_max_norm(T(x, dev))
    assert m == orc.max_norm(x)
    # device-result variants write the same numbers straight into `out`
    out = torch.full((1,), -1.0, dtype=torch.float64, device=dev)
    G.nvec_wrms_norm(T(x, dev), T(w, dev), out=out)
    assert out.item() == v
    G.nvec_max_norm(T(x, dev), out=out)
    assert out.item() == m


def test_wrms_constant_closed_form(dev, G):
    n = 1 << 20
    v = G.nvec_wrms_norm(torch.full((n,), -3.0, dtype=torch.float64, device=dev),
                         torch.full((n,), 0.25, dtype=torch.float64, device=dev))
    assert v == pytest.approx(0.75, rel=1e-15)


def test_full_size_microbench_parity(orc, dev, G):
    """The 2^26-element workload in the launch configuration the benchmark
    times: sampled elements of the 16-vector combination against the oracle
    element by element; the 8 dot products and the WRMS norm against the
    oracle over the whole vectors."""
    n = 1 << 26
    X = [W.torch_uniform_device(n, seed=1000 + j, device=dev) for j in range(16)]
    c = W.uniform_coefficients(16, seed=20242)
    z = torch.empty(n, dtype=torch.float64, device=dev)
    G.nvec_linear_combination(c, X, z)
    idx = torch.tensor(np.sort(W.rng_for(7).choice(n, 4096, replace=False)), device=dev)
    xs = torch.stack([x[idx] for x in X]).cpu().numpy()
    ref = orc.linear_combination(c, list(xs))
    bound = 1e-12 * np.abs(c[:, None] * xs).sum(0)
    assert np.all(np.abs(z[idx].cpu().numpy() - ref) <= bound)
    d = G.nvec_dot_prod_multi(X[0], X[1:9])
    x0 = X[0].cpu().numpy()
    for j in range(8):
        yj = X[1 + j].cpu().numpy()
        r = orc.dot_prod_multi(x0, [yj])[0]
        assert abs(d[j] - r) <= 1e-12 * np.abs(x0 * yj).sum()
    w = W.torch_uniform_device(n, seed=77, device=dev, lo=1e2, hi=1e8)
    v = G.nvec_wrms_norm(X[2], w)
    assert v == pytest.approx(orc.wrms_norm(X[2].cpu().numpy(), w.cpu().numpy()), rel=1e-12)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("shared", [True, False])
def test_wrms_norm_multi(orc, dev, G, n, shared):
    """WRMS norms of 5 vectors in one pass, with one shared weight vector or
    one per vector; each within 1e-12 relative of the oracle's WRMS norm of
    that vector (host and device results)."""
    nv = 5
    X = W.uniform_vectors(nv, n, seed=600 + n)
    Wv = [W.weight_vector(n, seed=700 + (0 if shared else j) + n) for j in range(nv)]
    Xd = [T(x, dev) for x in X]
    Wd = [T(w, dev) for w in Wv]
    if shared:
        Wd = [Wd[0]] * nv
    got = G.nvec_wrms_norm_multi(Xd, Wd)
    out = torch.empty(nv, dtype=torch.float64, device=dev)
    G.nvec_wrms_norm_multi(Xd, Wd, out=out)
    assert np.array_equal(np.array(got), out.cpu().numpy())
    for j in range(nv):
        ref = orc.wrms_norm(X[j], Wv[0] if shared else Wv[j]) if n else 0.0
        assert abs(got[j] - ref) <= 1e-12 * abs(ref)


def test_wrms_norm_multi_misaligned(orc, dev, G):
    n = 10001
    X = W.uniform_vectors(3, n + 1, seed=610)
    w = W.weight_vector(n + 1, seed=611)
    Xd = [T(x, dev)[1:] for x in X]
    wd = T(w, dev)[1:]
    got = G.nvec_wrms_norm_multi(Xd, [wd] * 3)
    for j in range(3):
        ref = orc.wrms_norm(X[j][1:], w[1:])
        assert abs(got[j] - ref) <= 1e-12 * ref
