"""nvec_dot_prod_multi_noalloc (static per-device scratch, no allocation)
against nvec_dot_prod_multi, through the C ABI.

Both run the same reduction kernels, so the results must be bitwise equal;
they are also held to the dot-product bar against the oracle,
|d - d_ref| <= 1e-12 * sum_i |x_i y_i|.  Two calls in a row, the second on
a smaller input (fewer blocks: the finishing kernel must read only the
partials the second call wrote), then length 0 and an out-of-range nv.
"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _check(orc, G, dev, n, nv, seed):
    X = W.uniform_vectors(nv + 1, n, seed=seed)
    xd = torch.tensor(X[0], device=dev)
    Yd = [torch.tensor(X[j + 1], device=dev) for j in range(nv)]
    out_na = torch.full((nv,), np.nan, dtype=torch.float64, device=dev)
    out_ref = torch.full((nv,), np.nan, dtype=torch.float64, device=dev)
    G.nvec_dot_prod_multi_noalloc(xd, Yd, out_na)
    got = out_na.cpu().numpy()
    G.nvec_dot_prod_multi(xd, Yd, out=out_ref)
    ref_gpu = out_ref.cpu().numpy()
    assert np.array_equal(got, ref_gpu), (got, ref_gpu)
    ref = orc.dot_prod_multi(X[0], list(X[1:]))
    bound = 1e-12 * np.abs(X[0][None, :] * X[1:]).sum(1)
    assert np.all(np.abs(got - ref) <= bound)


def test_noalloc_two_calls_then_smaller(orc, dev, G):
    # 2^22 + 5 elements: the grid fills all 8192 blocks and loops over tiles
    _check(orc, G, dev, (1 << 22) + 5, 8, seed=901)
    # second call, smaller: 4099 elements over a few blocks, 3 vectors
    _check(orc, G, dev, 4099, 3, seed=902)


def test_noalloc_misaligned(orc, dev, G):
    n = 70001
    X = W.uniform_vectors(3, n + 1, seed=903)
    base = [torch.tensor(x, device=dev) for x in X]
    xd, Yd = base[0][1:], [b[1:] for b in base[1:]]   # 8-byte offset: scalar kernels
    out = torch.empty(2, dtype=torch.float64, device=dev)
    G.nvec_dot_prod_multi_noalloc(xd, Yd, out)
    ref = orc.dot_prod_multi(X[0][1:], [x[1:] for x in X[1:]])
    bound = 1e-12 * np.abs(X[0][None, 1:] * X[1:, 1:]).sum(1)
    assert np.all(np.abs(out.cpu().numpy() - ref) <= bound)


def test_noalloc_empty_and_bad_nv(dev, G):
    x = torch.empty(0, dtype=torch.float64, device=dev)
    out = torch.full((4,), 7.0, dtype=torch.float64, device=dev)
    G.nvec_dot_prod_multi_noalloc(x, [x] * 4, out)
    assert out.cpu().numpy().tolist() == [0.0] * 4
    y = torch.ones(16, dtype=torch.float64, device=dev)
    with pytest.raises(G.BdfGpuError) as e:
        G.nvec_dot_prod_multi_noalloc(y, [y] * 9, torch.empty(9, dtype=torch.float64, device=dev))
    assert e.value.code == -1
