"""GPU parity of the batched dense LU against the CPU oracle.

Per-block getrf semantics of the block-diagonal direct solve (Section 5).
Bar: identical pivots and info (continuous random data, no ties); factors
within 50 n u |A| of the oracle's; solutions within 50 n u cond(A) |x|;
FP32 refinement reaches the FP64 solution with the same per-block
fallback decisions as the oracle on well- and ill-conditioned blocks.
"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
CASES = [(1, 1), (3, 2), (37, 3), (1000, 3), (37, 5), (513, 10), (37, 16), (300, 21),
         (37, 33), (100, 64)]


def to_dev(A, dev, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(np.transpose(A, (0, 2, 1))), dtype=dtype, device=dev)


def from_dev(Ad):
    return np.transpose(Ad.cpu().numpy(), (0, 2, 1))


@pytest.mark.parametrize("nb,n", CASES)
def test_factor_solve_f64(orc, dev, G, nb, n):
    A = W.random_blocks(nb, n, seed=1000 + 7 * n + nb)
    B = W.rng_for(n + nb).uniform(-1, 1, (nb, n))
    Ad = to_dev(A, dev)
    piv = torch.empty(nb * n, dtype=torch.int32, device=dev)
    info = torch.empty(nb, dtype=torch.int32, device=dev)
    G.batched_lu_factor_f64(Ad, piv, info)
    LU, pv, inf = orc.lu_factor(A)
    assert np.array_equal(piv.cpu().numpy().reshape(nb, n), pv)
    assert np.array_equal(info.cpu().numpy(), inf)
    LUg = from_dev(Ad)
    scale = np.abs(A).max(axis=(1, 2))[:, None, None]
    growth = np.abs(LU).max(axis=(1, 2))[:, None, None]
    assert np.all(np.abs(LUg - LU) <= 50 * n * U * np.maximum(scale, growth) * (1 + np.abs(LU)))
    Bd = torch.tensor(B, device=dev)
    G.batched_lu_solve_f64(Ad, piv, Bd)
    X = orc.lu_solve(LU, pv, B)
    for b in range(nb):
        kap = np.linalg.cond(A[b], np.inf)
        assert np.abs(Bd[b].cpu().numpy() - X[b]).max() <= 50 * n * U * kap * np.abs(X[b]).max()


def test_singular_and_permutation(orc, dev, G):
    A = np.zeros((3, 4, 4))
    A[0] = np.array([[1, 2, 3, 4], [2, 4, 6, 8], [1, 0, 1, 0], [0, 1, 0, 1.0]])
    A[1] = np.eye(4)[[2, 0, 3, 1]]
    A[2] = 0.0
    Ad = to_dev(A, dev)
    piv = torch.empty(12, dtype=torch.int32, device=dev)
    info = torch.empty(3, dtype=torch.int32, device=dev)
    G.batched_lu_factor_f64(Ad, piv, info)
    LU, pv, inf = orc.lu_factor(A)
    assert np.array_equal(info.cpu().numpy(), inf)
    assert np.array_equal(piv.cpu().numpy().reshape(3, 4), pv)
    assert inf[2] == 1 and inf[1] == 0


@pytest.mark.parametrize("nb,n", [(37, 3), (513, 10), (300, 21), (50, 64)])
def test_factor_solve_f32(orc, dev, G, nb, n):
    A = W.random_blocks(nb, n, seed=3000 + n, diag_shift=2.0).astype(np.float32)
    Ad = to_dev(A, dev, torch.float32)
    piv = torch.empty(nb * n, dtype=torch.int32, device=dev)
    info = torch.empty(nb, dtype=torch.int32, device=dev)
    G.batched_lu_factor_f32(Ad, piv, info)
    LU, pv, inf = orc.lu_factor_f32(A)
    assert np.array_equal(piv.cpu().numpy().reshape(nb, n), pv)
    u32 = 2.0 ** -24
    assert np.allclose(from_dev(Ad), LU, rtol=0, atol=200 * n * u32 * np.abs(LU).max())
    B = W.rng_for(5).uniform(-1, 1, (nb, n)).astype(np.float32)
    Bd = torch.tensor(B, device=dev)
    G.batched_lu_solve_f32(Ad, piv, Bd)
    X = orc.lu_solve_f32(LU, pv, B)
    Xg = Bd.cpu().numpy()
    for b in range(nb):
        kap = np.linalg.cond(A[b].astype(np.float64), np.inf)
        assert np.abs(Xg[b] - X[b]).max() <= 50 * n * u32 * kap * np.abs(X[b]).max()


@pytest.mark.parametrize("nb,n", [(200, 10), (100, 21), (30, 64)])
def test_refinement(orc, dev, G, nb, n):
    rng = W.rng_for(n)
    A = W.random_blocks(nb, n, seed=4000 + n, diag_shift=3.0)
    # make a third of the blocks ill conditioned (cond ~ 1e9): must fall back
    for b in range(0, nb, 3):
        Q1, _ = np.linalg.qr(rng.normal(size=(n, n)))
        Q2, _ = np.linalg.qr(rng.normal(size=(n, n)))
        A[b] = (Q1 * np.logspace(0, -9, n)) @ Q2.T
    B = rng.uniform(-1, 1, (nb, n))
    Md = to_dev(A, dev)
    L32 = to_dev(A.astype(np.float32), dev, torch.float32)
    piv = torch.empty(nb * n, dtype=torch.int32, device=dev)
    info = torch.empty(nb, dtype=torch.int32, device=dev)
    G.batched_lu_factor_f32(L32, piv, info)
    Xd = torch.empty(nb, n, dtype=torch.float64, device=dev)
    sw = torch.empty(nb, dtype=torch.int32, device=dev)
    st = torch.empty(nb, dtype=torch.int32, device=dev)
    G.batched_lu_solve_refine(Md, L32, piv, torch.tensor(B, device=dev), Xd, 5, sw, st)
    Xo, sto, swo = orc.refine_solve(A, B, max_it=5)
    stg = st.cpu().numpy()
    assert np.all(stg[::3] == 1) and np.all(sto[::3] == 1)
    agree = np.mean(stg == sto)
    assert agree >= 0.95
    LU, pv, _ = orc.lu_factor(A)
    X64 = orc.lu_solve(LU, pv, B)
    Xg = Xd.cpu().numpy()
    for b in range(nb):
        kap = np.linalg.cond(A[b], np.inf)
        assert np.abs(Xg[b] - X64[b]).max() <= 50 * n * U * kap * np.abs(X64[b]).max()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_uneven_block_sizes_var(orc, dev, G, dtype):
    """Blocks of sizes 1..64 (the uneven batch's classes plus odd sizes) packed
    one after the other, factored and solved in one launch each: per block
    the pivots and info of the oracle, factors and solutions to the bars of
    the uniform calls; an out-of-range size gets info = -1 and is untouched."""
    rng = W.rng_for(77)
    sizes = [int(s) for s in rng.choice([1, 3, 4, 8, 13, 16, 24, 32, 48, 64], size=90)]
    sizes[5] = 65                               # outside 0..nmax: rejected per block
    nmax = 64
    f64 = dtype == "f64"
    tdt, ndt = (torch.float64, np.float64) if f64 else (torch.float32, np.float32)
    u = U if f64 else 2.0 ** -24
    blocks = [W.random_blocks(1, n, seed=5000 + i, diag_shift=0.0 if f64 else 2.0)[0].astype(ndt)
              for i, n in enumerate(sizes)]
    packed = np.concatenate([b.ravel(order="F") for b in blocks])
    rhs = [rng.uniform(-1, 1, n).astype(ndt) for n in sizes]
    Ad = torch.tensor(packed, dtype=tdt, device=dev)
    Bd = torch.tensor(np.concatenate(rhs), dtype=tdt, device=dev)
    piv = torch.full((sum(sizes),), -7, dtype=torch.int32, device=dev)
    info = torch.empty(len(sizes), dtype=torch.int32, device=dev)
    G.batched_lu_factor_var(Ad, piv, info, sizes, nmax=nmax)
    G.batched_lu_solve_var(Ad, piv, Bd, sizes, nmax=nmax)
    LUg, pg, ig, xg = Ad.cpu().numpy(), piv.cpu().numpy(), info.cpu().numpy(), Bd.cpu().numpy()
    mo = vo = 0
    for i, n in enumerate(sizes):
        A = blocks[i]
        if n > nmax:
            assert ig[i] == -1
            assert np.array_equal(LUg[mo:mo + n * n], packed[mo:mo + n * n])
            assert np.all(pg[vo:vo + n] == -7)
        else:
            fac = orc.lu_factor if f64 else orc.lu_factor_f32
            sol = orc.lu_solve if f64 else orc.lu_solve_f32
            LU, pv, inf = fac(A[None])
            assert ig[i] == inf[0]
            assert np.array_equal(pg[vo:vo + n], pv[0])
            L = LUg[mo:mo + n * n].reshape(n, n, order="F")
            scale = max(np.abs(A).max(), np.abs(LU).max())
            assert np.all(np.abs(L - LU[0]) <= 200 * n * u * scale * (1 + np.abs(LU[0])))
            X = sol(LU, pv, rhs[i][None])[0]
            kap = np.linalg.cond(A.astype(np.float64), np.inf)
            assert np.abs(xg[vo:vo + n] - X).max() <= 50 * n * u * kap * np.abs(X).max()
        mo += n * n
        vo += n
