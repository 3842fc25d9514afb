"""Newton-Krylov (linsol GMRES) on the GPU against the oracle's.

Every Newton system is solved over all cells by right-preconditioned GMRES
scaled by the error weights, with the cells' LU factors at the last setup
as block-Jacobi preconditioner; the host drives the Krylov iteration and
the kernels apply the operator, the preconditioner and the inner
products (test_oracle_krylov.py pins the oracle's).  Trajectories are
compared in lockstep (parity_util.compare_trajectory): attempts, Newton
iterations, order, setups and the GMRES iteration count agree step by
step while the step sizes agree.
"""
import numpy as np
import pytest

import workloads as W
from parity_util import END_BAR_PER_STEP, END_BAR_PER_STEP_LAZY, compare_trajectory, gpu_bdf, wrms_diff

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("lazy", [False, True])
def test_trajectory_network10(orc, dev, G, lazy):
    p = W.random_network_batch(256, n=10, seed=31, t_end=0.2)
    ob, gb = compare_trajectory(orc, dev, G, p, linsol=G.LS_GMRES, okw=dict(lazy=lazy),
                                bar_per_step=END_BAR_PER_STEP_LAZY if lazy else END_BAR_PER_STEP,
                                lazy=lazy)
    s = gb.stats()
    print({k: s[k] for k in ("nsteps", "nattempts", "nsetups", "nniters", "nliters")})
    assert s["nliters"] > 0
    if not lazy:
        assert s["nliters"] <= s["nniters"]      # P = M: one iteration per solve


def test_trajectory_robertson_lazy(orc, dev, G):
    compare_trajectory(orc, dev, G, W.robertson_batch(1000), linsol=G.LS_GMRES,
                       okw=dict(lazy=True), bar_per_step=END_BAR_PER_STEP_LAZY, lazy=True)


def test_trajectory_brusselator_lazy(orc, dev, G):
    compare_trajectory(orc, dev, G, W.brusselator_batch(1000), linsol=G.LS_GMRES,
                       okw=dict(lazy=True), bar_per_step=END_BAR_PER_STEP_LAZY, lazy=True)


def test_krylov_at_scale_is_as_accurate(dev, G):
    """2^16 cells of the benchmark network to t = 1e-5 with the lazy
    preconditioner: error against a tight-tolerance run within 3x that of
    the direct solve, with fewer setups than attempts."""
    p = W.random_network_batch(1 << 16, n=10, seed=W.BASE_SEED + 3)
    t = 1e-5
    runs = {}
    for name, kw in (("lu", {}), ("gmres", dict(linsol=G.LS_GMRES, lazy=True)),
                     ("tight", dict(rtol=p.rtol * 1e-3, atol=p.atol * 1e-3))):
        b = gpu_bdf(G, p, dev, **kw)
        assert b.integrate(t) == t
        runs[name] = (b.y().cpu().numpy(), b.stats())
        b.close()
    yr = runs["tight"][0]
    err = {k: wrms_diff(runs[k][0], yr, p.rtol, p.atol) for k in ("lu", "gmres")}
    sg = runs["gmres"][1]
    print(f"errors: LU {err['lu']:.3e}, GMRES {err['gmres']:.3e}; GMRES {sg['nsteps']} steps, "
          f"{sg['nattempts']} attempts, {sg['nsetups']} setups, {sg['nniters']} Newton and "
          f"{sg['nliters']} Krylov iterations")
    assert err["gmres"] <= 3.0 * err["lu"] + 0.1
    assert sg["nsetups"] < sg["nattempts"]


@pytest.mark.parametrize("lazy", [False, True])
def test_krylov_padded_sizes_and_classes(orc, dev, G, lazy):
    """Three thread-per-cell classes (4, 8 and 12 species) in one Krylov
    space, and a padded size (5 species in the 6-wide kernels)."""
    for p in (W.uneven_batch(3000, seed=9, classes=(4, 8, 12), t_end=0.05),
              W.random_network_batch(300, n=5, seed=3, t_end=0.2)):
        compare_trajectory(orc, dev, G, p, linsol=G.LS_GMRES, okw=dict(lazy=lazy),
                           bar_per_step=END_BAR_PER_STEP_LAZY if lazy else END_BAR_PER_STEP,
                           lazy=lazy)
