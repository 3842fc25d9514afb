"""Per-cell adaptive stepping against the oracle run on each cell alone.

With per-cell stepping every cell is its own ODE (its own step size,
order, Newton and error tests on norms over its own species), so a cell's
trajectory is exactly the grouped method's trajectory for a problem made
of that one cell, which is what the oracle integrates.  Cells whose step
and attempt counts and last step size agree with the oracle's have end
states within the bars below; cells where a threshold decision went the
other way, or whose step sizes drifted apart, are judged by their error
against a tight-tolerance oracle run of the cell (check_cells).
"""
import numpy as np
import pytest
import torch

import workloads as W
from parity_util import FLIP_ERR_RATIO, FLIP_H, wrms_diff

# Cells with the oracle's decisions: end-state differences (WRMS over the
# cell).  A single cell's WRMS is not averaged over many cells, so the
# rounding of the unconverged Newton iterates that the lockstep bar allows
# per step shows fully in the worst cells.  Measured (median / 90th
# percentile / max): 10-species network 8.6e-7 / 3.8e-4 / 0.25 over 96
# cells, 4-species 5.7e-7 / 1.3e-3 / 0.17, Robertson 4.9e-9 / 5.5e-8 /
# 1.9e-6: typical cells agree to rounding, the worst to a fraction of the
# tolerance.
SAME_MEDIAN = 1e-3
SAME_MAX = 0.5

pytestmark = pytest.mark.gpu


def one_cell(p, c):
    """The problem made of cell c of p alone."""
    n = int(p.sizes[c])
    R = int(p.nreact[c])
    yo = int(p.sizes[:c].sum())
    ro = int(p.nreact[:c].sum())
    q = W.Problem(dict(p))
    q["cell_topo"] = np.array([p.cell_topo[c]], np.int32)
    q["rates"] = np.ascontiguousarray(p.rates[ro:ro + R])
    q["y0"] = np.ascontiguousarray(p.y0[yo:yo + n])
    q["label"] = f"{p.label}[{c}]"
    return q


def check_cells(orc, G, dev, p, cells, **kw):
    """Per-cell GPU run against the oracle on each listed cell alone.
    Cells with the oracle's step and attempt counts and last step size
    (relative difference <= FLIP_H): end-state differences (WRMS over the
    cell) with median <= SAME_MEDIAN and maximum <= SAME_MAX; cells where a
    decision went the other way, or whose step sizes drifted apart beyond
    FLIP_H (the same rounding-driven drift the lockstep comparison
    treats as a flip, with the same number of steps taken on different
    sizes): the largest GPU error against
    a tight-tolerance run of the cell within FLIP_ERR_RATIO of the largest
    oracle error over all listed cells (a single cell's global error at this
    tolerance is a few WRMS units, and which cells flip is a matter of
    rounding, so errors are compared as distributions)."""
    lin = kw.get("linsol", 0)
    b = G.Bdf.from_problem(p, device=dev, per_cell=True, **kw)
    assert b.integrate(p.t_end) == p.t_end
    y = b.y().cpu().numpy()
    counts, tc, hug = b.cell_stats(with_hu=True)
    assert np.all(tc == p.t_end)
    s = b.stats()
    assert s["nsteps"] == counts[:, 0].sum()
    offs = np.concatenate([[0], np.cumsum(p.sizes)])
    same, eg_flip, eo_all = [], [], []
    for c in cells:
        q = one_cell(p, c)
        ob = orc.Bdf(q, linsol=lin)
        assert ob.integrate(q.t_end) == 0
        so = ob.stats()
        yg = y[offs[c]:offs[c + 1]]
        yo = ob.y()
        ref = orc.Bdf(q, rtol=q.rtol * 1e-3, atol=q.atol * 1e-3)
        assert ref.integrate(q.t_end) == 0
        yr = ref.y()
        eg, eo = wrms_diff(yg, yr, p.rtol, p.atol), wrms_diff(yo, yr, p.rtol, p.atol)
        eo_all.append(eo)
        hu_o = ob.scalars()["hu"]
        drift = abs(hug[c] - hu_o) / abs(hu_o)
        if so["nsteps"] == counts[c, 0] and so["nattempts"] == counts[c, 1] and drift <= FLIP_H:
            same.append(wrms_diff(yg, yo, p.rtol, p.atol))
        else:
            eg_flip.append(eg)
            print(f"  cell {c}: steps oracle {so['nsteps']} gpu {counts[c, 0]}, last step size "
                  f"relative difference {drift:.2e}; error vs tight reference gpu {eg:.3e} "
                  f"oracle {eo:.3e}")
    same = np.array(same)
    print(f"{p.label}: {len(cells)} cells checked; {len(same)} with the oracle's step and "
          f"attempt counts, end-state difference median "
          f"{np.median(same) if len(same) else 0:.3e} p90 "
          f"{np.quantile(same, 0.9) if len(same) else 0:.3e} max {same.max() if len(same) else 0:.3e};"
          f" {len(eg_flip)} with a different decision or drifted step size, largest GPU error "
          f"{max(eg_flip) if eg_flip else 0:.3e} vs largest oracle error {max(eo_all):.3e}; "
          f"per-cell steps min {counts[:, 0].min()} median {int(np.median(counts[:, 0]))} "
          f"max {counts[:, 0].max()}")
    assert len(same) >= len(cells) // 2
    assert np.median(same) <= SAME_MEDIAN and same.max() <= SAME_MAX
    if eg_flip:
        assert max(eg_flip) <= FLIP_ERR_RATIO * max(eo_all)
    return b, counts


def test_per_cell_network10(orc, dev, G):
    p = W.random_network_batch(200, n=10, seed=W.BASE_SEED + 3)
    b, counts = check_cells(orc, G, dev, p, range(0, 200, 2))
    assert counts[:, 0].min() < counts[:, 0].max()   # the cells really step on their own


def test_per_cell_robertson_bdf2(orc, dev, G):
    p = W.robertson_batch(130)
    check_cells(orc, G, dev, p, range(130))


@pytest.mark.parametrize("solve", ["lu", "gauss_jordan"])
def test_per_cell_brusselator(orc, dev, G, solve):
    """The demonstration reaction (order three) with the cells stepping on
    their own, FP64 LU or the Gauss-Jordan inverse on both sides."""
    p = W.brusselator_batch(300)
    check_cells(orc, G, dev, p, range(0, 300, 3),
                linsol=G.LS_GJ if solve == "gauss_jordan" else G.LS_LU64)


def test_per_cell_padded_sizes_and_classes(orc, dev, G):
    """Two classes (4 and 8 species) and a padded size (5 species in the
    6-wide kernel), cells interleaved in user order."""
    a = W.random_network_batch(70, n=4, seed=61, t_end=1.0)
    c5 = W.random_network_batch(70, n=5, seed=62, t_end=1.0)
    for p in (a, c5):
        check_cells(orc, G, dev, p, range(0, 70, 3))
    u = W.uneven_batch(600, seed=63, classes=(4, 8), t_end=1.0)
    check_cells(orc, G, dev, u, range(0, u.ncells, 5))


def test_per_cell_continues_to_a_later_end(orc, dev, G):
    """Integrating to 1e-2 and then to t_end equals one integration to t_end
    whenever the cell's steps do not straddle 1e-2 (tstop clamps at 1e-2
    change the step sequence otherwise): the oracle does the same two calls."""
    p = W.random_network_batch(64, n=10, seed=7)
    b = G.Bdf.from_problem(p, device=dev, per_cell=True)
    assert b.integrate(1e-2) == 1e-2
    _, t1 = b.cell_stats()
    assert np.all(t1 == 1e-2)
    assert b.integrate(p.t_end) == p.t_end
    y = b.y().cpu().numpy()
    counts, _ = b.cell_stats()
    for c in range(0, 64, 4):
        q = one_cell(p, c)
        ob = orc.Bdf(q)
        assert ob.integrate(1e-2) == 0 and ob.integrate(q.t_end) == 0
        if ob.stats()["nsteps"] == counts[c, 0]:
            d = wrms_diff(y[10 * c:10 * c + 10], ob.y(), p.rtol, p.atol)
            assert d <= SAME_MAX


def test_per_cell_refuses_grouped_only_calls(dev, G):
    p = W.random_network_batch(10, n=10, seed=1)
    b = G.Bdf.from_problem(p, device=dev, per_cell=True)
    with pytest.raises(G.BdfGpuError):
        b.step(1.0)
    with pytest.raises(G.BdfGpuError):
        G.Bdf.from_problem(W.uneven_batch(1 << 10, seed=2), device=dev, per_cell=True)
