"""Variable-coefficient BDF and the lazy Newton matrix on the GPU against
the oracle with the same options (the oracle's forms are pinned in
test_oracle_vc.py).

The coefficients are scalars the device controller forms from the past
step sizes; the kernels apply the interpolation-keeping order lowering in
the deferred history update, scale the order-(q+1) sum, and with the lazy
Newton matrix store and reload each cell's factors.  Trajectories are
compared in lockstep (parity_util.compare_trajectory, the bars derived
there; END_BAR_PER_STEP_LAZY for the lazy forms): attempts, Newton
iterations, order, setups and retries with fresh factors must agree step
by step while the step sizes agree.
"""
import numpy as np
import pytest
import torch

import workloads as W
from parity_util import (END_BAR_PER_STEP, END_BAR_PER_STEP_LAZY, compare_trajectory, gpu_bdf,
                         wrms_diff)

pytestmark = pytest.mark.gpu

FORMS = {
    "vc": dict(vc=True),
    "lazy": dict(lazy=True),
    "vc_lazy": dict(vc=True, lazy=True),
}


def bar(kw):
    return END_BAR_PER_STEP_LAZY if kw.get("lazy") else END_BAR_PER_STEP


@pytest.mark.parametrize("form", list(FORMS))
def test_trajectory_network10(orc, dev, G, form):
    kw = FORMS[form]
    ob, gb = compare_trajectory(orc, dev, G, W.random_network_batch(256, n=10, seed=31),
                                okw=kw, bar_per_step=bar(kw), **kw)
    s = gb.stats()
    print(form, {k: s[k] for k in ("nsteps", "nattempts", "nsetups", "nstale_retries")})
    if kw.get("lazy"):
        assert s["nsetups"] * 3 < s["nattempts"]


@pytest.mark.parametrize("form", list(FORMS))
def test_trajectory_robertson_bdf2(orc, dev, G, form):
    kw = FORMS[form]
    compare_trajectory(orc, dev, G, W.robertson_batch(1000), okw=kw, bar_per_step=bar(kw), **kw)


@pytest.mark.parametrize("form", ["vc_lazy"])
@pytest.mark.parametrize("solve", ["lu", "gauss_jordan"])
def test_trajectory_brusselator(orc, dev, G, form, solve):
    kw = FORMS[form]
    compare_trajectory(orc, dev, G, W.brusselator_batch(1000), okw=kw, bar_per_step=bar(kw),
                       linsol=G.LS_GJ if solve == "gauss_jordan" else G.LS_LU64, **kw)


def test_bench_kernel_vc_lazy_two_reduction_groups(orc, dev, G):
    """The network-specialised kernel of the benchmark network with both
    options, 20,000 cells (more than one reduction group, a ragged tile),
    150 steps in lockstep."""
    p = W.random_network_batch(20000, n=10, seed=W.BASE_SEED + 3)
    kw = FORMS["vc_lazy"]
    compare_trajectory(orc, dev, G, p, max_steps=150, okw=kw, bar_per_step=bar(kw), jit=True,
                       **kw)


@pytest.mark.parametrize("form", list(FORMS))
def test_pauses_do_not_change_the_run(dev, G, form):
    """Stopping every 37 steps (the pending history update is flushed and
    picked up again) gives the same run bit for bit as one call."""
    kw = FORMS[form]
    p = W.random_network_batch(1000, n=10, seed=41)
    a = gpu_bdf(G, p, dev, **kw)
    b = gpu_bdf(G, p, dev, **kw)
    assert a.advance(p.t_end, 370)[1] == 370
    for _ in range(10):
        assert b.advance(p.t_end, 37)[1] == 37
    sa, sb = a.stats(), b.stats()
    for k in ("nsteps", "nattempts", "nniters", "nsetups", "nstale_retries", "order_hist"):
        assert sa[k] == sb[k], k
    assert torch.equal(a.y(), b.y())


def test_lazy_reduces_setups_at_scale(dev, G):
    """2^16 cells of the benchmark network to t = 3e-5 (about 400 steps):
    the lazy form with variable coefficients sets up at most one attempt in
    5, and its error against a tight-tolerance run (rtol and atol 1e-3 of
    the problem's) is within 3x that of the eager fixed-coefficient run
    (both hold only their local errors to the tolerance)."""
    p = W.random_network_batch(1 << 16, n=10, seed=W.BASE_SEED + 3)
    t = 3e-5
    runs = {}
    for name, kw in (("eager", {}), ("vc_lazy", dict(vc=True, lazy=True)),
                     ("tight", dict(rtol=p.rtol * 1e-3, atol=p.atol * 1e-3))):
        b = gpu_bdf(G, p, dev, jit=True, **kw)
        assert b.integrate(t) == t
        runs[name] = (b.y().cpu().numpy(), b.stats())
        b.close()
    yr = runs["tight"][0]
    err = {k: wrms_diff(runs[k][0], yr, p.rtol, p.atol) for k in ("eager", "vc_lazy")}
    sa, sb = runs["eager"][1], runs["vc_lazy"][1]
    print(f"to t = {t:.1e}: eager {sa['nsteps']} steps {sa['nsetups']} setups, error "
          f"{err['eager']:.3e}; vc+lazy {sb['nsteps']} steps {sb['nsetups']} setups "
          f"{sb['nstale_retries']} retries, error {err['vc_lazy']:.3e}")
    assert sb["nsetups"] * 5 <= sb["nattempts"]
    assert err["vc_lazy"] <= 3.0 * err["eager"]


@pytest.mark.parametrize("form", list(FORMS))
def test_padded_sizes_and_classes(orc, dev, G, form):
    """Three thread-per-cell classes (4, 8 and 12 species) and a padded size
    (5 species in the 6-wide kernels), with the generated kernels."""
    kw = FORMS[form]
    for p in (W.uneven_batch(3000, seed=9, classes=(4, 8, 12), t_end=0.05),
              W.random_network_batch(300, n=5, seed=3, t_end=0.2)):
        compare_trajectory(orc, dev, G, p, okw=kw, bar_per_step=bar(kw), jit=True, **kw)


@pytest.mark.parametrize("map_small", [False, True])
def test_lazy_uneven_segment_classes(orc, dev, G, map_small):
    """The lazy Newton matrix on the uneven batch (4..64 species): the
    segment-per-cell classes (16..64 species; with map_small every class)
    store their FP64 factors, one row per lane, and reload them, while the
    thread-per-cell classes do so in their tiled layout, all with the
    separate history update; lockstep against the oracle with the same
    option, setups and retries compared step by step."""
    kw = dict(lazy=True)
    ob, gb = compare_trajectory(orc, dev, G, W.uneven_batch(1 << 12, seed=9), okw=kw,
                                bar_per_step=END_BAR_PER_STEP_LAZY, map_small=map_small, **kw)
    s = gb.stats()
    print({k: s[k] for k in ("nsteps", "nattempts", "nsetups", "nstale_retries")})
    assert s["nsetups"] * 3 < s["nattempts"]


@pytest.mark.parametrize("classes,total", [((14, 42), 2800), ((20, 40, 60), 3000)])
def test_lazy_segment_padded_rows(orc, dev, G, classes, total):
    """Segment classes whose species count is not the row width: 14, 20,
    42 and 60 species in rows of 16, 24, 48 and 64 columns (identity rows
    and columns past n are stored and reloaded with the factors)."""
    kw = dict(lazy=True)
    p = W.uneven_batch(total, seed=23, classes=classes, t_end=0.05)
    compare_trajectory(orc, dev, G, p, okw=kw, bar_per_step=END_BAR_PER_STEP_LAZY, **kw)


@pytest.mark.parametrize("map_small", [False, True])
def test_lazy_gauss_jordan_uneven(orc, dev, G, map_small):
    """The lazy Newton matrix with the Gauss-Jordan inverse on blocks of
    4..64 species: the setup kernel inverts in place and stores the plain
    inverse, the reuse kernel reloads its rows and applies them (v_readlane
    broadcasts in whole-wave segments, LDS in smaller ones); lockstep
    against the oracle's lazy Gauss-Jordan run."""
    kw = dict(lazy=True)
    ob, gb = compare_trajectory(orc, dev, G, W.uneven_batch(1 << 12, seed=9), okw=kw,
                                bar_per_step=END_BAR_PER_STEP_LAZY, map_small=map_small,
                                linsol=G.LS_GJ, **kw)
    s = gb.stats()
    print({k: s[k] for k in ("nsteps", "nattempts", "nsetups", "nstale_retries")})
    assert s["nsetups"] * 3 < s["nattempts"]


@pytest.mark.parametrize("classes,total", [((14, 42), 2800), ((20, 40, 60), 3000)])
def test_lazy_gauss_jordan_padded_rows(orc, dev, G, classes, total):
    kw = dict(lazy=True)
    p = W.uneven_batch(total, seed=23, classes=classes, t_end=0.05)
    compare_trajectory(orc, dev, G, p, okw=kw, bar_per_step=END_BAR_PER_STEP_LAZY,
                       linsol=G.LS_GJ, **kw)


@pytest.mark.parametrize("solve", ["lu", "gauss_jordan"])
def test_lazy_uneven_2p16_unknowns_bench_configuration(orc, dev, G, solve):
    """The lazy forms of the bench's uneven legs at 2^16 unknowns (about
    2,300 cells of 4..64 species, several blocks per class and reduction
    group) in the bench's launch configuration (graph mode, autotuned
    launch, generated kernels for the small classes): 80 steps in lockstep
    with the oracle's lazy run, setups and retries compared step by step."""
    p = W.uneven_batch(1 << 16, seed=W.BASE_SEED + 4)
    kw = dict(lazy=True)
    ob, gb = compare_trajectory(orc, dev, G, p, max_steps=80, okw=kw,
                                bar_per_step=END_BAR_PER_STEP_LAZY,
                                linsol=G.LS_GJ if solve == "gauss_jordan" else G.LS_LU64,
                                launch=G.LAUNCH_AUTO, mode=G.MODE_GRAPH, jit=True, **kw)
    s = gb.stats()
    print({k: s[k] for k in ("nsteps", "nattempts", "nsetups", "nstale_retries")})
    assert s["nsetups"] < s["nattempts"]

