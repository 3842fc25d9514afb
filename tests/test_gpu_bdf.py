"""GPU parity of the grouped BDF integrator against the CPU oracle.

Grouped Newton with block-diagonal solves and whole-step retry (Section 7);
the BDF method itself is the fixed-coefficient Nordsieck reading.  Bars:
mass-action f and J within 1e-13 of the oracle (relative to the term
scale); one step from an identical state makes the same decisions and
lands within 1e-6 in WRMS units; trajectories are compared in lockstep
(parity_util.compare_trajectory): while every decision (attempts, Newton
iterations, order) agrees the states at common times agree within
1e-3 + 2e-5 per step WRMS (the rounding of the unconverged Newton iterates,
derived and measured in parity_util) and the step-size drift is printed; a
decision taken differently at a threshold is printed with the oracle's
threshold quantities, and the runs must then end equally accurate against a
tight-tolerance oracle run (the GPU's error within 3x the oracle's); graph
capture reproduces stream execution bit for bit.
"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


from parity_util import compare_trajectory, gpu_bdf, wrms_diff


def jac_entries(prob):
    return int((prob.sizes.astype(np.int64) ** 2).sum())


@pytest.mark.parametrize("maker", [
    lambda: W.robertson_batch(37),
    lambda: W.random_network_batch(300, n=10, seed=5),
    lambda: W.learned_batch(70),
    lambda: W.uneven_batch(1 << 12, seed=9),
    lambda: W.brusselator_batch(500),   # a reaction of order three
])
def test_rhs_jac_parity(orc, dev, G, maker):
    p = maker()
    b = gpu_bdf(G, p, dev)
    rng = W.rng_for(3)
    y = rng.uniform(0.0, 1.0, p.N)
    f, J = b.eval_rhs_jac(torch.tensor(y, device=dev), jac_entries(p))
    f, J = f.cpu().numpy(), J.cpu().numpy()
    sizes, R = p.sizes, p.nreact
    yo = ro = jo = 0
    for c in range(p.ncells):
        n, r = int(sizes[c]), int(R[c])
        nu, mu = p.topologies[p.cell_topo[c]]
        k = p.rates[ro:ro + r]
        fr = orc.ma_rhs(nu, mu, k, y[yo:yo + n])
        Jr = orc.ma_jac(nu, mu, k, y[yo:yo + n])
        scale = np.abs(k).sum() * 4
        assert np.abs(f[yo:yo + n] - fr).max() <= 1e-13 * scale
        Jg = J[jo:jo + n * n].reshape(n, n).T
        assert np.abs(Jg - Jr).max() <= 1e-13 * scale
        yo, ro, jo = yo + n, ro + r, jo + n * n


def test_single_step_from_identical_state(orc, dev, G):
    p = W.random_network_batch(512, n=10, seed=21)
    ob = orc.Bdf(p)
    for _ in range(30):
        assert ob.step(p.t_end) == 0
    sc = ob.scalars()
    z, dprev = ob.history()
    gb = gpu_bdf(G, p, dev)
    gb.set_state(sc["t"], sc["h"], sc["q"], sc["qwait"], torch.tensor(z, device=dev),
                 torch.tensor(dprev, device=dev))
    s0 = ob.stats()
    assert ob.step(p.t_end) == 0
    s1 = ob.stats()
    gb.step(p.t_end)
    gs = gb.stats()
    st = gb.get_state()
    sc1 = ob.scalars()
    assert gs["nattempts"] == s1["nattempts"] - s0["nattempts"]
    assert gs["nniters"] == s1["nniters"] - s0["nniters"]
    assert st["q"] == sc1["q"]
    assert st["t"] == pytest.approx(sc1["t"], rel=1e-14)
    assert st["h"] == pytest.approx(sc1["h"], rel=1e-12)
    z1, _ = ob.history()
    assert wrms_diff(st["z"][0].cpu().numpy(), z1[0], p.rtol, p.atol) <= 1e-6


def test_trajectory_robertson_bdf2(orc, dev, G):
    compare_trajectory(orc, dev, G, W.robertson_batch(1000))


@pytest.mark.parametrize("solve", ["lu", "gauss_jordan"])
def test_trajectory_brusselator(orc, dev, G, solve):
    """The demonstration reaction of Section 7 on 1,000 cells of the 1-D
    Gaussian profile, to t = 10, with the FP64 LU or the explicit
    Gauss-Jordan block inverse on both sides."""
    compare_trajectory(orc, dev, G, W.brusselator_batch(1000),
                       linsol=G.LS_GJ if solve == "gauss_jordan" else G.LS_LU64)


def test_gauss_jordan_differs_from_lu_by_rounding_only(dev, G):
    """The Gauss-Jordan handle really applies the explicit inverse (its
    state is not bit-identical to the LU handle's) and takes the same steps
    to a state within 1e-6 WRMS of it."""
    p = W.brusselator_batch(4096)
    a = gpu_bdf(G, p, dev, linsol=G.LS_GJ)
    b = gpu_bdf(G, p, dev, linsol=G.LS_LU64)
    assert a.integrate(p.t_end) == p.t_end and b.integrate(p.t_end) == p.t_end
    assert a.stats()["nsteps"] == b.stats()["nsteps"]
    ya, yb = a.y(), b.y()
    assert not torch.equal(ya, yb)
    assert wrms_diff(ya.cpu().numpy(), yb.cpu().numpy(), p.rtol, p.atol) <= 1e-6


def test_trajectory_network10(orc, dev, G):
    compare_trajectory(orc, dev, G, W.random_network_batch(256, n=10, seed=31))


def test_trajectory_network10_fp32_refined(orc, dev, G):
    ob, gb = compare_trajectory(orc, dev, G, W.random_network_batch(256, n=10, seed=31), linsol=1)
    assert gb.stats()["refine_sweeps"] > 0


@pytest.mark.parametrize("launch,map_small,linsol", [
    (0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 1), (1, 0, 1)])
def test_trajectory_uneven(orc, dev, G, launch, map_small, linsol):
    """Blocks of 4..64 species: per-class launches or one launch over every
    class, thread per cell or 16-lane segments for the small classes, FP64
    or FP32-refined LU."""
    compare_trajectory(orc, dev, G, W.uneven_batch(1 << 12, seed=9), launch=launch,
                       map_small=map_small, linsol=linsol)


@pytest.mark.parametrize("map_small", [0, 1])
def test_trajectory_uneven_gauss_jordan(orc, dev, G, map_small):
    """The Gauss-Jordan block inverse on blocks of 4..64 species: one lane
    per cell for 4 species (or a 16-lane segment with map_small), one row
    per lane of a segment beyond (in-place elimination over the lanes, the
    inverse applied as a matrix-vector product), against the oracle's
    Gauss-Jordan on the augmented block."""
    compare_trajectory(orc, dev, G, W.uneven_batch(1 << 12, seed=9), map_small=map_small,
                       linsol=G.LS_GJ)


@pytest.mark.parametrize("classes,total", [((14, 42), 2800), ((20, 40, 60), 3000)])
def test_trajectory_gauss_jordan_padded_rows(orc, dev, G, classes, total):
    """Segment classes whose species count is not the row width (14, 20,
    42 and 60 species in rows of 16, 24, 48 and 64 columns): the identity
    rows and columns past n take part in the elimination."""
    p = W.uneven_batch(total, seed=23, classes=classes, t_end=0.05)
    compare_trajectory(orc, dev, G, p, linsol=G.LS_GJ)


@pytest.mark.parametrize("launch", [0, 1])
def test_trajectory_uneven_fp32_fallback_path(orc, dev, G, launch):
    """One refinement sweep allowed: a block that needs a second one to pass
    the FP64 residual test goes to FP64 LU for the rest of the attempt, so
    the classes (4..64 species) run the FP64 fallback inside their
    FP32-refined Newton kernels."""
    p = W.uneven_batch(1 << 12, seed=9)
    assert int(np.max(p.sizes)) == 64
    ob, gb = compare_trajectory(orc, dev, G, p, launch=launch, linsol=1, refine_max_it=1)
    st = gb.stats()
    print("fallbacks", st["refine_fallbacks"], "sweeps", st["refine_sweeps"])
    assert st["refine_fallbacks"] > 0


def test_fused_launch_graph_bitwise_equal_to_stream(dev, G):
    p = W.uneven_batch(1 << 13, seed=19)
    a = gpu_bdf(G, p, dev, mode=G.MODE_STREAM, launch=G.LAUNCH_FUSED, linsol=1)
    b = gpu_bdf(G, p, dev, mode=G.MODE_GRAPH, launch=G.LAUNCH_FUSED, linsol=1,
                attempts_per_sync=5)
    for t in (1e-3, 1e-1, p.t_end):
        a.integrate(t)
        b.integrate(t)
    assert a.stats()["nsteps"] == b.stats()["nsteps"]
    assert torch.equal(a.y(), b.y())


def test_autotune_keeps_the_fastest_candidate(orc, dev, G):
    p = W.uneven_batch(1 << 12, seed=29)
    b = gpu_bdf(G, p, dev, launch=G.LAUNCH_AUTO, linsol=1, mode=G.MODE_GRAPH)
    tu = b.tuning()
    print(tu)
    ms = tu["ms_per_step"]
    assert len(ms) >= 2          # both small-block mappings, and the launch modes possible
    best = min(ms, key=ms.get)
    assert (tu["launch"], tu["map_small"]) == best
    assert b.integrate(p.t_end) == p.t_end
    ob = orc.Bdf(p, linsol=1)
    assert ob.integrate(p.t_end) == 0
    ref = orc.Bdf(p, rtol=p.rtol * 1e-3, atol=p.atol * 1e-3)
    assert ref.integrate(p.t_end) == 0
    yr = ref.y()
    eg = wrms_diff(b.y().cpu().numpy(), yr, p.rtol, p.atol)
    eo = wrms_diff(ob.y(), yr, p.rtol, p.atol)
    assert eg <= max(3.0 * eo, 1.0)


def test_trajectory_n21(orc, dev, G):
    compare_trajectory(orc, dev, G, W.learned_batch(64, seed=12))


@pytest.mark.parametrize("map_small", [0, 1])
def test_small_odd_sizes(orc, dev, G, map_small):
    # n = 1 (padded thread-per-cell), n = 5, and a ragged last tile
    for n, cells in ((1, 65), (5, 130), (2, 3)):
        p = W.linear_chain_batch(cells, n, seed=n)
        compare_trajectory(orc, dev, G, p, map_small=map_small)


def test_graph_mode_bitwise_equal_to_stream(dev, G):
    p = W.random_network_batch(1000, n=10, seed=41)
    a = gpu_bdf(G, p, dev, mode=G.MODE_STREAM)
    b = gpu_bdf(G, p, dev, mode=G.MODE_GRAPH, attempts_per_sync=3)
    a.integrate(1.0)
    b.integrate(1.0)
    b.integrate(p.t_end)     # graph replays across several host checks
    a.integrate(p.t_end)
    assert a.stats()["nsteps"] == b.stats()["nsteps"]
    assert torch.equal(a.y(), b.y())


def test_step_by_step_equals_integrate(dev, G):
    p = W.robertson_batch(100)
    a = gpu_bdf(G, p, dev)
    b = gpu_bdf(G, p, dev)
    a.integrate(1e-2)
    t = 0.0
    n = 0
    while t < 1e-2:
        t = b.step(1e-2)
        n += 1
    assert n == a.stats()["nsteps"] == b.stats()["nsteps"]
    assert torch.equal(a.y(), b.y())


def test_max_steps_error(dev, G):
    p = W.robertson_batch(10)
    b = gpu_bdf(G, p, dev, max_steps=4)
    with pytest.raises(G.BdfGpuError) as e:
        b.integrate(10.0)
    assert e.value.code == -4          # too much work


def test_conservation_without_projection(dev, G):
    # the method keeps sum(y) to rounding; a short horizon keeps every cell
    # away from the negative-concentration regime
    p = W.random_network_batch(4096, n=10, seed=8, t_end=1e-3)
    b = gpu_bdf(G, p, dev, nonneg=False)
    b.integrate(p.t_end)
    y = b.y().cpu().numpy().reshape(-1, 10)
    assert np.abs(y.sum(1) - p.y0.reshape(-1, 10).sum(1)).max() <= 1e-12


def test_projection_matches_oracle(orc, dev, G):
    """y >= 0 projection on a 1,024-cell batch that triggers it thousands of
    times: lockstep parity with the oracle's projected run, every component
    non-negative, and the mass the projection adds (the clipped negative
    parts, tolerance-level amounts summed along the path) of the same order
    as the oracle's: the largest per-cell drift within 10x the oracle's and
    the mean within 3x.  The drift is a property of the trajectory (1.2e-7
    in the worst cell for the oracle itself; the two runs separate at a
    step-size decision, after which each cell clips along its own path), so
    it is held to the oracle's rather than to a fixed bound."""
    p = W.random_network_batch(1024, n=10, seed=8)
    ob, gb = compare_trajectory(orc, dev, G, p)
    y = gb.y().cpu().numpy().reshape(-1, 10)
    yo = ob.y().reshape(-1, 10)
    assert y.min() >= 0.0
    assert gb.stats()["nprojections"] > 0 and ob.stats()["nprojections"] > 0
    m0 = p.y0.reshape(-1, 10).sum(1)
    dg, do = np.abs(y.sum(1) - m0), np.abs(yo.sum(1) - m0)
    print(f"mass drift: gpu max {dg.max():.3e} mean {dg.mean():.3e}, "
          f"oracle max {do.max():.3e} mean {do.mean():.3e}")
    assert dg.max() <= 10 * do.max()
    assert dg.mean() <= 3 * do.mean()


def test_bench_kernel_parity_two_reduction_groups(orc, dev, G):
    """The network-specialised Newton kernel the benchmark times, on 20,000
    cells of the benchmark's network (313 one-wave blocks: two first-level
    reduction groups, the last one ragged), 150 steps in lockstep with the
    oracle."""
    p = W.random_network_batch(20000, n=10, seed=W.BASE_SEED + 3)
    compare_trajectory(orc, dev, G, p, max_steps=150, jit=True)


def test_uneven_parity_2p16_unknowns(orc, dev, G):
    """Uneven batch at 2^16 unknowns (about 2,300 cells of 4..64 species,
    several blocks per class and reduction group), FP32-refined LU, graph
    mode and the autotuned launch, 40 steps in lockstep with the oracle."""
    p = W.uneven_batch(1 << 16, seed=W.BASE_SEED + 4)
    compare_trajectory(orc, dev, G, p, max_steps=40, linsol=1, launch=G.LAUNCH_AUTO,
                       mode=G.MODE_GRAPH, jit=True)


@pytest.mark.parametrize("linsol,jit", [(0, True), (1, False)])
def test_deferred_update_matches_separate_update(dev, G, linsol, jit):
    """The history update applied by the next attempt's Newton kernel (the
    default for thread-per-cell classes) against the separate update kernel:
    per cell the same operations on the same values; only the order
    selection's two norms are summed in another reduction tree, which can
    move a growth factor in its last bits (and, over thousands of steps,
    separate the step-size sequences as any rounding does).  Over the first
    300 steps, with a pause after 150 (the flush and resume path): the same
    steps, attempts, Newton iterations and orders, step sizes to 1e-12 and
    states within 1e-8 WRMS."""
    p = W.random_network_batch(1000, n=10, seed=41)
    a = gpu_bdf(G, p, dev, linsol=linsol, jit=jit, defer=True)
    b = gpu_bdf(G, p, dev, linsol=linsol, jit=jit, defer=False)
    for _ in range(2):
        ta, na = a.advance(p.t_end, 150)
        tb, nb = b.advance(p.t_end, 150)
        assert na == nb == 150
    sa, sb = a.stats(), b.stats()
    print({k: (sa[k], sb[k]) for k in ("nsteps", "nattempts", "nniters", "netfails", "nncfails")})
    for k in ("nsteps", "nattempts", "nniters", "order_hist"):
        assert sa[k] == sb[k], k
    assert sa["h"] == pytest.approx(sb["h"], rel=1e-12)
    assert sa["t"] == pytest.approx(sb["t"], rel=1e-12)
    d = wrms_diff(a.y().cpu().numpy(), b.y().cpu().numpy(), p.rtol, p.atol)
    print(f"deferred vs separate update after 300 steps: wrms diff {d:.3e}")
    assert d <= 1e-8
    assert sa["order_hist"][3] > 0          # the order selection ran (and raised)


@pytest.mark.parametrize("prob,kw", [
    ("net10", dict(jit=True)),                 # one lane per cell, deferred history update
    ("uneven", dict(linsol=1)),                # segment classes, FP32-refined LU
    ("uneven", dict(linsol=0, lazy=True)),     # lazy Newton matrix: setup and reuse kernels
])
def test_newton_continuation_launches_bitwise(dev, G, prob, kw):
    """An attempt's Newton iterations split over launches (1, 2 or all 3 per
    launch; a later launch continues from the stored iterate and forms the
    predictor, J and the factors again) give the same trajectory bit for
    bit: the same counters, t, h and states after 300 steps.  The
    one-iteration-per-launch run takes continuation launches, the
    all-in-one run none."""
    p = (W.random_network_batch(1000, n=10, seed=41) if prob == "net10"
         else W.uneven_batch(1 << 12, seed=9))
    runs = []
    for npl in (1, 2, 3):
        b = gpu_bdf(G, p, dev, newton_per_launch=npl, **kw)
        _, taken = b.advance(p.t_end, 300)
        assert taken == 300
        runs.append((b.stats(), b.y().cpu()))
        b.close()
    print({npl: (s["nattempts"], s["nniters"], s["ncont"]) for npl, (s, _) in zip((1, 2, 3), runs)})
    s1, y1 = runs[0]
    assert s1["ncont"] > 0 and runs[2][0]["ncont"] == 0
    for s, y in runs[1:]:
        for k in ("nsteps", "nattempts", "nniters", "netfails", "nncfails", "order_hist"):
            assert s[k] == s1[k], k
        assert s["t"] == s1["t"] and s["h"] == s1["h"]
        assert torch.equal(y, y1)


@pytest.mark.parametrize("kw", [dict(jit=True), dict(linsol=1, launch=2, mode=1)])
def test_caller_workspace(dev, G, kw):
    """A handle whose device state lives in caller memory sized by
    bdf_workspace_bytes reproduces the library-allocated handle bit for bit;
    a workspace one byte short is refused with the workspace status."""
    p = W.random_network_batch(3000, n=10, seed=43) if "launch" not in kw else \
        W.uneven_batch(1 << 12, seed=9)
    need = G.Bdf.workspace_bytes(p, **kw)
    assert need > 0
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    a = gpu_bdf(G, p, dev, workspace=ws, **kw)
    b = gpu_bdf(G, p, dev, **kw)
    for t in (1e-3, 1e-1):
        assert a.integrate(t) == t and b.integrate(t) == t
    assert a.stats()["nsteps"] == b.stats()["nsteps"]
    assert torch.equal(a.y(), b.y())
    a.close()
    small = torch.empty(need - 1, dtype=torch.uint8, device=dev)
    with pytest.raises(G.BdfGpuError) as e:
        gpu_bdf(G, p, dev, workspace=small, **kw)
    assert e.value.code == -3
