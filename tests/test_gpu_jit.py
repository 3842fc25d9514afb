"""Network-specialised Newton kernels (bdf_create with jit) against the
generic table-driven kernel.

The generated f, J and (I - gamma J) x perform the same floating-point
operations in the same order as the table-driven ones (terms with a zero
stoichiometric coefficient, which add +-0 exactly, are left out), so whole
trajectories must agree bit for bit: same step counts, same final state.
The generic kernel is itself held to the oracle in test_gpu_bdf.py.  Cases
cover padded block sizes (5 -> 6, 9 -> 10), several classes at once, a
reaction of order three, the three block solves, graph replay, and the compiled-library caches (per
process, and on disk under BDFGPU_JIT_DIR).
"""
import os
import time

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "robertson3": (lambda: W.robertson_batch(300), 1.0),
    "net10": (lambda: W.random_network_batch(1000, n=10, seed=41), 1.0),
    "net5_padded6": (lambda: W.random_network_batch(700, n=5, seed=3), 1.0),
    "net9_padded10": (lambda: W.random_network_batch(500, n=9, seed=4), 0.5),
    "net12": (lambda: W.random_network_batch(400, n=12, seed=6), 0.5),
    "uneven_4_8_12": (lambda: W.uneven_batch(6000, seed=9, classes=(4, 8, 12)), 0.2),
    "brusselator3": (lambda: W.brusselator_batch(2000), 10.0),   # order-3 reaction
}


def run(G, p, dev, t_end, **kw):
    b = G.Bdf.from_problem(p, device=dev, **kw)
    b.integrate(t_end)
    st, y = b.stats(), b.y().clone()
    b.close()
    return st, y


def check_equal(G, dev, name, linsol, **kw):
    maker, t_end = CASES[name]
    p = maker()
    sa, ya = run(G, p, dev, t_end, linsol=linsol, **kw)
    sb, yb = run(G, p, dev, t_end, linsol=linsol, jit=True, **kw)
    keys = ("nsteps", "nattempts", "nniters", "nncfails", "netfails", "refine_sweeps",
            "refine_fallbacks", "nprojections")
    print(name, {k: (sa[k], sb[k]) for k in keys})
    assert sa["nsteps"] > 10
    for k in keys:
        assert sa[k] == sb[k], k
    assert torch.equal(ya, yb)


@pytest.mark.parametrize("name", list(CASES))
def test_jit_bitwise_equal_to_generic_lu64(dev, G, name):
    check_equal(G, dev, name, G.LS_LU64)


@pytest.mark.parametrize("name", ["net10", "net5_padded6"])
def test_jit_bitwise_equal_to_generic_lu32_refined(dev, G, name):
    check_equal(G, dev, name, G.LS_LU32REF)


def test_jit_bitwise_equal_to_generic_gauss_jordan(dev, G):
    check_equal(G, dev, "brusselator3", G.LS_GJ)


def test_jit_graph_replay_and_library_cache(dev, G, tmp_path):
    """Graph capture of the generated kernel's launch reproduces stream
    execution; a second handle on the same network reuses the library
    loaded by the first, and a fresh cache directory gets the compiled
    library and its build log."""
    p = W.random_network_batch(2000, n=8, seed=17)
    old = os.environ.get("BDFGPU_JIT_DIR")
    os.environ["BDFGPU_JIT_DIR"] = str(tmp_path / "jit")
    try:
        t0 = time.perf_counter()
        a = G.Bdf.from_problem(p, device=dev, jit=True)
        t_first = time.perf_counter() - t0
        t0 = time.perf_counter()
        b = G.Bdf.from_problem(p, device=dev, jit=True, mode=G.MODE_GRAPH, attempts_per_sync=3)
        t_second = time.perf_counter() - t0
    finally:
        if old is None:
            del os.environ["BDFGPU_JIT_DIR"]
        else:
            os.environ["BDFGPU_JIT_DIR"] = old
    print(f"create with compile {t_first:.2f} s, from cache {t_second:.2f} s")
    libs = list((tmp_path / "jit").glob("*/net.so"))
    assert len(libs) == 1 and (libs[0].parent / "build.log").exists()
    assert t_second < 0.5 * t_first
    a.integrate(0.5)
    b.integrate(0.5)
    assert a.stats()["nsteps"] == b.stats()["nsteps"]
    assert torch.equal(a.y(), b.y())
    a.close()
    b.close()
