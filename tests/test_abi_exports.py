"""The C-ABI library loads and exports every entry point include/*.h
declares (no compute: this runs without a GPU)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2011_12984_amd", "libbdfgpu.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z][A-Za-z0-9_]*)\s*\(",
                             txt, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("nvec_linear_sum", "nvec_linear_combination", "nvec_scale_add_multi",
                     "nvec_dot_prod_multi", "nvec_wrms_norm", "batched_lu_factor_f64",
                     "batched_lu_solve_f64", "batched_lu_solve_refine", "bdf_create", "bdf_step",
                     "bdf_integrate", "bdf_destroy"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_names_match_header():
    from paper_2011_12984_amd import _lib
    assert set(_lib.SIGNATURES) == set(declared_functions())


def test_no_oracle_in_product_sources():
    """The product path never links, includes or imports the oracle."""
    pkg = os.path.join(ROOT, "paper_2011_12984_amd")
    for path in glob.glob(os.path.join(pkg, "**", "*"), recursive=True):
        if os.path.isdir(path) or path.endswith((".so", ".o", ".pyc")):
            continue
        txt = open(path, errors="ignore").read()
        assert "orc_" not in txt and "import oracle" not in txt and "liborc" not in txt, path


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_workspace_bytes_without_device_memory():
    """bdf_workspace_bytes is a dry run of the creation: it needs no device
    memory or GPU and grows with the number of cells."""
    import workloads as W
    from paper_2011_12984_amd import Bdf
    small = Bdf.workspace_bytes(W.random_network_batch(100, n=10, seed=1))
    big = Bdf.workspace_bytes(W.random_network_batch(10000, n=10, seed=1))
    # history (6 vectors), saved correction, 3 iterates and the rates: at
    # least 8 (10 n + R) bytes per cell
    assert big - small >= 8 * (10 * 10 + 20) * 9900
    assert Bdf.workspace_bytes(W.random_network_batch(100, n=10, seed=1), qmax=9) == 0


def test_gauss_jordan_and_order3_option_checks():
    """Option checks of the dry run: the Gauss-Jordan block inverse is
    accepted on per-class launches for blocks of any size (one lane per
    cell up to 4 species, a segment beyond; per-cell stepping only in the
    first case) and refused on one launch over all classes; a reaction of
    order three (the demonstration reaction's 2u + v -> 3u) is refused by
    the FP32 LU with refinement, whose matrix-free product covers order
    <= 2."""
    import workloads as W
    from paper_2011_12984_amd import LS_GJ, LS_LU32REF, LAUNCH_FUSED, Bdf
    br = W.brusselator_batch(100)
    assert Bdf.workspace_bytes(br, linsol=LS_GJ) > 0
    assert Bdf.workspace_bytes(br, linsol=LS_GJ, per_cell=True) > 0
    assert Bdf.workspace_bytes(br, linsol=LS_GJ, launch=LAUNCH_FUSED) == 0
    net = W.random_network_batch(100, n=10, seed=1)
    assert Bdf.workspace_bytes(net, linsol=LS_GJ) > 0
    assert Bdf.workspace_bytes(net, linsol=LS_GJ, per_cell=True) == 0
    assert Bdf.workspace_bytes(W.uneven_batch(1 << 12, seed=9), linsol=LS_GJ) > 0
    assert Bdf.workspace_bytes(net, linsol=LS_GJ, lazy=True) > Bdf.workspace_bytes(net, linsol=LS_GJ)
    assert Bdf.workspace_bytes(br, linsol=LS_LU32REF) == 0


def test_variable_coefficient_and_lazy_option_checks():
    """vc needs the deferred history update (thread-per-cell classes,
    per-class launches, grouped stepping); lazy takes any class size with
    per-class launches and grouped stepping, and needs FP64 LU or the
    Gauss-Jordan solve; the stored factors are counted in the workspace
    (segment classes: n rounded up to 8, squared, per cell)."""
    import numpy as np
    import workloads as W
    from paper_2011_12984_amd import LAUNCH_FUSED, LS_GJ, LS_LU32REF, Bdf
    net = W.random_network_batch(1000, n=10, seed=1)
    base = Bdf.workspace_bytes(net)
    lazy = Bdf.workspace_bytes(net, lazy=True)
    assert Bdf.workspace_bytes(net, vc=True) == base
    assert lazy - base >= 1000 * (10 * 10 * 8 + 10 * 4)
    assert Bdf.workspace_bytes(net, vc=True, lazy=True) == lazy
    assert Bdf.workspace_bytes(net, vc=True, linsol=LS_LU32REF) > 0
    assert Bdf.workspace_bytes(net, lazy=True, linsol=LS_LU32REF) == 0
    assert Bdf.workspace_bytes(W.brusselator_batch(100), lazy=True, linsol=LS_GJ) > 0
    assert Bdf.workspace_bytes(net, vc=True, defer=False) == 0
    assert Bdf.workspace_bytes(net, lazy=True, per_cell=True) == 0
    assert Bdf.workspace_bytes(net, lazy=True, launch=LAUNCH_FUSED) == 0
    assert Bdf.workspace_bytes(net, lazy=True, defer=False) > 0
    un = W.uneven_batch(1 << 12, seed=9)
    assert Bdf.workspace_bytes(un, vc=True) == 0
    sizes = np.array([un.topologies[t][0].shape[1] for t in un.cell_topo])
    spc = sum(((n + 7) // 8 * 8) ** 2 * 8 + ((n + 7) // 8 * 8) * 4 for n in sizes if n > 12)
    assert Bdf.workspace_bytes(un, lazy=True) - Bdf.workspace_bytes(un) >= spc
    assert Bdf.workspace_bytes(un, lazy=True, launch=LAUNCH_FUSED) == 0


def test_gmres_option_checks():
    """GMRES: thread-per-cell classes, per-class launches, stream mode,
    fixed coefficients; the Krylov basis (6 vectors), the predicted state,
    weights, iterate and the preconditioner's factors are counted in the
    workspace."""
    import workloads as W
    from paper_2011_12984_amd import LS_GMRES, MODE_GRAPH, Bdf
    net = W.random_network_batch(1000, n=10, seed=1)
    base = Bdf.workspace_bytes(net)
    kry = Bdf.workspace_bytes(net, linsol=LS_GMRES)
    assert kry - base >= 1024 * 10 * 8 * (6 + 4) + 1000 * (10 * 10 * 8)
    assert Bdf.workspace_bytes(net, linsol=LS_GMRES, lazy=True) == kry
    assert Bdf.workspace_bytes(net, linsol=LS_GMRES, vc=True) == 0
    assert Bdf.workspace_bytes(net, linsol=LS_GMRES, mode=MODE_GRAPH) == 0
    assert Bdf.workspace_bytes(net, linsol=LS_GMRES, per_cell=True) == 0
    assert Bdf.workspace_bytes(W.uneven_batch(1 << 12, seed=9), linsol=LS_GMRES) == 0
    assert Bdf.workspace_bytes(W.brusselator_batch(100), linsol=LS_GMRES) > 0
