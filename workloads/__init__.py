"""Seeded synthetic inputs for the batched stiff-ODE workloads.

This module only draws random numbers and lays them out; it holds none of
the integrator's arithmetic.  Both the CPU oracle tests and the GPU library
tests/benchmark take their inputs from here, so the two sides always see the
same arrays.

Grouping many small independent systems into one large ODE with a block
diagonal Jacobian is the paper's "submodel" use case (Section 2, Fig.
blockdiag_jacobian); vectors are cell-major: cell c owns the contiguous
entries [off_c, off_c + n_c).

Networks are mass-action networks given by two integer matrices of shape
(R, n): ``nu[k, s]`` is the number of molecules of species s consumed by
reaction k and ``mu[k, s]`` the number produced.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 20240

SIZE_CLASSES = (4, 8, 16, 24, 32, 48, 64)


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# Network topologies
# --------------------------------------------------------------------------

def robertson_topology():
    """Reactions A->B, 2B->B+C, B+C->A+C over species (A, B, C)."""
    nu = np.array([[1, 0, 0],
                   [0, 2, 0],
                   [0, 1, 1]], dtype=np.int32)
    mu = np.array([[0, 1, 0],
                   [0, 1, 1],
                   [1, 0, 1]], dtype=np.int32)
    return nu, mu


ROBERTSON_RATES = np.array([0.04, 3.0e7, 1.0e4])


# The reaction term of the paper's demonstration problem (a brusselator
# variant, Section 7): with u, v, w the three concentrations,
#   u' = A - (w + 1) u + v u^2,  v' = w u - v u^2,  w' = (B - w)/eps - w u,
# A = 1, B = 3.5, eps = 5e-6, written as mass-action reactions over
# (u, v, w): 0 -> u (rate A), u -> 0 (1), u + w -> v (1), 2u + v -> 3u (1),
# 0 -> w (B/eps), w -> 0 (1/eps).
BRUSSELATOR_A, BRUSSELATOR_B, BRUSSELATOR_EPS = 1.0, 3.5, 5e-6


def brusselator_topology():
    nu = np.array([[0, 0, 0], [1, 0, 0], [1, 0, 1], [2, 1, 0], [0, 0, 0], [0, 0, 1]],
                  dtype=np.int32)
    mu = np.array([[1, 0, 0], [0, 0, 0], [0, 1, 0], [3, 0, 0], [0, 0, 1], [0, 0, 0]],
                  dtype=np.int32)
    return nu, mu


def brusselator_rates(A=BRUSSELATOR_A, B=BRUSSELATOR_B, eps=BRUSSELATOR_EPS):
    return np.array([A, 1.0, 1.0, 1.0, B / eps, 1.0 / eps])


def random_network(n: int, R: int, rng: np.random.Generator):
    """Random count-conserving mass-action network.

    Each reaction has order o drawn uniformly from {1, 2}; o reactant and o
    product species are drawn uniformly with replacement; a reaction whose
    product multiset equals its reactant multiset is redrawn.
    """
    nu = np.zeros((R, n), dtype=np.int32)
    mu = np.zeros((R, n), dtype=np.int32)
    k = 0
    while k < R:
        o = int(rng.integers(1, 3))
        reac = rng.integers(0, n, size=o)
        prod = rng.integers(0, n, size=o)
        if sorted(reac.tolist()) == sorted(prod.tolist()):
            continue
        for s in reac:
            nu[k, s] += 1
        for s in prod:
            mu[k, s] += 1
        k += 1
    return nu, mu


def linear_chain_topology(n: int):
    """First-order reactions s -> s+1 (s < n-1) and n-1 -> 0: a linear ODE."""
    nu = np.zeros((n, n), dtype=np.int32)
    mu = np.zeros((n, n), dtype=np.int32)
    for s in range(n):
        nu[s, s] = 1
        mu[s, (s + 1) % n] = 1
    return nu, mu


# --------------------------------------------------------------------------
# Value draws
# --------------------------------------------------------------------------

def log_uniform(rng, lo_exp: float, hi_exp: float, size):
    return 10.0 ** rng.uniform(lo_exp, hi_exp, size=size)


def simplex_states(rng, ncells: int, n: int):
    y = rng.uniform(0.0, 1.0, size=(ncells, n))
    y /= y.sum(axis=1, keepdims=True)
    return y


def robertson_states(rng, ncells: int, signed_jitter: bool = False):
    """(1, 0, 0) plus a 1e-3 jitter.  B and C stay non-negative unless the
    literal signed reading is requested."""
    y = np.zeros((ncells, 3))
    y[:, 0] = 1.0 + rng.uniform(-1e-3, 1e-3, size=ncells)
    lo = -1e-3 if signed_jitter else 0.0
    y[:, 1] = rng.uniform(lo, 1e-3, size=ncells)
    y[:, 2] = rng.uniform(lo, 1e-3, size=ncells)
    return y


def uneven_sizes(rng, total: int, classes=SIZE_CLASSES):
    """Block sizes drawn uniformly from `classes` until fewer than max(classes)
    unknowns remain; the remainder is filled with blocks of the smallest
    size.  With all classes multiples of 4 and total a multiple of 4 the sum
    is exactly `total`."""
    sizes = []
    rem = total
    cls = np.asarray(classes)
    while rem >= cls.max():
        s = int(cls[rng.integers(0, len(cls))])
        sizes.append(s)
        rem -= s
    small = int(cls.min())
    assert rem % small == 0
    sizes.extend([small] * (rem // small))
    return np.asarray(sizes, dtype=np.int32)


# --------------------------------------------------------------------------
# Workload bundles
# --------------------------------------------------------------------------

class Problem(dict):
    """Plain dict with attribute access.

    Keys: topologies (list of (nu, mu)), cell_topo (int32[ncells]),
    rates (float64 concatenated per cell, R_c values each), y0 (float64
    concatenated, n_c values each), rtol, atol, t0, t_end, qmax, nonneg
    (non-negativity constraints on), label.
    """
    __getattr__ = dict.__getitem__

    @property
    def ncells(self):
        return int(len(self["cell_topo"]))

    @property
    def sizes(self):
        n_of = np.array([nu.shape[1] for nu, _ in self["topologies"]], dtype=np.int32)
        return n_of[self["cell_topo"]]

    @property
    def nreact(self):
        r_of = np.array([nu.shape[0] for nu, _ in self["topologies"]], dtype=np.int32)
        return r_of[self["cell_topo"]]

    @property
    def N(self):
        return int(self.sizes.sum())

    @property
    def uniform_n(self):
        s = self.sizes
        return int(s[0]) if len(s) and np.all(s == s[0]) else None


def robertson_batch(ncells: int = 1000, seed: int = BASE_SEED + 1,
                    signed_jitter: bool = False) -> Problem:
    """1,000 independent 3-species Robertson-type systems; per-cell rate
    constants log-uniform in [1e-2, 1e7]; fixed-order BDF2 to t = 10."""
    rng = rng_for(seed)
    nu, mu = robertson_topology()
    rates = log_uniform(rng, -2.0, 7.0, (ncells, 3))
    y0 = robertson_states(rng, ncells, signed_jitter)
    return Problem(topologies=[(nu, mu)], cell_topo=np.zeros(ncells, np.int32),
                   rates=rates.ravel().copy(), y0=y0.ravel().copy(),
                   rtol=1e-6, atol=1e-10, t0=0.0, t_end=10.0, qmax=2,
                   nonneg=True, label=f"robertson{ncells}x3")


def random_network_batch(ncells: int, n: int = 10, seed: int = BASE_SEED + 3,
                         lo_exp: float = -3.0, hi_exp: float = 8.0,
                         shared_rates: bool = False, qmax: int = 5,
                         t_end: float = 10.0) -> Problem:
    """ncells cells sharing one random network of n species and 2n
    reactions; rates log-uniform per cell (or one vector for all cells);
    initial states uniform on the simplex."""
    rng = rng_for(seed)
    R = 2 * n
    nu, mu = random_network(n, R, rng)
    if shared_rates:
        k = log_uniform(rng, lo_exp, hi_exp, R)
        rates = np.tile(k, ncells)
    else:
        rates = log_uniform(rng, lo_exp, hi_exp, (ncells, R)).ravel()
    y0 = simplex_states(rng, ncells, n).ravel()
    return Problem(topologies=[(nu, mu)], cell_topo=np.zeros(ncells, np.int32),
                   rates=rates.copy(), y0=y0.copy(), rtol=1e-6, atol=1e-10,
                   t0=0.0, t_end=t_end, qmax=qmax, nonneg=True,
                   label=f"net{ncells}x{n}")


def brusselator_batch(ncells: int, length: float = 10.0, t_end: float = 10.0,
                      rtol: float = 1e-6, atol: float = 1e-10) -> Problem:
    """The demonstration problem's reaction term at `ncells` points of the
    domain [0, length] (cell centres), each cell an independent 3-species
    system: the initial profile u = A + p, v = B/A + p, w = 3 + p with
    p = 0.1 exp(-(x - length/2)^2 / (2 (length/4)^2)); rates as in
    brusselator_rates for every cell.  (The advection coupling between
    cells is not part of this workload.)"""
    A, B = BRUSSELATOR_A, BRUSSELATOR_B
    x = (np.arange(ncells) + 0.5) * (length / ncells)
    mu_, sig = length / 2.0, length / 4.0
    pert = 0.1 * np.exp(-((x - mu_) ** 2) / (2.0 * sig * sig))
    y0 = np.stack([A + pert, B / A + pert, 3.0 + pert], axis=1)
    nu, mu = brusselator_topology()
    rates = np.tile(brusselator_rates(), ncells)
    return Problem(topologies=[(nu, mu)], cell_topo=np.zeros(ncells, np.int32),
                   rates=rates, y0=y0.ravel().copy(), rtol=rtol, atol=atol, t0=0.0,
                   t_end=t_end, qmax=5, nonneg=False, label=f"brusselator{ncells}")


def uneven_batch(total_unknowns: int, seed: int = BASE_SEED + 4,
                 classes=SIZE_CLASSES, lo_exp: float = -3.0,
                 hi_exp: float = 8.0, t_end: float = 10.0) -> Problem:
    """Cells with block sizes drawn uniformly from `classes` summing to
    total_unknowns; one random network (2n reactions) per size class."""
    rng = rng_for(seed)
    sizes = uneven_sizes(rng, total_unknowns, classes)
    topologies = []
    topo_of = {}
    for s in sorted(set(int(x) for x in classes)):
        topo_of[s] = len(topologies)
        topologies.append(random_network(s, 2 * s, rng))
    cell_topo = np.array([topo_of[int(s)] for s in sizes], dtype=np.int32)
    rates = []
    y0 = []
    for s in sizes:
        rates.append(log_uniform(rng, lo_exp, hi_exp, 2 * int(s)))
        y0.append(simplex_states(rng, 1, int(s))[0])
    return Problem(topologies=topologies, cell_topo=cell_topo,
                   rates=np.concatenate(rates), y0=np.concatenate(y0),
                   rtol=1e-6, atol=1e-10, t0=0.0, t_end=t_end, qmax=5,
                   nonneg=True, label=f"uneven{total_unknowns}")


def learned_batch(ncells: int, n: int = 21, seed: int = BASE_SEED + 5,
                  t_end: float = 10.0) -> Problem:
    """One 21-species network with one rate vector shared by every cell;
    cells differ only in their initial state."""
    p = random_network_batch(ncells, n=n, seed=seed, shared_rates=True,
                             t_end=t_end)
    p["label"] = f"learned{ncells}x{n}"
    return p


def linear_chain_batch(ncells: int, n: int, seed: int, lo_exp=-2.0,
                       hi_exp=7.0, t_end=10.0, qmax=5) -> Problem:
    """First-order chain networks: y' = A_c y with A_c = S diag(k_c) nu."""
    rng = rng_for(seed)
    nu, mu = linear_chain_topology(n)
    rates = log_uniform(rng, lo_exp, hi_exp, (ncells, n)).ravel()
    y0 = simplex_states(rng, ncells, n).ravel()
    return Problem(topologies=[(nu, mu)], cell_topo=np.zeros(ncells, np.int32),
                   rates=rates.copy(), y0=y0.copy(), rtol=1e-6, atol=1e-10,
                   t0=0.0, t_end=t_end, qmax=qmax, label=f"chain{ncells}x{n}")


# --------------------------------------------------------------------------
# Vectors for the fused-operation microbenchmark
# --------------------------------------------------------------------------

def uniform_vectors(count: int, length: int, seed: int, lo=-1.0, hi=1.0):
    rng = rng_for(seed)
    return rng.uniform(lo, hi, size=(count, length))


def weight_vector(length: int, seed: int, lo=1e2, hi=1e8):
    rng = rng_for(seed)
    return rng.uniform(lo, hi, size=length)


def uniform_coefficients(count: int, seed: int, lo=-1.0, hi=1.0):
    rng = rng_for(seed)
    return rng.uniform(lo, hi, size=count)


def random_blocks(nb: int, n: int, seed: int, diag_shift: float = 0.0):
    """nb dense n x n blocks, entries U(-1, 1), optional diagonal shift;
    returned as an (nb, n, n) array in row-major mathematical order."""
    rng = rng_for(seed)
    A = rng.uniform(-1.0, 1.0, size=(nb, n, n))
    if diag_shift:
        A += diag_shift * np.eye(n)[None]
    return A


def torch_uniform_device(shape, seed: int, device, lo=-1.0, hi=1.0,
                         dtype=None):
    """Large vectors drawn directly in device memory with torch's seeded
    generator (used where host generation would dominate run time)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    t = torch.empty(shape, dtype=dtype or torch.float64, device=device)
    t.uniform_(lo, hi, generator=g)
    return t


# --------------------------------------------------------------------------
# Initial weights of the learned preconditioner's MLP
# --------------------------------------------------------------------------

def mlp_init(n: int, hid: int = 256, seed: int = BASE_SEED + 6, out_scale: float = 1.0):
    """He-uniform initial weights (limit sqrt(6 / fan_in)), zero biases, as
    one FP32 array laid out W1 (hid x (n+1)) | b1 | W2 (hid x hid) | b2 |
    W3 (n^2 x hid) | b3, row-major.  out_scale multiplies W3 (a small value
    starts training near X = I)."""
    rng = rng_for(seed)
    nin, nout = n + 1, n * n

    def he(fan_in, shape):
        lim = np.sqrt(6.0 / fan_in)
        return rng.uniform(-lim, lim, size=shape)

    W1 = he(nin, (hid, nin))
    W2 = he(hid, (hid, hid))
    W3 = he(hid, (nout, hid)) * out_scale
    parts = [W1.ravel(), np.zeros(hid), W2.ravel(), np.zeros(hid), W3.ravel(), np.zeros(nout)]
    return np.concatenate(parts).astype(np.float32)


def mlp_split(params, n: int, hid: int = 256):
    """Views (W1, b1, W2, b2, W3, b3) of a flat parameter array."""
    nin, nout = n + 1, n * n
    shapes = [(hid, nin), (hid,), (hid, hid), (hid,), (nout, hid), (nout,)]
    out, o = [], 0
    for s in shapes:
        k = int(np.prod(s))
        out.append(np.asarray(params[o:o + k]).reshape(s))
        o += k
    assert o == len(params)
    return out
