"""Seeded synthetic spin-glass instances.

This module only builds inputs: coupling graphs, coupling values, fields,
3-spin hyper-couplings, optional explicit colourings and request traces.  It
holds none of the minimiser's arithmetic (no energies, fields, flips, random
starts or colouring algorithm), so both the CPU oracle and the HIP library can
be fed from it without sharing any computation.

Instances follow the hyper-Ising model of the paper (Sec. II eq. (1) and
Sec. VI eq. (5), restricted to couplings over 2 and 3 spins):

    E(s) = - sum_edges J_ij s_i s_j - sum_i h_i s_i - sum_triples K_ijk s_i s_j s_k

Lattices use one periodic wrap per dimension (Sec. II, boundary conditions).
Coupling distributions: the paper uses Gaussian or +-1 bimodal couplings
(Sec. II); this project keeps every value an integer so that energies are
exact, using +-1 and bounded integer ranges.
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Instance", "lattice", "chimera", "erdos_renyi_triples", "random_regular3",
    "ferromagnet", "gauge", "chain", "random_small", "complete_graph",
    "cfg1_square16", "cfg1_square4", "cfg2_cubic100", "cfg3_chimera_batch",
    "cfg4_uneven_batch", "cfg4_sizes", "cfg5_trace", "serving_instance",
]


@dataclasses.dataclass
class Instance:
    """One instance: undirected edges (ei, ej, J), fields h, triples (tri, K).

    All arrays are int32.  ``colour`` is an explicit proper colouring or None
    (then each solver computes its own first-fit colouring).  ``instance_id``
    is the RNG key word that identifies the instance; ``restarts`` is the
    number of independent random starts.
    """

    n: int
    ei: np.ndarray
    ej: np.ndarray
    J: np.ndarray
    h: Optional[np.ndarray] = None
    tri: Optional[np.ndarray] = None  # shape (t, 3)
    K: Optional[np.ndarray] = None
    colour: Optional[np.ndarray] = None
    instance_id: int = 0
    restarts: int = 1
    name: str = ""
    dims: Optional[tuple] = None      # lattice hint (periodic extents) passed to the solver, or None

    def __post_init__(self):
        self.ei = np.ascontiguousarray(self.ei, dtype=np.int32)
        self.ej = np.ascontiguousarray(self.ej, dtype=np.int32)
        self.J = np.ascontiguousarray(self.J, dtype=np.int32)
        if self.h is not None:
            self.h = np.ascontiguousarray(self.h, dtype=np.int32)
        if self.tri is None:
            self.tri = np.zeros((0, 3), dtype=np.int32)
            self.K = np.zeros(0, dtype=np.int32)
        self.tri = np.ascontiguousarray(np.asarray(self.tri, dtype=np.int32).reshape(-1, 3))
        self.K = np.ascontiguousarray(self.K, dtype=np.int32)
        if self.colour is not None:
            self.colour = np.ascontiguousarray(self.colour, dtype=np.int32)

    @property
    def m(self) -> int:
        return int(self.ei.shape[0])

    @property
    def t(self) -> int:
        return int(self.tri.shape[0])

    def h_or_zero(self) -> np.ndarray:
        return self.h if self.h is not None else np.zeros(self.n, dtype=np.int32)

    def replace(self, **kw) -> "Instance":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------
# building blocks


def _rng(seed) -> np.random.Generator:
    return np.random.default_rng(seed)


def _pm1(rng, size) -> np.ndarray:
    return np.where(rng.random(size) < 0.5, -1, 1).astype(np.int32)


def lattice(dims: Sequence[int], periodic=True, seed=0, j_values=(-1, 1),
            h_range: Optional[tuple] = None, checkerboard=True,
            instance_id=0, restarts=1, name="", hint=False) -> Instance:
    """d-dimensional hypercubic lattice, row-major site index (last axis fastest).

    Every site has one bond in the + direction of each axis; with ``periodic``
    the last site of an axis bonds to the first (one wrap per dimension, paper
    Sec. II).  Periodic axes need length >= 3 so that no pair is bonded twice.
    J is drawn uniformly from ``j_values``; h uniformly from the integer range
    ``h_range`` (inclusive) or absent.  With even periodic lengths (or open
    boundaries) the explicit colouring is the checkerboard sum(coords) mod 2.
    """
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    rng = _rng(seed)
    idx = np.arange(n, dtype=np.int64).reshape(dims)
    ei_l, ej_l = [], []
    for ax, L in enumerate(dims):
        if periodic and L < 3:
            raise ValueError("a periodic axis needs length >= 3")
        nb = np.roll(idx, -1, axis=ax)
        src = idx
        if not periodic:
            sl = [slice(None)] * len(dims)
            sl[ax] = slice(0, L - 1)
            src = idx[tuple(sl)]
            nb = nb[tuple(sl)]
        ei_l.append(src.reshape(-1))
        ej_l.append(nb.reshape(-1))
    # interleave so bonds of one site are adjacent: order (site, axis)
    ei = np.stack(ei_l, axis=1).reshape(-1) if periodic else np.concatenate(ei_l)
    ej = np.stack(ej_l, axis=1).reshape(-1) if periodic else np.concatenate(ej_l)
    jv = np.asarray(j_values, dtype=np.int32)
    J = jv[rng.integers(0, len(jv), size=ei.shape[0])]
    h = None
    if h_range is not None:
        h = rng.integers(h_range[0], h_range[1] + 1, size=n).astype(np.int32)
    colour = None
    if checkerboard and (not periodic or all(L % 2 == 0 for L in dims)):
        coords = np.indices(dims).reshape(len(dims), -1)
        colour = (coords.sum(axis=0) % 2).astype(np.int32)
    return Instance(n=n, ei=ei, ej=ej, J=J, h=h, colour=colour,
                    instance_id=instance_id, restarts=restarts,
                    name=name or "lattice" + "x".join(map(str, dims)),
                    dims=tuple(dims) if hint and periodic else None)


@functools.lru_cache(maxsize=16)
def _chimera_edges_cached(rows, cols):
    n, ei, ej = _chimera_edges_build(rows, cols)
    ei.setflags(write=False)
    ej.setflags(write=False)
    return n, ei, ej


def chimera_edges(rows=8, cols=8):
    """Chimera-like grid of K4,4 cells (see _chimera_edges_build)."""
    return _chimera_edges_cached(int(rows), int(cols))


def _chimera_edges_build(rows=8, cols=8):
    """Chimera-like grid of K4,4 cells, open boundary.

    Spin index = ((r*cols + c)*8 + side*4 + k).  Inside a cell every side-0
    spin couples to every side-1 spin (K4,4).  Side-0 spin k of cell (r,c)
    couples to side-0 spin k of cell (r+1,c); side-1 spin k couples to side-1
    spin k of cell (r,c+1).  8x8 cells: 512 spins, 1472 edges.
    """
    ei, ej = [], []

    def q(r, c, side, k):
        return ((r * cols + c) * 8 + side * 4 + k)

    for r in range(rows):
        for c in range(cols):
            for a in range(4):
                for b in range(4):
                    ei.append(q(r, c, 0, a))
                    ej.append(q(r, c, 1, b))
            if r + 1 < rows:
                for k in range(4):
                    ei.append(q(r, c, 0, k))
                    ej.append(q(r + 1, c, 0, k))
            if c + 1 < cols:
                for k in range(4):
                    ei.append(q(r, c, 1, k))
                    ej.append(q(r, c + 1, 1, k))
    return rows * cols * 8, np.asarray(ei, np.int32), np.asarray(ej, np.int32)


def chimera(rows=8, cols=8, seed=0, j_range=(-15, 15), h_range=(-7, 7),
            k_range=(-7, 7), triple_cells_frac=0.1, triples_per_cell=4,
            instance_id=0, restarts=1, name="") -> Instance:
    """Chimera-like instance with 3-spin hyper-couplings inside a few cells.

    J uniform on the integers of ``j_range`` without 0; h uniform on
    ``h_range``; round(frac * cells) distinct cells each get
    ``triples_per_cell`` distinct 3-subsets of their 8 spins, K uniform on
    ``k_range`` (0 included).
    """
    rng = _rng(seed)
    n, ei, ej = chimera_edges(rows, cols)
    ei, ej = ei.copy(), ej.copy()
    jv = np.array([v for v in range(j_range[0], j_range[1] + 1) if v != 0], np.int32)
    J = jv[rng.integers(0, len(jv), size=ei.shape[0])]
    h = rng.integers(h_range[0], h_range[1] + 1, size=n).astype(np.int32)
    ncell = rows * cols
    nsel = int(round(triple_cells_frac * ncell))
    cells = rng.choice(ncell, size=nsel, replace=False) if nsel > 0 else np.zeros(0, int)
    subsets = [(a, b, c) for a in range(8) for b in range(a + 1, 8) for c in range(b + 1, 8)]
    tri = []
    for cell in cells:
        pick = rng.choice(len(subsets), size=triples_per_cell, replace=False)
        for p in pick:
            a, b, c = subsets[p]
            tri.append((cell * 8 + a, cell * 8 + b, cell * 8 + c))
    tri = np.asarray(tri, np.int32).reshape(-1, 3)
    K = rng.integers(k_range[0], k_range[1] + 1, size=tri.shape[0]).astype(np.int32)
    return Instance(n=n, ei=ei, ej=ej, J=J, h=h, tri=tri, K=K,
                    instance_id=instance_id, restarts=restarts,
                    name=name or f"chimera{rows}x{cols}")


def _unique_pairs(rng, n, m) -> np.ndarray:
    """m distinct unordered pairs {i, j}, i != j, uniform (rejection)."""
    if m > n * (n - 1) // 2:
        raise ValueError("too many edges")
    have = np.zeros(0, dtype=np.int64)
    while have.shape[0] < m:
        need = m - have.shape[0]
        k = int(need * 1.1) + 16
        a = rng.integers(0, n, size=k, dtype=np.int64)
        b = rng.integers(0, n, size=k, dtype=np.int64)
        ok = a != b
        lo = np.minimum(a, b)[ok]
        hi = np.maximum(a, b)[ok]
        key = lo * n + hi
        # keep first occurrence order while removing duplicates
        allk = np.concatenate([have, key])
        _, first = np.unique(allk, return_index=True)
        first.sort()
        have = allk[first]
    have = have[:m]
    return np.stack([have // n, have % n], axis=1)


def _unique_triples(rng, n, t) -> np.ndarray:
    """t distinct 3-subsets of distinct spins, uniform (rejection); sorted rows."""
    if n < 3 and t > 0:
        raise ValueError("triples need n >= 3")
    have = np.zeros((0, 3), dtype=np.int64)
    while have.shape[0] < t:
        need = t - have.shape[0]
        k = int(need * 1.1) + 16
        x = rng.integers(0, n, size=(k, 3), dtype=np.int64)
        ok = (x[:, 0] != x[:, 1]) & (x[:, 0] != x[:, 2]) & (x[:, 1] != x[:, 2])
        x = np.sort(x[ok], axis=1)
        allx = np.concatenate([have, x])
        key = (allx[:, 0] * n + allx[:, 1]) * n + allx[:, 2]
        _, first = np.unique(key, return_index=True)
        first.sort()
        have = allx[first]
    return have[:t]


def erdos_renyi_triples(n, seed=0, mean_degree=6, triples_per_spin=0.5,
                        instance_id=0, restarts=1, name="") -> Instance:
    """G(n, m = mean_degree*n/2) simple random graph plus floor(frac*n) distinct
    random 3-spin triples; J and K uniform on {-1,+1}; h = 0."""
    rng = _rng(seed)
    m = int(mean_degree * n // 2)
    pairs = _unique_pairs(rng, n, m)
    t = int(math.floor(triples_per_spin * n))
    tri = _unique_triples(rng, n, t)
    return Instance(n=n, ei=pairs[:, 0], ej=pairs[:, 1], J=_pm1(rng, m),
                    h=None, tri=tri, K=_pm1(rng, t),
                    instance_id=instance_id, restarts=restarts,
                    name=name or f"er{n}")


def random_regular3(n, seed=0, j_range=(-15, 15), instance_id=0, restarts=1,
                    name="") -> Instance:
    """Random 3-regular simple graph (configuration model, rejection of
    self-loops and multi-edges by restarting), J uniform on the integers of
    ``j_range`` (0 included), h = 0.  n must be even."""
    if n % 2 or n < 4:
        raise ValueError("3-regular needs even n >= 4")
    rng = _rng(seed)
    for _ in range(1000):
        stubs = np.repeat(np.arange(n, dtype=np.int64), 3)
        rng.shuffle(stubs)
        a, b = stubs[0::2], stubs[1::2]
        if np.any(a == b):
            continue
        key = np.minimum(a, b) * n + np.maximum(a, b)
        if np.unique(key).shape[0] != key.shape[0]:
            # repair by random swaps is biased; simply retry
            continue
        J = rng.integers(j_range[0], j_range[1] + 1, size=a.shape[0]).astype(np.int32)
        return Instance(n=n, ei=a, ej=b, J=J, instance_id=instance_id,
                        restarts=restarts, name=name or f"reg3_{n}")
    # large n: the pairing succeeds with probability ~exp(-2); fall back to
    # a switch-based repair that keeps degrees exact
    return _regular3_switch(n, rng, j_range, instance_id, restarts, name)


def _regular3_switch(n, rng, j_range, instance_id, restarts, name):
    stubs = np.repeat(np.arange(n, dtype=np.int64), 3)
    rng.shuffle(stubs)
    a, b = stubs[0::2].copy(), stubs[1::2].copy()
    m = a.shape[0]
    for _ in range(200):
        key = np.minimum(a, b) * n + np.maximum(a, b)
        _, first, counts = np.unique(key, return_index=True, return_counts=True)
        dup = np.ones(m, bool)
        dup[first] = False
        bad = np.nonzero((a == b) | dup)[0]
        if bad.shape[0] == 0:
            J = rng.integers(j_range[0], j_range[1] + 1, size=m).astype(np.int32)
            return Instance(n=n, ei=a, ej=b, J=J, instance_id=instance_id,
                            restarts=restarts, name=name or f"reg3_{n}")
        other = rng.integers(0, m, size=bad.shape[0])
        for e, f in zip(bad, other):
            a[e], b[f] = b[f], a[e]
    raise RuntimeError("3-regular generation failed")


def chain(n, seed=0, j_range=(-3, 3), periodic=False, instance_id=0) -> Instance:
    """1-D chain with nonzero integer couplings, h = 0."""
    rng = _rng(seed)
    jv = np.array([v for v in range(j_range[0], j_range[1] + 1) if v != 0], np.int32)
    ei = np.arange(n - 1 + (1 if periodic else 0)) % n
    ej = (ei + 1) % n
    J = jv[rng.integers(0, len(jv), size=ei.shape[0])]
    return Instance(n=n, ei=ei, ej=ej, J=J, instance_id=instance_id, name=f"chain{n}")


def complete_graph(n, seed=0, j_range=(-3, 3), instance_id=0) -> Instance:
    rng = _rng(seed)
    a, b = np.triu_indices(n, 1)
    J = rng.integers(j_range[0], j_range[1] + 1, size=a.shape[0]).astype(np.int32)
    return Instance(n=n, ei=a, ej=b, J=J, instance_id=instance_id, name=f"K{n}")


def random_small(n, seed=0, p_edge=0.3, n_triples=None, j_range=(-5, 5),
                 h_range=(-4, 4), k_range=(-5, 5), instance_id=0, restarts=1) -> Instance:
    """Small random instance for exhaustive checks: G(n, p) edges, a few
    triples, integer J, h, K (0 allowed)."""
    rng = _rng(seed)
    a, b = np.triu_indices(n, 1)
    keep = rng.random(a.shape[0]) < p_edge
    a, b = a[keep], b[keep]
    J = rng.integers(j_range[0], j_range[1] + 1, size=a.shape[0]).astype(np.int32)
    h = rng.integers(h_range[0], h_range[1] + 1, size=n).astype(np.int32)
    if n_triples is None:
        n_triples = n // 2
    tri = _unique_triples(rng, n, n_triples) if n >= 3 else np.zeros((0, 3), np.int64)
    K = rng.integers(k_range[0], k_range[1] + 1, size=tri.shape[0]).astype(np.int32)
    # shuffle edge endpoint order and triple member order (inputs are unordered)
    flip = rng.random(a.shape[0]) < 0.5
    ei = np.where(flip, b, a)
    ej = np.where(flip, a, b)
    for row in tri:
        rng.shuffle(row)
    return Instance(n=n, ei=ei, ej=ej, J=J, h=h, tri=tri, K=K,
                    instance_id=instance_id, restarts=restarts, name=f"small{n}")


def ferromagnet(inst: Instance) -> Instance:
    """Same graph with every coupling, field and hyper-coupling made
    non-negative (|J|, |h|, |K|): no term can be frustrated."""
    return inst.replace(J=np.abs(inst.J), h=None if inst.h is None else np.abs(inst.h),
                        K=np.abs(inst.K), name=inst.name + "-ferro")


def gauge(inst: Instance, xi: np.ndarray, absolute=False) -> Instance:
    """Gauge transform by xi in {-1,+1}^n.

    absolute=False: J'_ij = xi_i xi_j J_ij, h'_i = xi_i h_i,
    K'_ijk = xi_i xi_j xi_k K_ijk (same spectrum, E'(xi*s) = E(s)).
    absolute=True: Mattis instance J'_ij = xi_i xi_j |J_ij| etc., whose
    unique-energy ground state is s = xi with E = -sum|J| - sum|h| - sum|K|.
    """
    xi = np.asarray(xi, dtype=np.int32)
    J = np.abs(inst.J) if absolute else inst.J
    K = np.abs(inst.K) if absolute else inst.K
    h = inst.h
    if h is not None:
        h = (np.abs(h) if absolute else h) * xi
    Jp = (J * xi[inst.ei] * xi[inst.ej]).astype(np.int32)
    Kp = (K * xi[inst.tri[:, 0]] * xi[inst.tri[:, 1]] * xi[inst.tri[:, 2]]).astype(np.int32)
    return inst.replace(J=Jp, h=h, K=Kp, name=inst.name + ("-mattis" if absolute else "-gauge"))


# --------------------------------------------------------------------------
# the five workloads (sizes, distributions and seeds are fixed here)


def cfg1_square16(restarts=64) -> Instance:
    """16x16 periodic square lattice, J in {-1,+1}, h = 0, checkerboard."""
    return lattice((16, 16), periodic=True, seed=1, restarts=restarts, name="square16")


def cfg1_square4() -> Instance:
    """4x4 periodic square lattice (16 spins, 32 bonds) for exhaustive search."""
    return lattice((4, 4), periodic=True, seed=11, name="square4")


def cfg2_cubic100(L=100, seed=2) -> Instance:
    """L^3 periodic cubic lattice, J in {-1,+1}, h uniform on {-2..2},
    checkerboard colouring; L=100 gives 10^6 spins and 3*10^6 bonds."""
    return lattice((L, L, L), periodic=True, seed=seed, h_range=(-2, 2),
                   name=f"cubic{L}")


def cfg3_chimera_batch(count=4096, restarts=256, seed=3) -> List[Instance]:
    """``count`` Chimera-like 8x8-cell instances (512 spins) with
    hyper-couplings; instance ids 0..count-1."""
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(count)
    return [chimera(8, 8, seed=children[i], instance_id=i, restarts=restarts,
                    name=f"chimera#{i}") for i in range(count)]


def cfg4_sizes(count=2000, seed=4) -> np.ndarray:
    rng = _rng(seed)
    return np.round(np.exp(rng.uniform(math.log(100), math.log(1e5), size=count))).astype(np.int64)


def cfg4_uneven_batch(count=2000, seed=4, sizes=None) -> List[Instance]:
    """``count`` Erdos-Renyi instances, n log-uniform on [100, 1e5], mean
    degree 6, n/2 triples, J and K in {-1,+1}, h = 0."""
    if sizes is None:
        sizes = cfg4_sizes(count, seed)
    ss = np.random.SeedSequence(seed + 1000)
    children = ss.spawn(len(sizes))
    return [erdos_renyi_triples(int(nv), seed=children[i], instance_id=i,
                                name=f"er#{i}") for i, nv in enumerate(sizes)]


def serving_instance(family: str, n_target: int, seed, instance_id: int) -> Instance:
    """One request of the mixed serving workload (families: 'sq2', 'cub3',
    'chimera', 'reg3'), sized near ``n_target`` spins.  Lattice requests carry
    their periodic extents as the solver's lattice hint."""
    if family == "sq2":
        L = max(4, int(round(math.sqrt(n_target) / 2)) * 2)
        return lattice((L, L), seed=seed, instance_id=instance_id, name=f"sq{L}", hint=True)
    if family == "cub3":
        L = max(4, int(round(n_target ** (1 / 3) / 2)) * 2)
        return lattice((L, L, L), seed=seed, instance_id=instance_id, name=f"cub{L}", hint=True)
    if family == "chimera":
        G = max(2, int(round(math.sqrt(n_target / 8))))
        return chimera(G, G, seed=seed, instance_id=instance_id, name=f"chim{G}")
    if family == "reg3":
        nn = max(4, int(n_target) // 2 * 2)
        return random_regular3(nn, seed=seed, instance_id=instance_id)
    raise ValueError(family)


def cfg5_trace(count=2000, seed=5, n_lo=1e3, n_hi=1e6):
    """Request trace: list of (family, n_target, seed, instance_id) and
    unit-rate exponential inter-arrival gaps (scale by 1/lambda)."""
    rng = _rng(seed)
    fams = np.array(["sq2", "cub3", "chimera", "reg3"])
    fam = fams[rng.integers(0, 4, size=count)]
    n = np.round(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=count))).astype(np.int64)
    gaps = rng.exponential(1.0, size=count)
    seeds = rng.integers(0, 2**31 - 1, size=count)
    reqs = [(str(fam[i]), int(n[i]), int(seeds[i]), i) for i in range(count)]
    return reqs, gaps


@dataclasses.dataclass
class DenseInstance:
    """At most 64 spins; term t is the set of spins in bit mask ``masks[t]``
    with coefficient ``coefs[t]`` (energy -sum coef prod S)."""
    n: int
    masks: np.ndarray
    coefs: np.ndarray
    instance_id: int = 0
    restarts: int = 1
    name: str = ""

    def replace(self, **kw) -> "DenseInstance":
        return dataclasses.replace(self, **kw)


def random_dense(n: int, nterms: int, max_order: int = 4, coef_range=(-50, 50), seed=0, instance_id=0,
                 restarts=1, name="") -> DenseInstance:
    """Distinct random terms of 1..max_order spins with uniform integer coefficients."""
    rng = _rng(seed)
    seen = {}
    tries = 0
    while len(seen) < nterms and tries < 100 * nterms:
        tries += 1
        k = int(rng.integers(1, min(max_order, n) + 1))
        members = rng.choice(n, size=k, replace=False)
        m = 0
        for i in members:
            m |= 1 << int(i)
        if m not in seen:
            seen[m] = int(rng.integers(coef_range[0], coef_range[1] + 1))
    masks = np.array(list(seen.keys()), dtype=np.uint64)
    coefs = np.array(list(seen.values()), dtype=np.int64)
    return DenseInstance(n=n, masks=masks, coefs=coefs, instance_id=instance_id, restarts=restarts,
                         name=name or f"dense{n}_{len(seen)}")


def dense_from_sparse(inst: Instance) -> DenseInstance:
    """The same energy function written as dense terms (n <= 64): fields as
    one-spin terms, couplings and triples by their member sets."""
    masks, coefs = [], []
    h = inst.h_or_zero()
    for i in range(inst.n):
        if h[i]:
            masks.append(1 << i)
            coefs.append(int(h[i]))
    for a, b, j in zip(inst.ei, inst.ej, inst.J):
        masks.append((1 << int(a)) | (1 << int(b)))
        coefs.append(int(j))
    for (a, b, c), k in zip(inst.tri, inst.K):
        masks.append((1 << int(a)) | (1 << int(b)) | (1 << int(c)))
        coefs.append(int(k))
    return DenseInstance(n=inst.n, masks=np.array(masks, dtype=np.uint64), coefs=np.array(coefs, dtype=np.int64),
                         instance_id=inst.instance_id, restarts=inst.restarts, name=inst.name + "_dense")
