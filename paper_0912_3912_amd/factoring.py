"""Ising hypergraphs for integer factoring (Sec. VI, eqs. (6)-(8)).

Factoring an odd N is the minimisation of f(x, y) = (N - x y)^2 over odd
positive integers x and y.  With n_x and n_y free bits (the least-significant
bit of each factor is 1), x = 1 + sum_{i=1..n_x} 2^i b_i and likewise y, and
every bit is a spin through b = (1 - S) / 2.  Expanding the square with
S^2 = 1 gives a multilinear polynomial f = c0 + sum_t a_t prod_{i in t} S_i
with terms of one to four spins; the instance is its energy
E = f - c0 = -sum_t coef_t prod S with coef_t = -a_t, so E = -c0 exactly at
a factorisation.

Spin numbering: spins 0 .. n_x - 1 are the free bits of x from the most
significant down, spins n_x .. n_x + n_y - 1 those of y, the same way (this
reproduces the polynomial printed for N = 21 with n_x = 1, n_y = 2).

All coefficients are exact Python integers; the builder refuses instances
whose energy could leave the int64 range of the dense kernels.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Tuple

import numpy as np

__all__ = ["FactoringInstance", "factoring_instance", "factoring_polynomial"]

_INT64_SAFE = 1 << 62


def _mul(p: Dict[int, int], q: Dict[int, int]) -> Dict[int, int]:
    """Product of multilinear polynomials in +-1 spins (keys: member masks;
    S_i^2 = 1 makes the product of two monomials their symmetric difference)."""
    out: Dict[int, int] = {}
    for m1, c1 in p.items():
        for m2, c2 in q.items():
            m = m1 ^ m2
            out[m] = out.get(m, 0) + c1 * c2
    return {m: c for m, c in out.items() if c}


def _factor_poly(nbits: int, first_spin: int) -> Dict[int, int]:
    """1 + sum_{i=1..nbits} 2^i (1 - S)/2 with bit i on spin first_spin + nbits - i."""
    p = {0: 1}
    for i in range(1, nbits + 1):
        spin = first_spin + nbits - i
        w = 1 << (i - 1)  # 2^i / 2
        p[0] = p.get(0, 0) + w
        p[1 << spin] = p.get(1 << spin, 0) - w
    return p


def factoring_polynomial(N: int, nx: int, ny: int) -> Tuple[int, Dict[int, int]]:
    """(c0, {mask: a_t}) with (N - x y)^2 = c0 + sum_t a_t prod_{i in t} S_i."""
    if N < 1 or N % 2 == 0:
        raise ValueError("N must be a positive odd integer")
    if nx < 0 or ny < 0 or nx + ny < 1 or nx + ny > 64:
        raise ValueError("need 1 <= n_x + n_y <= 64 free bits")
    x = _factor_poly(nx, 0)
    y = _factor_poly(ny, nx)
    xy = _mul(x, y)
    g = {m: -c for m, c in xy.items()}
    g[0] = g.get(0, 0) + N
    g = {m: c for m, c in g.items() if c}
    f = _mul(g, g)
    c0 = f.pop(0, 0)
    return c0, f


@dataclasses.dataclass
class FactoringInstance:
    """Dense hyper-Ising instance of a factoring problem: ``masks`` (uint64,
    bit i = spin i) and ``coefs`` (int64) with E = -sum coef prod S."""
    N: int
    nx: int
    ny: int
    const: int
    masks: np.ndarray
    coefs: np.ndarray
    instance_id: int = 0
    restarts: int = 1
    name: str = ""

    @property
    def n(self) -> int:
        return self.nx + self.ny

    def replace(self, **kw) -> "FactoringInstance":
        return dataclasses.replace(self, **kw)

    def decode(self, s) -> Tuple[int, int]:
        """(x, y) of a spin state (+-1 per spin)."""
        s = [int(v) for v in s]
        x = 1 + sum((1 << i) * (1 - s[self.nx - i]) // 2 for i in range(1, self.nx + 1))
        y = 1 + sum((1 << i) * (1 - s[self.nx + self.ny - i]) // 2 for i in range(1, self.ny + 1))
        return x, y

    def ground_energy(self) -> int:
        """The energy of an exact factorisation (f = 0)."""
        return -self.const


def factoring_instance(N: int, nx: int, ny: int, instance_id: int = 0, restarts: int = 1,
                       drop_order_above: int = 0) -> FactoringInstance:
    """Factoring hypergraph of N with n_x and n_y free bits.  With
    ``drop_order_above`` = k > 0 the terms over more than k spins are omitted
    (the paper's comparison of factoring with and without hyper-couplings)."""
    c0, f = factoring_polynomial(N, nx, ny)
    items = sorted(f.items(), key=lambda mc: (bin(mc[0]).count("1"), mc[0]))
    if drop_order_above:
        items = [(m, c) for m, c in items if bin(m).count("1") <= drop_order_above]
    if sum(abs(c) for _, c in items) >= _INT64_SAFE:
        raise ValueError(f"N = {N} with {nx}+{ny} free bits: coefficients exceed the int64 energy range")
    masks = np.array([m for m, _ in items], dtype=np.uint64)
    coefs = np.array([-c for _, c in items], dtype=np.int64)
    return FactoringInstance(N=N, nx=nx, ny=ny, const=c0, masks=masks, coefs=coefs, instance_id=instance_id,
                             restarts=restarts, name=f"factor{N}_{nx}x{ny}")
