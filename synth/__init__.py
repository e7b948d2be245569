"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds only input data: random parameter vectors, random
one- and two-electron integral tensors and lattice bond lists.  It contains
none of the arithmetic of the simulation method (no Jordan-Wigner mapping, no
gates, no expectation values), so that the oracle and the GPU library stay
independent of each other while reading identical inputs.

The workloads stand in for the paper's molecular Hamiltonians (CO2 at 28
qubits, C3H6 at 32 qubits, STO-3G; Sec. II-B), whose integrals are not
available: Fermi-Hubbard lattices and a "molecule-shaped" integral generator
with the same O(n^4) growth of the number of Pauli terms.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "theta", "theta_batch", "molecule_integrals", "chain_bonds", "snake_bonds",
    "Lattice", "Workload", "WORKLOADS", "serving_instance",
]


def theta(seed: int, size: int) -> np.ndarray:
    """Ansatz angles drawn uniform in [-pi, pi) from ``default_rng(seed)``."""
    return np.random.default_rng(seed).uniform(-math.pi, math.pi, size=size)


def theta_batch(seed: int, batch: int, size: int) -> np.ndarray:
    """A batch of angle vectors; row r is vector r of one draw of shape (batch, size)."""
    return np.random.default_rng(seed).uniform(-math.pi, math.pi, size=(batch, size))


def molecule_integrals(n_orb: int, seed: int = 0):
    """Molecule-shaped one- and two-electron integrals (chemist notation).

    h[p, q] = h[q, p] ~ N(0, 1) * exp(-|p-q|/2), drawn for p <= q in row-major order.
    g[p, q, r, s] = (pq|rs) with 8-fold symmetry; one value is drawn per unique
    representative p >= q, r >= s, pq >= rs (pq = p(p+1)/2 + q) in ascending
    (pq, rs) order, ~ N(0, sd=0.01) * exp(-(|p-q| + |r-s|)/2).
    The h draws come first, then the g draws, from ``default_rng(seed)``.
    """
    rng = np.random.default_rng(seed)
    n = n_orb
    h = np.zeros((n, n))
    for p in range(n):
        for q in range(p, n):
            v = rng.normal(0.0, 1.0) * math.exp(-abs(p - q) / 2.0)
            h[p, q] = v
            h[q, p] = v
    pairs = [(p, q) for p in range(n) for q in range(p + 1)]
    pairs.sort(key=lambda t: t[0] * (t[0] + 1) // 2 + t[1])
    g = np.zeros((n, n, n, n))
    for i, (p, q) in enumerate(pairs):
        for (r, s) in pairs[: i + 1]:
            v = rng.normal(0.0, 0.01) * math.exp(-(abs(p - q) + abs(r - s)) / 2.0)
            for (a, b) in ((p, q), (q, p)):
                for (c, d) in ((r, s), (s, r)):
                    g[a, b, c, d] = v
                    g[c, d, a, b] = v
    return h, g


def chain_bonds(n_sites: int):
    """Open 1-D chain: bonds (i, i+1), each undirected bond listed once."""
    return [(i, i + 1) for i in range(n_sites - 1)]


def snake_bonds(rows: int, cols: int, periodic_long: bool):
    """Bonds of a rows x cols lattice in snake (boustrophedon) site order.

    Rows run along the long axis; site(r, c) = r*cols + (c if r even else cols-1-c).
    Row bonds join (r, c)-(r, c+1); with ``periodic_long`` each row also wraps
    (r, cols-1)-(r, 0).  Column bonds join (r, c)-(r+1, c); there is no wrap on
    the short axis.  Each undirected bond is listed once, as (min, max).
    """
    def site(r, c):
        return r * cols + (c if r % 2 == 0 else cols - 1 - c)

    bonds = []
    for r in range(rows):
        for c in range(cols - 1):
            bonds.append((site(r, c), site(r, c + 1)))
        if periodic_long and cols > 2:
            bonds.append((site(r, cols - 1), site(r, 0)))
    for r in range(rows - 1):
        for c in range(cols):
            bonds.append((site(r, c), site(r + 1, c)))
    return [tuple(sorted(b)) for b in bonds]


@dataclass(frozen=True)
class Lattice:
    n_sites: int
    bonds: tuple
    t: float
    U: float


@dataclass(frozen=True)
class Workload:
    """One benchmark / parity workload: Hamiltonian source, ansatz depth, angle seed."""
    name: str
    n_qubits: int
    layers: int
    theta_seed: int
    kind: str                      # "hubbard" or "molecule"
    lattice: Lattice | None = None
    n_orb: int = 0
    integral_seed: int = 0
    thresholds: tuple = field(default=(0.0,))
    batch: int = 1

    @property
    def n_params(self) -> int:
        return 2 * self.n_qubits * self.layers

    def thetas(self) -> np.ndarray:
        if self.batch == 1:
            return theta(self.theta_seed, self.n_params)[None, :]
        return theta_batch(self.theta_seed, self.batch, self.n_params)


def _hub(n_sites, bonds, t, U):
    return Lattice(n_sites=n_sites, bonds=tuple(bonds), t=t, U=U)


WORKLOADS = {
    # 12 qubits: 1-D Hubbard, 6 sites, open, t=1, U=4; 4 layers; seed 0.
    "hubbard1d_6": Workload("hubbard1d_6", 12, 4, 0, "hubbard",
                            lattice=_hub(6, chain_bonds(6), 1.0, 4.0)),
    # 20 qubits: molecule-shaped, 10 orbitals, integral seed 0; 8 layers; seed 0.
    "molecule_10": Workload("molecule_10", 20, 8, 0, "molecule", n_orb=10,
                            integral_seed=0, thresholds=(0.0, 1e-6, 1e-4, 1e-3)),
    # 28 qubits: 2x7 Hubbard, periodic long axis, t=1, U=8; 16 layers; seed 1; batch 8.
    "hubbard2x7": Workload("hubbard2x7", 28, 16, 1, "hubbard",
                           lattice=_hub(14, snake_bonds(2, 7, True), 1.0, 8.0), batch=8),
    # 32 qubits: 4x4 Hubbard, open, t=1, U=4; 8 layers; seed 0.
    "hubbard4x4": Workload("hubbard4x4", 32, 8, 0, "hubbard",
                           lattice=_hub(16, snake_bonds(4, 4, False), 1.0, 4.0)),
    # 24 qubits: 2x6 Hubbard, open, t=1, U=4; 8 layers; seed 2 (generic-angle
    # gradient parity where reverse passes walk several units per block).
    "hubbard2x6": Workload("hubbard2x6", 24, 8, 2, "hubbard",
                           lattice=_hub(12, snake_bonds(2, 6, False), 1.0, 4.0)),
    # 26 qubits: 1-D Hubbard, 13 sites, open, t=1, U=4; 4 layers; seed 3.
    "hubbard1d_13": Workload("hubbard1d_13", 26, 4, 3, "hubbard",
                             lattice=_hub(13, chain_bonds(13), 1.0, 4.0)),
    # 32 qubits: molecule-shaped, 16 orbitals, slimmed at 1e-4 and 1e-3; 8 layers.
    "molecule_16": Workload("molecule_16", 32, 8, 0, "molecule", n_orb=16,
                            integral_seed=0, thresholds=(1e-4, 1e-3)),
}


def serving_instance(i: int):
    """Optimiser instance i of the served stream: its own generator from seed 10000+i.

    Returns (n_qubits, kind, lattice_or_norb, layers, rng).  n is uniform over
    {12,16,20,24,28}; the Hamiltonian source is uniform over a 1-D Hubbard chain
    with n/2 sites, a molecule-shaped generator with n/2 orbitals and a 2 x (n/4)
    Hubbard ladder; the depth is uniform over [4, 16].  The returned generator
    keeps drawing the instance's angle vectors.
    """
    rng = np.random.default_rng(10_000 + i)
    n = int(rng.choice([12, 16, 20, 24, 28]))
    kind = int(rng.integers(0, 3))
    layers = int(rng.integers(4, 17))
    if kind == 0:
        src = ("hubbard", _hub(n // 2, chain_bonds(n // 2), 1.0, 4.0))
    elif kind == 1:
        src = ("molecule", (n // 2, 10_000 + i))
    else:
        cols = n // 4
        src = ("hubbard", _hub(n // 2, snake_bonds(2, cols, False), 1.0, 4.0))
    return n, src, layers, rng
