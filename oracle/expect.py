"""Pauli expectation values and the VQE energy (oracle side).

E = <psi|H|psi> / <psi|psi>  (eq. 7) with H = sum_i w_i P_i (eq. 2), summed
term by term as in the paper's evaluation (Sec. III-D).

Two independent routes to <psi|P|psi>:
  * ``expect_term_gates``: copy psi, apply each non-identity single-qubit
    Pauli as a 2x2 matrix with the simulator, take vdot (used for n <= 14);
  * ``expect_term_masks``: P(x, z)|b> = i^{popcount(x&z)} (-1)^{popcount(z&b)} |b^x>,
    vectorised over all b (any n).
The tests cross-check the two routes.
"""
from __future__ import annotations

import math

import numpy as np

from . import statevector as sv

_PAULI = {
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def expect_term_gates(psi, n, string):
    phi = psi.copy()
    for q, c in enumerate(string):
        if c != "I":
            sv.apply_1q(phi, n, q, _PAULI[c])
    return np.vdot(psi, phi)


def expect_term_masks(psi, n, x, z):
    b = np.arange(1 << n, dtype=np.uint64)
    src = b ^ np.uint64(x)
    sign = 1.0 - 2.0 * (np.bitwise_count(src & np.uint64(z)) & 1).astype(np.float64)
    y = bin(int(x) & int(z)).count("1") % 4
    phase = (1, 1j, -1, -1j)[y]
    phi = phase * sign * psi[src.astype(np.int64)]
    return np.vdot(psi, phi)


def string_masks(string):
    x = z = 0
    for j, c in enumerate(string):
        if c in "XY":
            x |= 1 << j
        if c in "ZY":
            z |= 1 << j
    return x, z


def energy(psi, n, H, route="auto"):
    """E = fsum_i w_i Re<P_i> / Re<psi|psi>, one term at a time.

    H is {string: w}.  Returns (E, norm).
    """
    if route == "auto":
        route = "gates" if n <= 14 else "masks"
    parts = []
    for s, w in H.items():
        if route == "gates":
            v = expect_term_gates(psi, n, s)
        else:
            x, z = string_masks(s)
            v = expect_term_masks(psi, n, x, z)
        parts.append(w * v.real)
    norm = float(np.vdot(psi, psi).real)
    return math.fsum(parts) / norm, norm


def energy_masks(psi, n, x, z, w):
    """The same energy from (x, z, w) arrays."""
    parts = [float(wi) * expect_term_masks(psi, n, int(xi), int(zi)).real
             for xi, zi, wi in zip(x.tolist(), z.tolist(), w.tolist())]
    norm = float(np.vdot(psi, psi).real)
    return math.fsum(parts) / norm, norm


def apply_hamiltonian(psi, n, H):
    """H psi, term by term (used by the oracle adjoint)."""
    out = np.zeros_like(psi)
    b = np.arange(1 << n, dtype=np.uint64)
    for s, w in H.items():
        x, z = string_masks(s)
        src = b ^ np.uint64(x)
        sign = 1.0 - 2.0 * (np.bitwise_count(src & np.uint64(z)) & 1).astype(np.float64)
        y = bin(x & z).count("1") % 4
        out += (w * (1, 1j, -1, -1j)[y]) * sign * psi[src.astype(np.int64)]
    return out
