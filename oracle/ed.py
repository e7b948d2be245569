"""Exact diagonalisation and the free-fermion energy (oracle side).

Pins the oracle's Hamiltonians and its variational energies: for any state,
E(theta) >= E_0, the lowest eigenvalue over the whole 2^n space (eq. 7 is a
Rayleigh quotient).  The layered RY/RZ/CNOT ansatz does not conserve particle
number, so E_0 is the global minimum, not that of one sector.
"""
from __future__ import annotations

from functools import reduce

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_M = {
    "I": np.eye(2, dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def dense(H, n):
    """Dense matrix by Kronecker products; qubit n-1 is the leftmost factor."""
    out = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for s, w in H.items():
        out += w * reduce(np.kron, [_M[s[q]] for q in reversed(range(n))])
    return out


def sparse(H, n):
    """CSR matrix, each term a signed permutation P|b> = i^y (-1)^{z.b} |b^x>."""
    dim = 1 << n
    b = np.arange(dim, dtype=np.uint64)
    rows, cols, vals = [], [], []
    for s, w in H.items():
        x = z = 0
        for j, c in enumerate(s):
            if c in "XY":
                x |= 1 << j
            if c in "ZY":
                z |= 1 << j
        y = bin(x & z).count("1") % 4
        sign = 1.0 - 2.0 * (np.bitwise_count(b & np.uint64(z)) & 1)
        rows.append((b ^ np.uint64(x)).astype(np.int64))
        cols.append(b.astype(np.int64))
        vals.append(w * (1, 1j, -1, -1j)[y] * sign)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(dim, dim))


def ground_energy(H, n):
    if n <= 10:
        return float(np.linalg.eigvalsh(dense(H, n))[0])
    vals = spla.eigsh(sparse(H, n), k=1, which="SA", tol=1e-12)[0]
    return float(vals[0])


def free_fermion_energy(n_sites, bonds, t):
    """U = 0 Hubbard ground energy: 2 * sum of the negative single-particle levels."""
    T = np.zeros((n_sites, n_sites))
    for (i, j) in bonds:
        T[i, j] += -t
        T[j, i] += -t
    eps = np.linalg.eigvalsh(T)
    return 2.0 * float(eps[eps < 0].sum())


def restricted(H, n, basis):
    """P H P on the span of the basis states `basis` (a list of indices), as a
    dense matrix M[i, j] = <basis_i|H|basis_j>, built term by term from
    P|b> = i^y (-1)^{z.b} |b^x>.  Its lowest eigenvalue bounds <psi|H|psi>
    from below for every normalised psi inside that span (e.g. a particle-number
    and spin sector), whether or not H itself conserves the span."""
    basis = np.asarray(basis, dtype=np.int64)
    order = np.argsort(basis)
    srt = basis[order]
    M = np.zeros((len(basis), len(basis)), dtype=np.complex128)
    bu = basis.astype(np.uint64)
    cols = np.arange(len(basis))
    for s, w in H.items():
        x = z = 0
        for j, c in enumerate(s):
            if c in "XY":
                x |= 1 << j
            if c in "ZY":
                z |= 1 << j
        y = bin(x & z).count("1") % 4
        sign = 1.0 - 2.0 * (np.bitwise_count(bu & np.uint64(z)) & 1)
        tgt = (bu ^ np.uint64(x)).astype(np.int64)
        val = w * (1, 1j, -1, -1j)[y] * sign
        k = np.minimum(np.searchsorted(srt, tgt), len(srt) - 1)
        inside = srt[k] == tgt                      # b^x is a basis state of the span
        np.add.at(M, (order[k[inside]], cols[inside]), val[inside])
    return M


def sector_basis(n, n_up, n_dn):
    """Basis indices with n_up electrons on the even (up) spin-orbitals and
    n_dn on the odd (down) ones (spin-orbital 2 i + sigma)."""
    up = sum(1 << q for q in range(0, n, 2))
    return [b for b in range(1 << n) if bin(b & up).count("1") == n_up and bin(b & ~up).count("1") == n_dn]

