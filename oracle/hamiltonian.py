"""Qubit Hamiltonians from fermionic operators by Jordan-Wigner (oracle side).

Follows Sec. II-B: the second-quantised H of eq. (1) is mapped by the
Jordan-Wigner transform to a sum of Pauli strings H = sum_i w_i P_i with
P_i a tensor product of I, X, Y, Z (eqs. 2-4).

Conventions (the paper names openfermion but does not state one):
  * qubit j is bit j of the basis index; a Pauli string is a length-n tuple
    of characters, position j acting on qubit j;
  * occupied orbital = |1>;  a_j = Z_0 ... Z_{j-1} (X_j + i Y_j)/2 and
    a_j^dag = Z_0 ... Z_{j-1} (X_j - i Y_j)/2;
  * spin-orbital index 2*site + sigma (sigma = 0 for up).
Strings are multiplied qubit by qubit with the single-qubit product table
(XY = iZ, YZ = iX, ZX = iY, reversed order -i, squares I).  Like strings are
combined; the imaginary parts must cancel (Hermiticity) and are checked.
"""
from __future__ import annotations

import numpy as np

# Single-qubit products: (a, b) -> (phase, c) with a*b = phase * c.
_PROD = {}
for _a in "IXYZ":
    _PROD[("I", _a)] = (1, _a)
    _PROD[(_a, "I")] = (1, _a)
    _PROD[(_a, _a)] = (1, "I")
_PROD[("X", "Y")] = (1j, "Z")
_PROD[("Y", "X")] = (-1j, "Z")
_PROD[("Y", "Z")] = (1j, "X")
_PROD[("Z", "Y")] = (-1j, "X")
_PROD[("Z", "X")] = (1j, "Y")
_PROD[("X", "Z")] = (-1j, "Y")


def string_product(s1, s2):
    """Product of two Pauli strings: returns (phase, string)."""
    phase = 1 + 0j
    out = []
    for a, b in zip(s1, s2):
        ph, c = _PROD[(a, b)]
        phase *= ph
        out.append(c)
    return phase, tuple(out)


def op_product(A, B):
    """Product of two operators given as {string: complex coefficient}."""
    out = {}
    for s1, c1 in A.items():
        for s2, c2 in B.items():
            ph, s = string_product(s1, s2)
            out[s] = out.get(s, 0) + c1 * c2 * ph
    return out


def op_accumulate(A, B):
    """A += B in place (operators as {string: coefficient})."""
    for s, c in B.items():
        A[s] = A.get(s, 0) + c
    return A


def ladder(j, n, dagger):
    """Jordan-Wigner image of a_j (dagger=False) or a_j^dag (dagger=True)."""
    zs = ["Z"] * j + ["I"] * (n - j)
    sx = list(zs)
    sx[j] = "X"
    sy = list(zs)
    sy[j] = "Y"
    cy = -0.5j if dagger else 0.5j
    return {tuple(sx): 0.5 + 0j, tuple(sy): cy}


def fermion_term(n, ops, coeff):
    """JW image of coeff * prod(ops), ops = [(orbital, dagger), ...] left to right."""
    acc = {tuple("I" * n): complex(coeff)}
    for (j, dag) in ops:
        acc = op_product(acc, ladder(j, n, dag))
    return acc


def finalize(op, tol=1e-12):
    """Check Hermiticity (real coefficients), drop |w| < tol; returns {string: float}."""
    if not op:
        return {}
    wmax = max(abs(c) for c in op.values())
    out = {}
    for s, c in op.items():
        assert abs(c.imag) <= 1e-12 * max(wmax, 1.0), (s, c)
        if abs(c.real) >= tol:
            out[s] = float(c.real)
    return out


def hubbard(n_sites, bonds, t, U):
    """Fermi-Hubbard model H = -t sum_<ij>,s (a+_is a_js + h.c.) + U sum_i n_iu n_id."""
    n = 2 * n_sites
    H = {}
    for (i, j) in bonds:
        for s in (0, 1):
            p, q = 2 * i + s, 2 * j + s
            op_accumulate(H, fermion_term(n, [(p, True), (q, False)], -t))
            op_accumulate(H, fermion_term(n, [(q, True), (p, False)], -t))
    for i in range(n_sites):
        op_accumulate(H, fermion_term(n, [(2 * i, True), (2 * i, False),
                                       (2 * i + 1, True), (2 * i + 1, False)], U))
    return finalize(H)


def molecule(h, g):
    """H = sum_{pq,s} h_pq a+_ps a_qs + 1/2 sum_{pqrs,s,t} g_pqrs a+_ps a+_rt a_st a_qs.

    Eq. (1) with spin made explicit and chemist-notation two-electron
    integrals g_pqrs = (pq|rs); there is no constant term.
    """
    N = h.shape[0]
    n = 2 * N
    H = {}
    for p in range(N):
        for q in range(N):
            if h[p, q] == 0.0:
                continue
            for s in (0, 1):
                op_accumulate(H, fermion_term(n, [(2 * p + s, True), (2 * q + s, False)], h[p, q]))
    for p in range(N):
        for q in range(N):
            for r in range(N):
                for s_ in range(N):
                    v = g[p, q, r, s_]
                    if v == 0.0:
                        continue
                    for a in (0, 1):
                        for b in (0, 1):
                            P, Q, R, S = 2 * p + a, 2 * q + a, 2 * r + b, 2 * s_ + b
                            if P == R or Q == S:
                                continue      # a+_P a+_P = 0 and a_S a_S = 0
                            op_accumulate(H, fermion_term(
                                n, [(P, True), (R, True), (S, False), (Q, False)], 0.5 * v))
    return finalize(H)


def to_masks(H):
    """Pauli dict -> (x, z, w) arrays sorted by (x, z); Y sets both bits.

    Encoding: (x_j, z_j) = (0,0) I, (1,0) X, (0,1) Z, (1,1) Y.
    """
    rows = []
    for s, w in H.items():
        x = z = 0
        for j, c in enumerate(s):
            if c in "XY":
                x |= 1 << j
            if c in "ZY":
                z |= 1 << j
        rows.append((x, z, w))
    rows.sort(key=lambda r: (r[0], r[1]))
    x = np.array([r[0] for r in rows], dtype=np.uint64)
    z = np.array([r[1] for r in rows], dtype=np.uint64)
    w = np.array([r[2] for r in rows], dtype=np.float64)
    return x, z, w


def from_masks(n, x, z, w):
    """(x, z, w) arrays -> {string: w}."""
    H = {}
    for xi, zi, wi in zip(x.tolist(), z.tolist(), w.tolist()):
        s = []
        for j in range(n):
            bx, bz = (xi >> j) & 1, (zi >> j) & 1
            s.append("IXZY"[bx + 2 * bz])
        H[tuple(s)] = H.get(tuple(s), 0.0) + wi
    return H
