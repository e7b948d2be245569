"""Qubit Hamiltonians from fermionic operators by Jordan-Wigner, on bit masks.

Builds H = sum_i w_i P_i (eqs. 2-4) from the second-quantised form of eq. (1)
(Sec. II-B) with the Jordan-Wigner transform, working directly on (x, z) bit
masks with P(x,z) = i^popcount(x&z) X^x Z^z:
  * a_j    = 1/2 P(e_j, m_j) + i/2 P(e_j, m_j | e_j)
  * a_j^+  = 1/2 P(e_j, m_j) - i/2 P(e_j, m_j | e_j),   m_j = 2^j - 1;
  * P(x1,z1) P(x2,z2) = i^(x1.z1 + x2.z2 + 2 z1.x2 - x3.z3) P(x1^x2, z1^z2),
    a.b = popcount(a & b) (moving Z^z1 past X^x2 gives (-1)^(z1.x2)).
Products are evaluated for all terms at once with NumPy; like terms are
combined by sorting on (x, z).  Occupied orbital = |1>; spin-orbital index
2*site + spin.
"""
from __future__ import annotations

import numpy as np

_IPOW = np.array([1, 1j, -1, -1j], dtype=np.complex128)


def _pc(v):
    return np.bitwise_count(v).astype(np.int64)


def _mul(xa, za, ca, xb, zb, cb):
    """Elementwise product of Pauli-term arrays (broadcasting)."""
    x3 = xa ^ xb
    z3 = za ^ zb
    k = (_pc(xa & za) + _pc(xb & zb) + 2 * _pc(za & xb) - _pc(x3 & z3)) % 4
    return x3, z3, ca * cb * _IPOW[k]


def _ladder(j, dagger):
    """(x, z, c) arrays of the two Pauli terms of a_j or a_j^+ (j: int array)."""
    j = np.asarray(j, dtype=np.uint64)
    e = np.left_shift(np.uint64(1), j)
    m = e - np.uint64(1)
    x = np.stack([e, e], axis=-1)
    z = np.stack([m, m | e], axis=-1)
    cy = -0.5j if dagger else 0.5j
    c = np.broadcast_to(np.array([0.5 + 0j, cy]), x.shape)
    return x, z, c


def fermion_products(ops, coeff):
    """JW images of coeff_t * prod_k op_k for a batch of operator strings.

    ops: list of (orbital_array, dagger) of equal-length integer arrays, applied
    left to right; coeff: array of the same length.  Returns flat (x, z, c).
    """
    T = len(coeff)
    if T == 0:
        return np.zeros(0, np.uint64), np.zeros(0, np.uint64), np.zeros(0, np.complex128)
    x = np.zeros((T, 1), dtype=np.uint64)
    z = np.zeros((T, 1), dtype=np.uint64)
    c = np.asarray(coeff, dtype=np.complex128).reshape(T, 1)
    for orb, dag in ops:
        lx, lz, lc = _ladder(orb, dag)          # (T, 2)
        x3, z3, c3 = _mul(x[:, :, None], z[:, :, None], c[:, :, None],
                          lx[:, None, :], lz[:, None, :], lc[:, None, :])
        x, z, c = x3.reshape(T, -1), z3.reshape(T, -1), c3.reshape(T, -1)
    return x.ravel(), z.ravel(), c.ravel()


def combine(x, z, c, tol=1e-12):
    """Sum like (x, z) terms; check the imaginary parts cancel; drop |w| < tol.

    Returns (x, z, w) sorted by (x, z)."""
    order = np.lexsort((z, x))
    x, z, c = x[order], z[order], c[order]
    new = np.ones(len(x), dtype=bool)
    new[1:] = (x[1:] != x[:-1]) | (z[1:] != z[:-1])
    gid = np.cumsum(new) - 1
    wr = np.bincount(gid, weights=c.real)
    wi = np.bincount(gid, weights=c.imag)
    xs, zs = x[new], z[new]
    if len(wr):
        scale = max(float(np.max(np.abs(wr + 1j * wi))), 1.0)
        if np.max(np.abs(wi)) > 1e-12 * scale:
            raise ValueError("operator is not Hermitian: imaginary Pauli coefficients remain")
    keep = np.abs(wr) >= tol
    return xs[keep], zs[keep], wr[keep]


def hubbard(n_sites, bonds, t, U):
    """H = -t sum_<ij>,s (a+_is a_js + h.c.) + U sum_i n_i,up n_i,dn as (x, z, w)."""
    P, Q, cf = [], [], []
    for (i, j) in bonds:
        for s in (0, 1):
            p, q = 2 * i + s, 2 * j + s
            P += [p, q]
            Q += [q, p]
            cf += [-t, -t]
    hx, hz, hc = fermion_products([(np.array(P), True), (np.array(Q), False)], np.array(cf, dtype=float))
    up = 2 * np.arange(n_sites)
    dn = up + 1
    ux, uz, uc = fermion_products([(up, True), (up, False), (dn, True), (dn, False)],
                                  np.full(n_sites, float(U)))
    return combine(np.concatenate([hx, ux]), np.concatenate([hz, uz]), np.concatenate([hc, uc]))


def molecule(h, g):
    """H = sum_{pq,s} h_pq a+_ps a_qs + 1/2 sum_{pqrs,s,t} g_pqrs a+_ps a+_rt a_st a_qs (chemist g)."""
    N = h.shape[0]
    xs, zs, cs = [], [], []
    p, q = np.nonzero(h)
    for s in (0, 1):
        x1, z1, c1 = fermion_products([(2 * p + s, True), (2 * q + s, False)], h[p, q])
        xs.append(x1), zs.append(z1), cs.append(c1)
    p, q, r, s_ = np.nonzero(g)
    v = g[p, q, r, s_]
    for a in (0, 1):
        for b in (0, 1):
            P, Q, R, S = 2 * p + a, 2 * q + a, 2 * r + b, 2 * s_ + b
            ok = (P != R) & (Q != S)
            if not np.any(ok):
                continue
            x2, z2, c2 = fermion_products(
                [(P[ok], True), (R[ok], True), (S[ok], False), (Q[ok], False)], 0.5 * v[ok])
            xs.append(x2), zs.append(z2), cs.append(c2)
    return combine(np.concatenate(xs), np.concatenate(zs), np.concatenate(cs))


def from_lattice(lattice):
    return hubbard(lattice.n_sites, list(lattice.bonds), lattice.t, lattice.U)
