"""Closed-form results that pin the oracle simulator without running it.

* Bloch vector of RZ(p) RY(t)|0>: (sin t cos p, sin t sin p, cos t).
* The CNOT ladder CNOT(0,1) ... CNOT(n-2,n-1), applied in ascending order,
  maps |b> to |M b> with (M b)_j = b_0 xor ... xor b_j (prefix XOR).
* One layer of the ansatz, psi = L R |0>, with R the product of RZ(p_q) RY(t_q)
  on every qubit: by Clifford conjugation, L^dag P(x,z) L = i^{x.z - x'.z'} P(x',z')
  where X^x Z^z -> X^{x'} Z^{z'} exactly, so <P> = i^{x.z - x'.z'} prod_q <sigma'_q>
  over the Bloch vectors.  Valid at any n (used up to 32 qubits).
* Stabiliser tableau (Aaronson & Gottesman 2004) for circuits whose angles are
  multiples of pi/2: exact <P> in {0, +1, -1} at any n and depth.
"""
from __future__ import annotations

import math

import numpy as np


def bloch_ry_rz(t, p):
    return (math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t))


def ladder_map(b, n):
    out = 0
    acc = 0
    for j in range(n):
        acc ^= (b >> j) & 1
        out |= acc << j
    return out


def _popcount(v):
    return bin(v).count("1")


def conj_cnot(x, z, c, t):
    """CNOT X^x Z^z CNOT = X^{x'} Z^{z'}: X on c copies to t, Z on t copies to c."""
    if (x >> c) & 1:
        x ^= 1 << t
    if (z >> t) & 1:
        z ^= 1 << c
    return x, z


def one_layer_expectation(n, thetas, phis, x, z):
    """<P(x,z)> for psi = L (prod_q RZ(phis[q]) RY(thetas[q])) |0...0>."""
    # L = C_{n-2,n-1} ... C_{0,1};  L^dag P L conjugates by C_{n-2,n-1} first.
    xp, zp = x, z
    for q in reversed(range(n - 1)):
        xp, zp = conj_cnot(xp, zp, q, q + 1)
    phase = (1, 1j, -1, -1j)[(_popcount(x & z) - _popcount(xp & zp)) % 4]
    val = 1.0 + 0j
    for q in range(n):
        bx, bz = (xp >> q) & 1, (zp >> q) & 1
        if bx == 0 and bz == 0:
            continue
        r = bloch_ry_rz(thetas[q], phis[q])
        val *= r[0] if (bx, bz) == (1, 0) else (r[1] if (bx, bz) == (1, 1) else r[2])
    out = phase * val
    assert abs(out.imag) < 1e-12
    return out.real


# ---------------------------------------------------------------- tableau
def _mul1(a, b):
    """(x,z) single-qubit Hermitian Paulis: returns (k, c) with a*b = i^k c."""
    names = {(0, 0): "I", (1, 0): "X", (1, 1): "Y", (0, 1): "Z"}
    inv = {v: k for k, v in names.items()}
    A, B = names[a], names[b]
    if A == "I":
        return 0, b
    if B == "I":
        return 0, a
    if A == B:
        return 0, (0, 0)
    cyc = {("X", "Y"): "Z", ("Y", "Z"): "X", ("Z", "X"): "Y"}
    if (A, B) in cyc:
        return 1, inv[cyc[(A, B)]]
    return 3, inv[cyc[(B, A)]]


class Tableau:
    """Stabiliser state as 2n rows (destabilisers 0..n-1, stabilisers n..2n-1).

    Row i is the Pauli (-1)^{r_i} prod_j sigma(x_ij, z_ij) with (1,1) = Y.
    Starts in |0...0>: destabilisers X_j, stabilisers Z_j.
    """

    def __init__(self, n):
        self.n = n
        self.x = np.zeros((2 * n, n), dtype=np.uint8)
        self.z = np.zeros((2 * n, n), dtype=np.uint8)
        self.r = np.zeros(2 * n, dtype=np.uint8)
        for j in range(n):
            self.x[j, j] = 1
            self.z[n + j, j] = 1

    def h(self, a):
        self.r ^= self.x[:, a] & self.z[:, a]
        self.x[:, a], self.z[:, a] = self.z[:, a].copy(), self.x[:, a].copy()

    def s(self, a):
        self.r ^= self.x[:, a] & self.z[:, a]
        self.z[:, a] ^= self.x[:, a]

    def cnot(self, a, b):
        self.r ^= self.x[:, a] & self.z[:, b] & (self.x[:, b] ^ self.z[:, a] ^ 1)
        self.x[:, b] ^= self.x[:, a]
        self.z[:, a] ^= self.z[:, b]

    def zgate(self, a):
        self.s(a)
        self.s(a)

    def xgate(self, a):
        self.h(a)
        self.zgate(a)
        self.h(a)

    def apply(self, kind, q, angle):
        k = int(round(angle / (math.pi / 2))) % 4
        assert abs(angle - round(angle / (math.pi / 2)) * (math.pi / 2)) < 1e-9, angle
        if kind == "RZ":            # RZ(k pi/2) ~ S^k
            for _ in range(k):
                self.s(q)
        elif kind == "RY":          # RY(pi/2) ~ H Z, RY(pi) ~ X Z, RY(-pi/2) ~ Z H
            if k == 1:
                self.zgate(q)
                self.h(q)
            elif k == 2:
                self.zgate(q)
                self.xgate(q)
            elif k == 3:
                self.h(q)
                self.zgate(q)
        else:
            raise ValueError(kind)

    def _row(self, i):
        return [(int(self.x[i, j]), int(self.z[i, j])) for j in range(self.n)], 2 * int(self.r[i])

    def expectation(self, x, z):
        """<P(x,z)> with P(x,z) = prod_j sigma_j (Y where both bits set)."""
        n = self.n
        px = np.array([(x >> j) & 1 for j in range(n)], dtype=np.uint8)
        pz = np.array([(z >> j) & 1 for j in range(n)], dtype=np.uint8)
        # anticommutes with stabiliser i  <=>  symplectic product is odd
        for i in range(n, 2 * n):
            if (int(np.sum(self.x[i] & pz)) + int(np.sum(self.z[i] & px))) % 2:
                return 0.0
        prod = [(0, 0)] * n
        k = 0
        for i in range(n):
            if (int(np.sum(self.x[i] & pz)) + int(np.sum(self.z[i] & px))) % 2:
                row, kr = self._row(n + i)
                k += kr
                for j in range(n):
                    kk, c = _mul1(prod[j], row[j])
                    k += kk
                    prod[j] = c
        target = [(int(px[j]), int(pz[j])) for j in range(n)]
        assert prod == target
        ph = (1, 1j, -1, -1j)[k % 4]
        assert abs(ph.imag) < 1e-12
        return float(ph.real)


def clifford_expectations(n, gates, params, terms):
    """Run a circuit whose rotation angles are multiples of pi/2; return <P> per (x, z)."""
    T = Tableau(n)
    for (kind, q0, q1, pidx, angle) in gates:
        a = params[pidx] if pidx >= 0 else angle
        if kind == "CNOT":
            T.cnot(q0, q1)
        elif kind in ("RY", "RZ"):
            T.apply(kind, q0, a)
        elif kind == "H":
            T.h(q0)
        elif kind == "X":
            T.xgate(q0)
        elif kind == "CZ":
            T.h(q1)
            T.cnot(q0, q1)
            T.h(q1)
        else:
            raise ValueError(kind)
    return [T.expectation(int(x), int(z)) for (x, z) in terms]
