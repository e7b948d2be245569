"""Gate-by-gate FP64 state-vector simulator (oracle side).

psi(theta) = U(theta) psi_ref (eq. 6), with U a product of gates applied one
at a time to 2^n complex128 amplitudes; memory 2^(n+4) bytes (Sec. I).
No fusion, no reordering.

Conventions (the paper, whose ansatz is built from S/D excitation gate sets
(eq. 5), does not fix the matrices of the hardware-efficient ansatz used here):
  qubit j = bit j of the basis index;
  RY(t) = exp(-i t Y/2) = [[c, -s], [s, c]],  c = cos(t/2), s = sin(t/2);
  RZ(t) = exp(-i t Z/2) = diag(e^{-it/2}, e^{+it/2});
  RX(t) = exp(-i t X/2) = [[c, -is], [-is, c]];
  CNOT(c -> t) maps |b> to |b xor (b_c << t)>;  CZ(a, b) = (-1)^{b_a b_b}.
The paper's excitation gate sets (eq. 5; one- and two-electron excitations in
the style of the gate-fabric ansatz) are read as particle-number-conserving
real rotations by t/2 inside a two-state subspace, without Jordan-Wigner
strings:
  SEXC(t) on qubits (p, q): A = {b_p = 1, b_q = 0}, B = {b_p = 0, b_q = 1};
  DEXC(t) on qubits (p, q, r, s): A = {b_p = b_q = 1, b_r = b_s = 0},
                                  B = {b_p = b_q = 0, b_r = b_s = 1};
  for every pair (a in A, a' = a with the A bits replaced by the B bits):
      psi'[a] = c psi[a] - s psi[a'],  psi'[a'] = s psi[a] + c psi[a'];
  all other amplitudes unchanged.  R(t) = exp(-i t G / 2) with
  G = i(|B><A| - |A><B|) on each pair, whose eigenvalues are 0 and +-1.
A circuit is a list of gates (kind, q0, q1, param_index, angle); for SEXC and
DEXC the q0 slot holds the tuple of qubits (p, q) or (p, q, r, s) and q1 is -1.
A gate with param_index >= 0 takes its angle from the parameter vector, else
``angle``.
"""
from __future__ import annotations

import math

import numpy as np

RY, RZ, RX, H, X, CNOT, CZ = "RY", "RZ", "RX", "H", "X", "CNOT", "CZ"
SEXC, DEXC = "SEXC", "DEXC"
ROTATIONS = (RY, RZ, RX)
EXCITATIONS = (SEXC, DEXC)


def basis_state(n, b=0):
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[b] = 1.0
    return psi


def gate_matrix(kind, angle=0.0):
    c, s = math.cos(angle / 2.0), math.sin(angle / 2.0)
    if kind == RY:
        return np.array([[c, -s], [s, c]], dtype=np.complex128)
    if kind == RZ:
        return np.array([[complex(c, -s), 0], [0, complex(c, s)]], dtype=np.complex128)
    if kind == RX:
        return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)
    if kind == H:
        r = 1.0 / math.sqrt(2.0)
        return np.array([[r, r], [r, -r]], dtype=np.complex128)
    if kind == X:
        return np.array([[0, 1], [1, 0]], dtype=np.complex128)
    raise ValueError(kind)


def generator(kind):
    """G with R(t) = exp(-i t G / 2)."""
    if kind == RY:
        return np.array([[0, -1j], [1j, 0]])
    if kind == RZ:
        return np.array([[1, 0], [0, -1]], dtype=np.complex128)
    if kind == RX:
        return np.array([[0, 1], [1, 0]], dtype=np.complex128)
    raise ValueError(kind)


def apply_1q(psi, n, q, U):
    """Apply a 2x2 matrix U to qubit q; psi viewed as (2^(n-q-1), 2, 2^q)."""
    v = psi.reshape(1 << (n - q - 1), 2, 1 << q)
    a = v[:, 0, :].copy()
    b = v[:, 1, :].copy()
    v[:, 0, :] = U[0, 0] * a + U[0, 1] * b
    v[:, 1, :] = U[1, 0] * a + U[1, 1] * b
    return psi


def apply_dense(psi, n, qubits, U):
    """psi <- U psi for a dense 2^k x 2^k matrix on k listed qubits (a fused
    window of the circuit of eq. 6 as one matrix).  Bit i of U's row and
    column indices is qubit qubits[i].  Definition, for every basis index b:
        psi'[b] = sum_p U[pat(b), p] psi[rest(b) | off(p)],
    pat(b) = the window bits of b in list order, rest(b) = b with the window
    bits cleared, off(p) = the window bits of pattern p placed at their
    qubits."""
    k = len(qubits)
    idx = np.arange(1 << n, dtype=np.int64)
    pat = np.zeros_like(idx)
    rest = idx.copy()
    for i, q in enumerate(qubits):
        pat |= ((idx >> q) & 1) << i
        rest &= ~(1 << q)
    src = psi.copy()
    out = np.zeros_like(psi)
    for p in range(1 << k):
        off = 0
        for i, q in enumerate(qubits):
            if (p >> i) & 1:
                off |= 1 << q
        out += U[pat, p] * src[rest | off]
    psi[:] = out
    return psi


def apply_cnot(psi, n, c, t):
    """Swap the target pairs inside the control = 1 slice."""
    idx = np.arange(1 << n, dtype=np.int64)
    sel = ((idx >> c) & 1 == 1) & ((idx >> t) & 1 == 0)
    i0 = idx[sel]
    i1 = i0 | (1 << t)
    tmp = psi[i0].copy()
    psi[i0] = psi[i1]
    psi[i1] = tmp
    return psi


def apply_cz(psi, n, a, b):
    idx = np.arange(1 << n, dtype=np.int64)
    sel = ((idx >> a) & 1 == 1) & ((idx >> b) & 1 == 1)
    psi[sel] *= -1.0
    return psi


def excitation_patterns(kind, qubits):
    """(mask, A pattern, B pattern) of an excitation gate on `qubits`."""
    bit = [1 << q for q in qubits]
    if kind == SEXC:
        p, q = bit
        return p | q, p, q
    p, q, r, s = bit
    return p | q | r | s, p | q, r | s


def apply_excitation(psi, n, kind, qubits, angle):
    """Rotation by angle/2 between the A and B patterns (see the module docstring)."""
    mask, A, B = excitation_patterns(kind, qubits)
    idx = np.arange(1 << n, dtype=np.int64)
    ia = idx[(idx & mask) == A]
    ib = ia ^ A ^ B
    c, s = math.cos(angle / 2.0), math.sin(angle / 2.0)
    a = psi[ia].copy()
    b = psi[ib].copy()
    psi[ia] = c * a - s * b
    psi[ib] = s * a + c * b
    return psi


def apply_excitation_generator(psi, n, kind, qubits):
    """G psi with G = i(|B><A| - |A><B|) on every pair; zero elsewhere."""
    mask, A, B = excitation_patterns(kind, qubits)
    idx = np.arange(1 << n, dtype=np.int64)
    ia = idx[(idx & mask) == A]
    ib = ia ^ A ^ B
    out = np.zeros_like(psi)
    out[ib] = 1j * psi[ia]
    out[ia] = -1j * psi[ib]
    return out


def gate_angle(g, params):
    kind, q0, q1, pidx, angle = g
    return params[pidx] if pidx >= 0 else angle


def apply_gate(psi, n, g, params, inverse=False):
    kind, q0, q1, pidx, angle = g
    if kind in EXCITATIONS:
        t = gate_angle(g, params)
        return apply_excitation(psi, n, kind, q0, -t if inverse else t)
    if kind == CNOT:
        return apply_cnot(psi, n, q0, q1)
    if kind == CZ:
        return apply_cz(psi, n, q0, q1)
    U = gate_matrix(kind, gate_angle(g, params))
    if inverse:
        U = U.conj().T
    return apply_1q(psi, n, q0, U)


def run(n, gates, params, psi=None):
    """psi = G_m ... G_1 psi_ref, one gate at a time (default psi_ref = |0...0>)."""
    psi = basis_state(n) if psi is None else psi.copy()
    for g in gates:
        apply_gate(psi, n, g, params)
    return psi


def hartree_fock_index(n_electrons):
    """Basis index of the Hartree-Fock reference: spin-orbitals 0..N_e-1 occupied."""
    return (1 << n_electrons) - 1


def excitation_ansatz(n, n_electrons, layers=1):
    """Spin-conserving single and double excitations from the occupied
    spin-orbitals 0..N_e-1 (spin-orbital 2i + sigma) to the virtual ones,
    singles first and then doubles (eq. 5 applies the D product after the S
    product), repeated `layers` times with fresh parameters."""
    occ = list(range(n_electrons))
    vir = list(range(n_electrons, n))
    singles = [(i, a) for i in occ for a in vir if (i - a) % 2 == 0]
    doubles = [(i, j, a, b) for ii, i in enumerate(occ) for j in occ[ii + 1:]
               for ai, a in enumerate(vir) for b in vir[ai + 1:]
               if (i % 2 + j % 2) == (a % 2 + b % 2)]
    gates, k = [], 0
    for _ in range(layers):
        for (i, a) in singles:
            gates.append((SEXC, (i, a), -1, k, 0.0))
            k += 1
        for (i, j, a, b) in doubles:
            gates.append((DEXC, (i, j, a, b), -1, k, 0.0))
            k += 1
    return gates


def layered_ansatz(n, layers):
    """L layers of [RY on every qubit; RZ on every qubit; CNOT q -> q+1 ladder].

    Layer l uses theta[l*2n + q] for RY on qubit q and theta[l*2n + n + q] for
    RZ on qubit q; the ladder runs q = 0 .. n-2 in ascending order.
    """
    gates = []
    for l in range(layers):
        for q in range(n):
            gates.append((RY, q, -1, l * 2 * n + q, 0.0))
        for q in range(n):
            gates.append((RZ, q, -1, l * 2 * n + n + q, 0.0))
        for q in range(n - 1):
            gates.append((CNOT, q, q + 1, -1, 0.0))
    return gates
