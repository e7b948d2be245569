"""Gate lists for the library's circuits.

* The layered hardware-efficient ansatz used by the benchmark workloads: L
  layers of [RY on every qubit; RZ on every qubit; CNOT q -> q+1 for
  q = 0 .. n-2], with layer l using theta[l*2n + q] for RY(q) and
  theta[l*2n + n + q] for RZ(q).
* The paper's form (eq. 5): excitation gates from the Hartree-Fock reference
  (eq. 6).  The paper keeps the excitations whose CISD coefficients pass a
  threshold and starts from those coefficients; without molecular CISD data,
  `excitations` takes every spin-conserving single and double excitation
  from the occupied to the virtual spin-orbitals (UCCSD-like selection).
"""
from __future__ import annotations

import numpy as np

from . import _lib


def gates_array(gates):
    """Gates -> structured array for the C ABI.  Each gate is
    (kind, q0, q1, param_index, angle), or for excitation gates
    (kind, (q0, q1[, q2, q3]), param_index, angle)."""
    a = np.zeros(len(gates), dtype=_lib.GATE_DTYPE)
    for i, g in enumerate(gates):
        if len(g) == 4:
            k, qs, p, ang = g
            qs = tuple(qs) + (0,) * (4 - len(qs))
        else:
            k, q0, q1, p, ang = g
            qs = (q0, max(q1, 0), 0, 0)
        a[i]["kind"] = k
        a[i]["q0"], a[i]["q1"], a[i]["q2"], a[i]["q3"] = qs
        a[i]["param_index"] = p
        a[i]["angle"] = ang
    return a


def hartree_fock(n_electrons):
    """Basis index of the Hartree-Fock reference (spin-orbitals 0 .. N_e - 1 occupied)."""
    return (1 << n_electrons) - 1


def excitations(n, n_electrons, layers=1, reference=True):
    """Single then double excitation gates, spin-conserving (spin-orbital
    2 i + sigma), occupied -> virtual, `layers` repetitions with fresh
    parameters, preceded (reference=True) by X on the occupied spin-orbitals
    so that the circuit maps |0...0> to U(theta)|HF>; returns (gates array,
    number of parameters)."""
    occ, vir = range(n_electrons), range(n_electrons, n)
    spin = lambda q: q & 1
    singles = [(i, a) for i in occ for a in vir if spin(i) == spin(a)]
    doubles = [(i, j, a, b) for i in occ for j in occ if i < j for a in vir for b in vir
               if a < b and spin(i) + spin(j) == spin(a) + spin(b)]
    g = [(_lib.GATE_X, q, 0, -1, 0.0) for q in occ] if reference else []
    k = 0
    for _ in range(layers):
        for q in singles:
            g.append((_lib.GATE_SEXC, q, k, 0.0))
            k += 1
        for q in doubles:
            g.append((_lib.GATE_DEXC, q, k, 0.0))
            k += 1
    return gates_array(g), k


def layered(n, layers):
    g = []
    for l in range(layers):
        for q in range(n):
            g.append((_lib.GATE_RY, q, 0, l * 2 * n + q, 0.0))
        for q in range(n):
            g.append((_lib.GATE_RZ, q, 0, l * 2 * n + n + q, 0.0))
        for q in range(n - 1):
            g.append((_lib.GATE_CNOT, q, q + 1, -1, 0.0))
    return gates_array(g)
