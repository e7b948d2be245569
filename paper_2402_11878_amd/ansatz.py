"""Gate lists for the library's circuits.

The layered hardware-efficient ansatz used by the workloads: L layers of
[RY on every qubit; RZ on every qubit; CNOT q -> q+1 for q = 0 .. n-2], with
layer l using theta[l*2n + q] for RY(q) and theta[l*2n + n + q] for RZ(q).
It stands in for the paper's CISD-derived S/D excitation ansatz (eq. 5),
which needs molecular data not available here.
"""
from __future__ import annotations

import numpy as np

from . import _lib


def gates_array(gates):
    """List of (kind, q0, q1, param_index, angle) -> structured array for the C ABI."""
    a = np.zeros(len(gates), dtype=_lib.GATE_DTYPE)
    for i, (k, q0, q1, p, ang) in enumerate(gates):
        a[i] = (k, q0, max(q1, 0), 0, p, ang)
    return a


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
