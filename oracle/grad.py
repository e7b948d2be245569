"""Gradients of E(theta) (oracle side).

The paper's optimiser runs one circuit per parameter per iteration (the N_p
independent runs of Sec. II-C); here the same derivatives are computed three
independent ways:
  * parameter shift, exact for R(t) = exp(-i t G/2) with G^2 = I:
      dE/dt_k = [E(t + pi/2 e_k) - E(t - pi/2 e_k)] / 2;
    and, for excitation gates (eigenvalues of G in {0, +-1}, so E(t) holds
    frequencies 1/2 and 1), the four-term rule of Anselmetti et al. (2021):
      dE/dt_k = d1 [E(t + a) - E(t - a)] - d2 [E(t + b) - E(t - b)],
      a = pi/2, b = 3 pi/2, d1 = (sqrt2 + 1)/(4 sqrt2), d2 = (sqrt2 - 1)/(4 sqrt2);
  * central finite differences with step h;
  * adjoint reverse sweep (Jones & Gacon 2020): with lambda = H psi, walk the
    gates backwards; just after gate k, dE/dt_k = Im<lambda|G_k|psi>/<psi|psi>,
    then un-apply gate k from both psi and lambda.
"""
from __future__ import annotations

import math

import numpy as np

from . import expect, statevector as sv


def _energy(n, gates, params, H):
    psi = sv.run(n, gates, params)
    return expect.energy(psi, n, H)[0]


def _check_single_use(gates, n_params):
    counts = np.zeros(n_params, dtype=int)
    for g in gates:
        if g[3] >= 0:
            counts[g[3]] += 1
    assert np.all(counts <= 1), "parameter shift here assumes each parameter drives one gate"


def _shifted(n, gates, params, H, k, d):
    tp = params.copy()
    tp[k] += d
    tm = params.copy()
    tm[k] -= d
    return _energy(n, gates, tp, H) - _energy(n, gates, tm, H)


def param_shift(n, gates, params, H, indices=None):
    params = np.asarray(params, dtype=np.float64)
    _check_single_use(gates, len(params))
    kind_of = {g[3]: g[0] for g in gates if g[3] >= 0}
    idx = range(len(params)) if indices is None else indices
    r2 = math.sqrt(2.0)
    d1, d2 = (r2 + 1) / (4 * r2), (r2 - 1) / (4 * r2)
    out = {}
    for k in idx:
        if kind_of.get(k) in sv.EXCITATIONS:
            out[k] = d1 * _shifted(n, gates, params, H, k, math.pi / 2) - \
                d2 * _shifted(n, gates, params, H, k, 3 * math.pi / 2)
        else:
            out[k] = 0.5 * _shifted(n, gates, params, H, k, math.pi / 2)
    return out


def finite_diff(n, gates, params, H, indices=None, h=1e-4):
    params = np.asarray(params, dtype=np.float64)
    idx = range(len(params)) if indices is None else indices
    out = {}
    for k in idx:
        tp = params.copy()
        tp[k] += h
        tm = params.copy()
        tm[k] -= h
        out[k] = (_energy(n, gates, tp, H) - _energy(n, gates, tm, H)) / (2 * h)
    return out


def adjoint(n, gates, params, H):
    """Energy and the full gradient by one reverse sweep; returns (E, grad)."""
    params = np.asarray(params, dtype=np.float64)
    psi = sv.run(n, gates, params)
    lam = expect.apply_hamiltonian(psi, n, H)
    norm = float(np.vdot(psi, psi).real)
    E = float(np.vdot(psi, lam).real) / norm
    grad = np.zeros(len(params))
    for g in reversed(gates):
        kind, q0, q1, pidx, angle = g
        if pidx >= 0 and kind in sv.ROTATIONS:
            Gpsi = sv.apply_1q(psi.copy(), n, q0, sv.generator(kind))
            grad[pidx] += float(np.vdot(lam, Gpsi).imag) / norm
        elif pidx >= 0 and kind in sv.EXCITATIONS:
            Gpsi = sv.apply_excitation_generator(psi, n, kind, q0)
            grad[pidx] += float(np.vdot(lam, Gpsi).imag) / norm
        sv.apply_gate(psi, n, g, params, inverse=True)
        sv.apply_gate(lam, n, g, params, inverse=True)
    return E, grad
