"""The classical loop around the device: minimise E(theta) (eq. 7 over the
ansatz of eqs. 5-6, the VQE main part of the paper's Fig. 1 flow) with the
energy and adjoint gradient of `vqe_energy_grad`, and the cutoff-ratio
search of Algorithm 1.

The paper optimises with SLSQP (few circuit runs in a noiseless setting,
Sec. II-B); here the gradient comes from one adjoint sweep instead of one
circuit run per parameter.

Algorithm 1 as printed is garbled (no decrement of the ratio, mismatched
names); it is read as: with the N non-identity terms ordered by importance
and E_k the converged energy with the top floor(N k / 10) of them kept (k = 10
is the full Hamiltonian), walk k = 10, 9, ..., 1 and return (k + 1)/10 at the
first k with |E_k - E_10| >= delta_E, or 0.1 if none.  Integer tenths avoid
the drift of repeated `ratio - 0.1`.  The identity term is always kept.
"""
from __future__ import annotations

import numpy as np

from . import _lib


def minimize(n, circuit, hamiltonian, theta0, dtype=_lib.VQE_C128, method="SLSQP", tol=1e-12, maxiter=1000):
    """Minimise E(theta) for circuit and Hamiltonian handles of n qubits from
    theta0 with scipy's `method` and the device gradient.  Returns a dict:
    energy, theta, grad_norm, n_evals, n_iter, success, message."""
    import torch
    from scipy.optimize import minimize as sp_minimize

    from .core import State
    kind = "c128" if dtype == _lib.VQE_C128 else "c64"
    psi, lam = State(n, kind), State(n, kind)
    evals = [0]

    def fun(theta):
        E, g = _lib.vqe_energy_grad(psi.handle, lam.handle, circuit, np.asarray(theta, dtype=np.float64), hamiltonian)
        evals[0] += 1
        return E, g

    try:
        opts = {"maxiter": maxiter}
        if method in ("SLSQP",):
            opts["ftol"] = tol
        else:
            opts["gtol"] = tol
        res = sp_minimize(fun, np.asarray(theta0, dtype=np.float64), jac=True, method=method, options=opts)
        E, g = fun(res.x)
        torch.cuda.synchronize()
        return {"energy": float(E), "theta": res.x, "grad_norm": float(np.linalg.norm(g)), "n_evals": evals[0],
                "n_iter": int(getattr(res, "nit", 0)), "success": bool(res.success), "message": str(res.message)}
    finally:
        psi.free()
        lam.free()


def kept_terms(x, z, w, k):
    """Keep mask of the top floor(N k / 10) non-identity terms (N of them) in
    the order of importance, plus the identity, and the number of terms kept
    (vqe_slim_hamiltonian, KEEP_TOP)."""
    n_nonid = int(np.count_nonzero((np.asarray(x) != 0) | (np.asarray(z) != 0)))
    keep, n_kept, _ = _lib.vqe_slim_hamiltonian(x, z, w, _lib.SLIM_KEEP_TOP, (n_nonid * k) // 10)
    return keep, n_kept


def cutoff_ratio(energy_of_tenths, delta_e):
    """Algorithm 1 (read as in the module docstring): energy_of_tenths(k)
    returns the converged energy with the top k tenths of the terms kept;
    returns the kept fraction as a float in {0.1, ..., 1.0} (1.0 when already
    the first cut, to 9 tenths, moves the energy by delta_e or more)."""
    e_full = energy_of_tenths(10)
    for k in range(10, 0, -1):
        e_k = e_full if k == 10 else energy_of_tenths(k)
        if abs(e_k - e_full) >= delta_e:
            return (k + 1) / 10.0
    return 0.1


def cutoff_ratio_vqe(n, x, z, w, circuit, theta0, delta_e, dtype=_lib.VQE_C128, method="SLSQP"):
    """Algorithm 1 on the device: for each k the Hamiltonian keeps the top
    floor(N k / 10) of its N non-identity terms in the order of importance
    (`kept_terms`), is minimised from theta0, and the rule of `cutoff_ratio`
    picks the ratio.  Returns (ratio, {k: energy})."""
    energies = {}

    def energy_of_tenths(k):
        keep, _ = kept_terms(x, z, w, k)
        m = keep == 1
        h = _lib.vqe_hamiltonian_create(n, x[m], z[m], w[m])
        try:
            energies[k] = minimize(n, circuit, h, theta0, dtype=dtype, method=method)["energy"]
        finally:
            _lib.vqe_hamiltonian_free(h)
        return energies[k]

    return cutoff_ratio(energy_of_tenths, delta_e), energies
