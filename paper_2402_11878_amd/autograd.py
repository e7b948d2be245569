"""torch.autograd.Function for the VQE energy E(theta) = <psi|H|psi>/<psi|psi>
(eq. 7) whose backward is the adjoint gradient computed by libvqe.so.

When theta needs a gradient, the forward call runs one fused forward sweep,
lam = H psi and the reverse sweep, so the gradient is ready when backward is
called (about three circuit costs in all, against 2P + 1 circuit runs for
parameter shift).  Otherwise (theta without requires_grad, or under
torch.no_grad) it runs the forward sweep and the grouped energy only (eq. 7),
about one circuit cost.  State buffers are kept in a workspace keyed by
(qubits, dtype, checkpoints) and reused across calls.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib
from .core import State


class Workspace:
    """Device state buffers reused across evaluations."""

    def __init__(self):
        self._cache = {}

    def get(self, n, dtype, n_ckpt, count=None):
        """The first `count` (default 2 + n_ckpt: psi, lam and the
        checkpoints) states of the entry for (n, dtype, n_ckpt) on the
        current stream, allocated on first use."""
        key = (n, dtype, n_ckpt, torch.cuda.current_stream().cuda_stream)
        states = self._cache.setdefault(key, [])
        want = 2 + n_ckpt if count is None else count
        while len(states) < want:
            states.append(State(n, dtype))
        return states[:want]

    def clear(self):
        for states in self._cache.values():
            for s in states:
                s.free()
        self._cache.clear()


_default = None


def default_workspace():
    global _default
    if _default is None:
        _default = Workspace()
    return _default


class EnergyFn(torch.autograd.Function):
    """E = EnergyFn.apply(theta, hamiltonian, circuit, dtype="c64", n_ckpt=0, workspace=None).

    theta: 1-D tensor of the circuit's n_params angles (any device, float
    dtype).  Returns a 0-d tensor of theta's dtype and device.
    """

    @staticmethod
    def forward(ctx, theta, hamiltonian, circuit, dtype="c64", n_ckpt=0, workspace=None):
        ws = workspace or default_workspace()
        if not ctx.needs_input_grad[0]:
            return _energy_only(theta, hamiltonian, circuit, dtype, ws)
        states = ws.get(circuit.n, dtype, n_ckpt)
        th = theta.detach().to("cpu", torch.float64).numpy()
        E, g = _lib.vqe_energy_grad(states[0].handle, states[1].handle, circuit.handle, th, hamiltonian.handle,
                                    ckpt=[s.handle for s in states[2:]])
        ctx.save_for_backward(torch.from_numpy(np.asarray(g)).to(device=theta.device, dtype=theta.dtype))
        return torch.tensor(E, dtype=theta.dtype, device=theta.device)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g, None, None, None, None, None


def _energy_only(theta, hamiltonian, circuit, dtype, ws):
    """E(theta) without the gradient: psi = U(theta)|0...0>, then the grouped
    energy <psi|H|psi>/<psi|psi>."""
    psi = ws.get(circuit.n, dtype, 0, count=1)[0]  # no lam: the energy needs psi only
    th = theta.detach().to("cpu", torch.float64).numpy()
    _lib.vqe_state_set_basis(psi.handle, 0)
    _lib.vqe_apply_circuit(psi.handle, circuit.handle, th)
    E, _ = _lib.vqe_expect_pauli(psi.handle, hamiltonian.handle, _lib.EXPECT_GROUPED)
    return torch.tensor(E, dtype=theta.dtype, device=theta.device)


def energy(theta, hamiltonian, circuit, dtype="c64", n_ckpt=0, workspace=None):
    """E(theta); the adjoint sweep runs only when theta needs a gradient."""
    if not (torch.is_grad_enabled() and theta.requires_grad):
        return _energy_only(theta, hamiltonian, circuit, dtype, workspace or default_workspace())
    return EnergyFn.apply(theta, hamiltonian, circuit, dtype, n_ckpt, workspace)
