"""Handle classes over the C ABI, with PyTorch as the device-memory and
stream provider.

A ``State`` borrows a torch CUDA (HIP) tensor of 2^n complex amplitudes and
runs on torch's current stream; ``Circuit`` and ``Hamiltonian`` wrap the
library's handles.  All computation runs in libvqe.so.
"""
from __future__ import annotations

import numpy as np

from . import _lib
from . import ansatz as _ansatz


def _torch():
    import torch
    return torch


class State:
    """2^n amplitudes in device memory (qubit j = bit j of the index)."""

    def __init__(self, n_qubits, dtype="c64", tensor=None, device=None, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("State needs a HIP device")
        self.n = int(n_qubits)
        self.dtype = _lib.VQE_C64 if dtype in ("c64", _lib.VQE_C64, torch.complex64) else _lib.VQE_C128
        tdt = torch.complex64 if self.dtype == _lib.VQE_C64 else torch.complex128
        if tensor is None:
            tensor = torch.empty(1 << self.n, dtype=tdt, device=device or "cuda")
        if tensor.dtype != tdt or not tensor.is_cuda or not tensor.is_contiguous() or tensor.numel() < (1 << self.n):
            raise ValueError("tensor must be a contiguous device tensor of 2^n amplitudes of the state's dtype")
        self.tensor = tensor
        st = stream if stream is not None else torch.cuda.current_stream(tensor.device)
        self.stream = st
        self.handle = _lib.vqe_state_alloc(self.n, self.dtype, tensor.data_ptr(),
                                           tensor.numel() * tensor.element_size(), st.cuda_stream)

    def set_basis(self, b=0):
        _lib.vqe_state_set_basis(self.handle, b)

    def read(self, offset=0, count=None):
        count = (1 << self.n) - offset if count is None else count
        return _lib.vqe_state_read(self.handle, offset, count, self.dtype)

    def write(self, values, offset=0):
        _lib.vqe_state_write(self.handle, offset, values, self.dtype)

    def free(self):
        if getattr(self, "handle", None):
            _lib.vqe_state_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Circuit:
    def __init__(self, n_qubits, gates):
        self.n = int(n_qubits)
        self.gates = np.ascontiguousarray(gates, dtype=_lib.GATE_DTYPE)
        self.handle = _lib.vqe_circuit_create(self.n, self.gates)
        self.n_params, self.n_passes = _lib.vqe_circuit_info(self.handle)

    @classmethod
    def layered(cls, n, layers):
        return cls(n, _ansatz.layered(n, layers))

    def passes(self, dtype=_lib.VQE_C64):
        out = []
        for p in range(self.passes_count(dtype)):
            out.append(_lib.vqe_circuit_pass(self.handle, dtype, p))
        return out

    def passes_count(self, dtype=_lib.VQE_C64):
        n = 0
        while True:
            try:
                _lib.vqe_circuit_pass(self.handle, dtype, n)
            except _lib.VqeError:
                return n
            n += 1

    def apply(self, state, params):
        _lib.vqe_apply_circuit(state.handle, self.handle, params)

    def free(self):
        if getattr(self, "handle", None):
            _lib.vqe_circuit_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Hamiltonian:
    """H = sum_i w_i P(x_i, z_i) (eqs. 2-4), grouped by X mask in the library."""

    def __init__(self, n_qubits, x, z, w):
        self.n = int(n_qubits)
        self.x = np.ascontiguousarray(x, dtype=np.uint64)
        self.z = np.ascontiguousarray(z, dtype=np.uint64)
        self.w = np.ascontiguousarray(w, dtype=np.float64)
        self.handle = _lib.vqe_hamiltonian_create(self.n, self.x, self.z, self.w)
        self.n_terms, self.n_groups, self.identity = _lib.vqe_hamiltonian_info(self.handle)

    def slim(self, mode, value):
        """Slimmed copy (Sec. II-D): returns (Hamiltonian, dropped sum of |w|)."""
        keep, _, dropped = _lib.vqe_slim_hamiltonian(self.x, self.z, self.w, mode, value)
        k = keep.astype(bool)
        return Hamiltonian(self.n, self.x[k], self.z[k], self.w[k]), dropped

    def expect(self, state, mode=_lib.EXPECT_GROUPED):
        return _lib.vqe_expect_pauli(state.handle, self.handle, mode)

    def free(self):
        if getattr(self, "handle", None):
            _lib.vqe_hamiltonian_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def energy_grad(psi, lam, circuit, params, ham, method=_lib.GRAD_ADJOINT, expect_mode=_lib.EXPECT_GROUPED,
                ckpt=()):
    return _lib.vqe_energy_grad(psi.handle, lam.handle if lam is not None else None, circuit.handle, params,
                                ham.handle, method, expect_mode, [c.handle for c in ckpt])
