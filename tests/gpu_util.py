"""Helpers for the GPU parity tests: library calls through the C ABI on
states whose memory torch provides, and oracle references on the CPU."""
import sys

import numpy as np

from oracle import statevector as osv
from paper_2402_11878_amd import _lib

NAMES = {0: "RY", 1: "RZ", 2: "RX", 3: "H", 4: "X", 5: "CNOT", 6: "CZ", 7: "SEXC", 8: "DEXC"}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_gates(arr):
    out = []
    for g in arr:
        k = int(g["kind"])
        if k == 7:
            out.append(("SEXC", (int(g["q0"]), int(g["q1"])), -1, int(g["param_index"]), float(g["angle"])))
        elif k == 8:
            out.append(("DEXC", (int(g["q0"]), int(g["q1"]), int(g["q2"]), int(g["q3"])), -1,
                        int(g["param_index"]), float(g["angle"])))
        else:
            out.append((NAMES[k], int(g["q0"]), int(g["q1"]), int(g["param_index"]), float(g["angle"])))
    return out


class Dev:
    """A state handle on torch-owned device memory (torch's current stream)."""

    def __init__(self, n, dtype):
        import torch
        self.n, self.dtype = n, dtype
        tdt = torch.complex64 if dtype == _lib.VQE_C64 else torch.complex128
        self.t = torch.empty(1 << n, dtype=tdt, device="cuda")
        st = torch.cuda.current_stream().cuda_stream
        self.h = _lib.vqe_state_alloc(n, dtype, self.t.data_ptr(), self.t.numel() * self.t.element_size(), st)

    def read(self):
        return _lib.vqe_state_read(self.h, 0, 1 << self.n, self.dtype)

    def free(self):
        if self.h:
            _lib.vqe_state_free(self.h)
            self.h = None
        self.t = None


def tol_energy(dtype):
    return 1e-10 if dtype == _lib.VQE_C128 else 1e-5


def rel_err(a, b):
    return abs(a - b) / max(abs(b), 1.0)
