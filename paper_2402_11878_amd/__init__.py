"""MI355X (gfx950) VQE state-vector hot path (arXiv 2402.11878).

The computation lives in libvqe.so (hand-written HIP kernels behind a C ABI,
declared in include/vqe.h); this package is its Python binding:
  _lib          ctypes entry points with the C names
  core          State / Circuit / Hamiltonian handles (torch for memory, streams)
  hamiltonians  Jordan-Wigner Hamiltonians on bit masks
  ansatz        gate lists of the layered ansatz
  autograd      torch.autograd.Function for the energy and its adjoint gradient
  serving       continuous-batching request loop
"""
from . import _lib
from ._lib import VqeError

__all__ = ["_lib", "VqeError"]
