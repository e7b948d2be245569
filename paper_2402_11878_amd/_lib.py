"""ctypes binding of libvqe.so: one Python function per C entry point.

Argument marshalling only; every step of the computation runs in the
library.  Importing this module loads the in-tree libvqe.so and raises if it
is missing (build it with ``python -m paper_2402_11878_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvqe.so")

VQE_OK, VQE_ERR_ARG, VQE_ERR_OOM, VQE_ERR_DEVICE, VQE_ERR_UNSUPPORTED, VQE_ERR_STATE = 0, -1, -2, -3, -4, -5
VQE_C64, VQE_C128 = 1, 2
GATE_RY, GATE_RZ, GATE_RX, GATE_H, GATE_X, GATE_CNOT, GATE_CZ, GATE_SEXC, GATE_DEXC = range(9)
EXPECT_GROUPED, EXPECT_PER_TERM = 0, 1
GRAD_ADJOINT, GRAD_PARAM_SHIFT = 0, 1
SLIM_THRESHOLD, SLIM_REMOVE_PERCENT, SLIM_BUDGET, SLIM_KEEP_TOP = 0, 1, 2, 3
SPECIALIZE_NEVER, SPECIALIZE_AUTO, SPECIALIZE_ALWAYS = 0, 1, 2
SPECIALIZE_AUTO_MIN_QUBITS = 20
MAX_WINDOW = 7
KERNEL_WINDOW_FWD, KERNEL_WINDOW_REV, KERNEL_HPSI, KERNEL_EXPECT_HALF, KERNEL_PER_TERM, KERNEL_DENSE = range(6)
KERNEL_KINDS = 6
NOALLOC_SCRATCH_BYTES = 65792
DENSE_K = 5


class VqeError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed ({code}): {msg}")
        self.code = code


class vqe_gate(C.Structure):
    _fields_ = [("kind", C.c_uint8), ("q0", C.c_uint8), ("q1", C.c_uint8), ("q2", C.c_uint8), ("q3", C.c_uint8),
                ("reserved", C.c_uint8 * 3), ("param_index", C.c_int32), ("reserved2", C.c_int32),
                ("angle", C.c_double)]


class vqe_grad_opts(C.Structure):
    _fields_ = [("method", C.c_int32), ("expect_mode", C.c_int32), ("n_ckpt", C.c_int32),
                ("chunk_passes", C.c_int32), ("ckpt", C.POINTER(C.c_void_p))]


class vqe_batch_item(C.Structure):
    _fields_ = [("circuit", C.c_void_p), ("hamiltonian", C.c_void_p), ("params", C.POINTER(C.c_double)),
                ("n_params", C.c_size_t), ("energy", C.POINTER(C.c_double)), ("grad", C.POINTER(C.c_double))]


BATCH_MAX_QUBITS = {1: 13, 2: 12}  # whole state in LDS (complex64, complex128)
BATCH_MAX_QUBITS_MID = 24          # larger items run as tile passes, up to this size
HPSI_WINDOW_QUBITS = 13            # qubits per window pass of H psi

GATE_DTYPE = np.dtype([("kind", "u1"), ("q0", "u1"), ("q1", "u1"), ("q2", "u1"), ("q3", "u1"),
                       ("reserved", "u1", (3,)), ("param_index", "<i4"), ("reserved2", "<i4"),
                       ("angle", "<f8")], align=True)
assert GATE_DTYPE.itemsize == C.sizeof(vqe_gate) == 24

_P = C.c_void_p
_SZ = C.c_size_t
_SIGS = {
    "vqe_last_error": (C.c_char_p, []),
    "vqe_version": (C.c_char_p, []),
    "vqe_device_count": (C.c_int, []),
    "vqe_state_alloc": (C.c_int, [C.c_int, C.c_int, _P, _SZ, _P, C.POINTER(_P)]),
    "vqe_state_free": (C.c_int, [_P]),
    "vqe_state_set_basis": (C.c_int, [_P, C.c_uint64]),
    "vqe_state_info": (C.c_int, [_P, C.POINTER(_P), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "vqe_state_read": (C.c_int, [_P, C.c_uint64, C.c_uint64, _P]),
    "vqe_state_write": (C.c_int, [_P, C.c_uint64, C.c_uint64, _P]),
    "vqe_circuit_create": (C.c_int, [C.c_int, _P, _SZ, C.POINTER(_P)]),
    "vqe_circuit_free": (C.c_int, [_P]),
    "vqe_circuit_info": (C.c_int, [_P, C.POINTER(_SZ), C.POINTER(_SZ)]),
    "vqe_circuit_pass": (C.c_int, [_P, C.c_int, _SZ, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                   C.POINTER(_SZ), C.POINTER(C.c_int32), _SZ]),
    "vqe_apply_circuit": (C.c_int, [_P, _P, C.POINTER(C.c_double), _SZ]),
    "vqe_apply_dense": (C.c_int, [_P, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_double)]),
    "vqe_hamiltonian_create": (C.c_int, [C.c_int, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                         C.POINTER(C.c_double), _SZ, C.POINTER(_P)]),
    "vqe_hamiltonian_free": (C.c_int, [_P]),
    "vqe_hamiltonian_info": (C.c_int, [_P, C.POINTER(_SZ), C.POINTER(_SZ), C.POINTER(C.c_double)]),
    "vqe_expect_pauli": (C.c_int, [_P, _P, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "vqe_expect_pauli_noalloc": (C.c_int, [_P, _P, _P]),
    "vqe_apply_hamiltonian": (C.c_int, [_P, _P, _P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "vqe_energy_grad": (C.c_int, [_P, _P, _P, C.POINTER(C.c_double), _SZ, _P, C.POINTER(vqe_grad_opts),
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "vqe_batch_create": (C.c_int, [C.c_int, _P, C.POINTER(_P)]),
    "vqe_batch_free": (C.c_int, [_P]),
    "vqe_batch_energy_grad": (C.c_int, [_P, _SZ, C.POINTER(vqe_batch_item)]),
    "vqe_set_specialize": (C.c_int, [C.c_int]),
    "vqe_hamiltonian_plan": (C.c_int, [_P, C.POINTER(_SZ), C.POINTER(C.c_uint64), _SZ]),
    "vqe_circuit_prepare": (C.c_int, [_P, C.c_int]),
    "vqe_stream_create": (C.c_int, [C.POINTER(C.c_uint32), _SZ, C.POINTER(_P)]),
    "vqe_stream_destroy": (C.c_int, [_P]),
    "vqe_profile_enable": (C.c_int, [C.c_int]),
    "vqe_profile_reset": (C.c_int, []),
    "vqe_profile_read": (C.c_int, [C.c_int, C.POINTER(C.c_uint64), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "vqe_slim_hamiltonian": (C.c_int, [C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_double),
                                       _SZ, C.c_int, C.c_double, C.POINTER(C.c_uint8), C.POINTER(_SZ),
                                       C.POINTER(C.c_double)]),
}

_lib = None


def lib():
    """The loaded library; raises if libvqe.so has not been built.

    torch is imported first: its bundled HIP runtime has the same SONAME as
    ROCm's, so loading torch first makes libvqe.so bind to that one runtime
    (device memory and streams from torch are then the library's too).
    Loading libvqe.so first would put a second HIP runtime in the process.
    """
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2402_11878_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def check(fn, rc):
    if rc != VQE_OK:
        raise VqeError(fn, rc, lib().vqe_last_error().decode(errors="replace"))
    return rc


def _arr(a, dtype, ctype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.POINTER(ctype))


# ----------------------------------------------------------------- thin wrappers
def vqe_version():
    return lib().vqe_version().decode()


def vqe_device_count():
    return lib().vqe_device_count()


def vqe_state_alloc(n_qubits, dtype, device_buf=None, buf_bytes=0, hip_stream=None):
    out = _P()
    check("vqe_state_alloc", lib().vqe_state_alloc(n_qubits, dtype, device_buf, buf_bytes, hip_stream, C.byref(out)))
    return out.value


def vqe_state_free(s):
    check("vqe_state_free", lib().vqe_state_free(s))


def vqe_state_set_basis(s, b):
    check("vqe_state_set_basis", lib().vqe_state_set_basis(s, b))


def vqe_state_read(s, offset, count, dtype):
    out = np.empty(count, dtype=np.complex64 if dtype == VQE_C64 else np.complex128)
    check("vqe_state_read", lib().vqe_state_read(s, offset, count, out.ctypes.data))
    return out


def vqe_state_write(s, offset, values, dtype):
    v = np.ascontiguousarray(values, dtype=np.complex64 if dtype == VQE_C64 else np.complex128)
    check("vqe_state_write", lib().vqe_state_write(s, offset, len(v), v.ctypes.data))


def vqe_circuit_create(n_qubits, gates):
    g = np.ascontiguousarray(gates, dtype=GATE_DTYPE)
    out = _P()
    check("vqe_circuit_create", lib().vqe_circuit_create(n_qubits, g.ctypes.data, len(g), C.byref(out)))
    return out.value


def vqe_circuit_free(c):
    check("vqe_circuit_free", lib().vqe_circuit_free(c))


def vqe_circuit_info(c):
    npar, npass = _SZ(), _SZ()
    check("vqe_circuit_info", lib().vqe_circuit_info(c, C.byref(npar), C.byref(npass)))
    return npar.value, npass.value


def vqe_circuit_pass(c, dtype, p):
    K = C.c_int()
    q = (C.c_int * MAX_WINDOW)()
    ng = _SZ()
    check("vqe_circuit_pass", lib().vqe_circuit_pass(c, dtype, p, C.byref(K), q, C.byref(ng), None, 0))
    idx = (C.c_int32 * max(ng.value, 1))()
    check("vqe_circuit_pass", lib().vqe_circuit_pass(c, dtype, p, None, None, None, idx, ng.value))
    return list(q)[: K.value], list(idx)[: ng.value]


def vqe_apply_circuit(s, c, params):
    p, pp = _arr(params, np.float64, C.c_double)
    check("vqe_apply_circuit", lib().vqe_apply_circuit(s, c, pp, len(p)))


def vqe_apply_dense(s, qubits, u):
    """psi <- U psi on `qubits` (bit i of U's indices is qubits[i]); u is a
    complex (2^k, 2^k) array, k = DENSE_K."""
    q, qp = _arr(qubits, np.int32, C.c_int)
    u = np.ascontiguousarray(u, dtype=np.complex128)
    if u.shape != (1 << len(q), 1 << len(q)):
        raise ValueError("u must be 2^k x 2^k for k = len(qubits)")
    uf, up = _arr(u.view(np.float64).reshape(-1), np.float64, C.c_double)
    check("vqe_apply_dense", lib().vqe_apply_dense(s, qp, len(q), up))


def vqe_hamiltonian_create(n_qubits, x, z, w):
    x, xp = _arr(x, np.uint64, C.c_uint64)
    z, zp = _arr(z, np.uint64, C.c_uint64)
    w, wp = _arr(w, np.float64, C.c_double)
    out = _P()
    check("vqe_hamiltonian_create", lib().vqe_hamiltonian_create(n_qubits, xp, zp, wp, len(w), C.byref(out)))
    return out.value


def vqe_hamiltonian_free(h):
    check("vqe_hamiltonian_free", lib().vqe_hamiltonian_free(h))


def vqe_hamiltonian_info(h):
    nt, ng, idw = _SZ(), _SZ(), C.c_double()
    check("vqe_hamiltonian_info", lib().vqe_hamiltonian_info(h, C.byref(nt), C.byref(ng), C.byref(idw)))
    return nt.value, ng.value, idw.value


def vqe_hamiltonian_plan(h):
    """Qubit masks of the window passes of H psi (empty list: the tile form)."""
    m = _SZ()
    check("vqe_hamiltonian_plan", lib().vqe_hamiltonian_plan(h, C.byref(m), None, 0))
    arr = (C.c_uint64 * max(m.value, 1))()
    check("vqe_hamiltonian_plan", lib().vqe_hamiltonian_plan(h, C.byref(m), arr, m.value))
    return [int(v) for v in arr[: m.value]]


def vqe_expect_pauli(s, h, mode=EXPECT_GROUPED):
    e, n = C.c_double(), C.c_double()
    check("vqe_expect_pauli", lib().vqe_expect_pauli(s, h, mode, C.byref(e), C.byref(n)))
    return e.value, n.value


def vqe_expect_pauli_noalloc(s, h, d_out):
    """Grouped energy into device memory d_out (2 doubles: energy, norm);
    d_out is a device pointer (int).  Enqueued, not synchronised."""
    return check("vqe_expect_pauli_noalloc", lib().vqe_expect_pauli_noalloc(s, h, C.c_void_p(d_out)))


def vqe_apply_hamiltonian(psi, lam, h):
    e, n = C.c_double(), C.c_double()
    check("vqe_apply_hamiltonian", lib().vqe_apply_hamiltonian(psi, lam, h, C.byref(e), C.byref(n)))
    return e.value, n.value


def vqe_energy_grad(psi, lam, c, params, h, method=GRAD_ADJOINT, expect_mode=EXPECT_GROUPED, ckpt=(), chunk_passes=0):
    p, pp = _arr(params, np.float64, C.c_double)
    g = np.zeros(len(p), dtype=np.float64)
    arr = (C.c_void_p * max(len(ckpt), 1))(*ckpt)
    opts = vqe_grad_opts(method, expect_mode, len(ckpt), int(chunk_passes), C.cast(arr, C.POINTER(C.c_void_p)))
    e = C.c_double()
    check("vqe_energy_grad", lib().vqe_energy_grad(psi, lam, c, pp, len(p), h, C.byref(opts), C.byref(e),
                                                   g.ctypes.data_as(C.POINTER(C.c_double))))
    return e.value, g


def vqe_slim_hamiltonian(x, z, w, mode, value):
    x, xp = _arr(x, np.uint64, C.c_uint64)
    z, zp = _arr(z, np.uint64, C.c_uint64)
    w, wp = _arr(w, np.float64, C.c_double)
    keep = np.zeros(len(w), dtype=np.uint8)
    nk, dropped = _SZ(), C.c_double()
    check("vqe_slim_hamiltonian", lib().vqe_slim_hamiltonian(
        xp, zp, wp, len(w), mode, float(value), keep.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(nk),
        C.byref(dropped)))
    return keep, nk.value, dropped.value


def vqe_set_specialize(mode):
    """Kernel form of window passes (interpreted / specialised); returns the previous mode."""
    r = lib().vqe_set_specialize(int(mode))
    if r < 0:
        check("vqe_set_specialize", r)
    return r


def vqe_circuit_prepare(c, dtype):
    """Compiles/loads the specialised kernels an evaluation of dtype would use (no-op otherwise)."""
    check("vqe_circuit_prepare", lib().vqe_circuit_prepare(c, dtype))


def vqe_stream_create(cus=None):
    """A stream restricted to the compute units in `cus` (iterable of CU
    indices; None: an ordinary non-blocking stream); returns the hipStream_t as int."""
    out = C.c_void_p()
    if cus is None:
        check("vqe_stream_create", lib().vqe_stream_create(None, 0, C.byref(out)))
    else:
        cus = sorted(set(int(c) for c in cus))
        words = (max(cus) // 32 + 1) if cus else 1
        m = (C.c_uint32 * words)()
        for c in cus:
            m[c // 32] |= 1 << (c % 32)
        check("vqe_stream_create", lib().vqe_stream_create(m, words, C.byref(out)))
    return out.value


def vqe_stream_destroy(stream):
    check("vqe_stream_destroy", lib().vqe_stream_destroy(C.c_void_p(stream)))


def vqe_profile_enable(on=True):
    check("vqe_profile_enable", lib().vqe_profile_enable(1 if on else 0))


def vqe_profile_reset():
    check("vqe_profile_reset", lib().vqe_profile_reset())


def vqe_profile_read(kind):
    n, ms, b = C.c_uint64(), C.c_double(), C.c_double()
    check("vqe_profile_read", lib().vqe_profile_read(kind, C.byref(n), C.byref(ms), C.byref(b)))
    return n.value, ms.value, b.value


def vqe_batch_create(dtype, hip_stream=None):
    out = _P()
    check("vqe_batch_create", lib().vqe_batch_create(dtype, hip_stream, C.byref(out)))
    return out.value


def vqe_batch_free(b):
    check("vqe_batch_free", lib().vqe_batch_free(b))


def vqe_batch_energy_grad(b, items):
    """items: list of (circuit_handle, hamiltonian_handle, params).  Returns [(E, grad)]."""
    n = len(items)
    arr = (vqe_batch_item * max(n, 1))()
    keep = []
    outs = []
    for i, (c, h, p) in enumerate(items):
        p = np.ascontiguousarray(p, dtype=np.float64)
        e = np.zeros(1)
        g = np.zeros(len(p))
        keep += [p, e, g]
        arr[i] = vqe_batch_item(c, h, p.ctypes.data_as(C.POINTER(C.c_double)), len(p),
                                e.ctypes.data_as(C.POINTER(C.c_double)), g.ctypes.data_as(C.POINTER(C.c_double)))
        outs.append((e, g))
    check("vqe_batch_energy_grad", lib().vqe_batch_energy_grad(b, n, arr))
    return [(float(e[0]), g) for e, g in outs]
