"""Dense window by MFMA (vqe_apply_dense) against the oracle's dense window
(the definition psi'[b] = sum_p U[pat(b), p] psi[rest(b) | off(p)]), element
by element; at 30 qubits on a basis state, whose exact result is one column of
U on one coset and zero elsewhere."""
import numpy as np
import pytest

from oracle import statevector as osv
from paper_2402_11878_amd import _lib

from gpu_util import Dev, say

pytestmark = pytest.mark.gpu

DT = {"c64": _lib.VQE_C64, "c128": _lib.VQE_C128}
TOL = {"c64": 1e-5, "c128": 1e-13}  # max |error| / max |psi|: 64-term FP32 / FP64 sums


def _unitary(k, rng):
    a = rng.normal(size=(1 << k, 1 << k)) + 1j * rng.normal(size=(1 << k, 1 << k))
    q, r = np.linalg.qr(a)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _state(n, rng):
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n,qubits", [(9, [4, 5, 6, 7, 8]), (10, [9, 4, 6, 5, 8]), (11, [4, 10, 7, 5, 6]),
                                      (12, [11, 4, 9, 6, 7]), (14, [13, 5, 10, 4, 8])])
def test_dense_matches_oracle(n, qubits, dt):
    """n = 9, 10, 11: one block with 1, 2 or 4 of its 4 waves holding a tile."""
    dtype = DT[dt]
    rng = np.random.default_rng(n)
    U, psi = _unitary(5, rng), _state(n, rng)
    say(f"case dense n={n} qubits={qubits} {dt}")
    want = osv.apply_dense(psi.copy(), n, qubits, U)
    s = Dev(n, dtype)
    try:
        _lib.vqe_state_write(s.h, 0, psi, dtype)
        _lib.vqe_apply_dense(s.h, qubits, U)
        got = s.read()
        assert np.max(np.abs(got - want)) <= TOL[dt] * np.max(np.abs(want))
        _lib.vqe_apply_dense(s.h, qubits, U.conj().T)  # and back
        assert np.max(np.abs(s.read() - psi)) <= 2 * TOL[dt] * np.max(np.abs(psi))
    finally:
        s.free()


def test_dense_argument_errors():
    n = 10
    s = Dev(n, _lib.VQE_C128)
    U = np.eye(32)
    try:
        for qubits in ([4, 5, 6, 7], [3, 5, 6, 7, 8], [4, 5, 6, 7, 7], [4, 5, 6, 7, 10]):
            with pytest.raises((_lib.VqeError, ValueError)):
                _lib.vqe_apply_dense(s.h, qubits, U if len(qubits) == 5 else np.eye(16))
    finally:
        s.free()


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_dense_basis_state_30_qubits(dt):
    """psi = |b>: afterwards the coset of b holds column pat(b) of U, every
    other amplitude is zero (sampled), for two windows in a row."""
    n, dtype = 30, DT[dt]
    rng = np.random.default_rng(30)
    b = int(rng.integers(0, 1 << n))
    s = Dev(n, dtype)
    try:
        for qubits in ([29, 4, 17, 23, 8], [5, 6, 7, 28, 12]):
            say(f"case dense basis n={n} qubits={qubits} {dt}")
            _lib.vqe_state_set_basis(s.h, b)
            U = _unitary(5, rng)
            _lib.vqe_apply_dense(s.h, qubits, U)
            pat = sum(((b >> q) & 1) << i for i, q in enumerate(qubits))
            rest = b
            for q in qubits:
                rest &= ~(1 << q)
            for p in range(32):
                idx = rest | sum(((p >> i) & 1) << q for i, q in enumerate(qubits))
                v = _lib.vqe_state_read(s.h, idx, 1, dtype)[0]
                assert abs(v - U[p, pat]) <= 4 * TOL[dt]
            for idx in rng.integers(0, 1 << n, 64).tolist():
                r = idx
                for q in qubits:
                    r &= ~(1 << q)
                if r != rest:
                    assert _lib.vqe_state_read(s.h, idx, 1, dtype)[0] == 0
    finally:
        s.free()
