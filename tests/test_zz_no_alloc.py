"""vqe_expect_pauli_noalloc: the grouped energy (eq. 7) with no allocation,
through the C ABI, against vqe_expect_pauli on the same state (bitwise: same
kernels, same block counts, same reduction order) and against the CPU oracle
(complex128 within 1e-10, complex64 within 1e-5 relative).  Two calls in a
row, the second on a smaller state, then the first again: the shared scratch
array keeps the last call's values, and nothing from an earlier call may
leak into a later result."""
import numpy as np
import pytest

import synth
from oracle import expect as oex, hamiltonian as oham, statevector as osv
from paper_2402_11878_amd import _lib, ansatz

from gpu_util import Dev, oracle_gates, rel_err, say, tol_energy

pytestmark = pytest.mark.gpu

DT = {"c64": _lib.VQE_C64, "c128": _lib.VQE_C128}


def _case(n, sites, bonds, U, seed):
    H = oham.hubbard(sites, bonds, 1.0, U)
    x, z, w = oham.to_masks(H)
    arr = ansatz.layered(n, 2)
    th = synth.theta(seed, 4 * n)
    psi_ref = osv.run(n, oracle_gates(arr), th)
    E_ref, _ = oex.energy(psi_ref, n, H)
    return (x, z, w), arr, th, E_ref


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_noalloc_matches_expect_pauli(dt):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    dtype = DT[dt]
    cases = [
        # 16 qubits, 2x4 ladder: the energy-only window passes
        (16, _case(16, 8, synth.snake_bonds(2, 4, False), 8.0, 21)),
        # 10 qubits, 5-site chain: below the window size, the tile sweep
        (10, _case(10, 5, synth.chain_bonds(5), 4.0, 22)),
    ]
    d_out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    handles = []
    try:
        for n, ((x, z, w), arr, th, E_ref) in cases:
            h = _lib.vqe_hamiltonian_create(n, x, z, w)
            c = _lib.vqe_circuit_create(n, arr)
            s = Dev(n, dtype)
            handles.append((n, h, c, s, th, E_ref))
            _lib.vqe_state_set_basis(s.h, 0)
            _lib.vqe_apply_circuit(s.h, c, th)
        for rep in range(2):
            for n, h, c, s, th, E_ref in handles:
                say(f"case noalloc {dt} n={n} call {rep}")
                E, nrm = _lib.vqe_expect_pauli(s.h, h, _lib.EXPECT_GROUPED)   # uploads h on the first call
                _lib.vqe_expect_pauli_noalloc(s.h, h, d_out.data_ptr())
                torch.cuda.synchronize()
                got = d_out.cpu().numpy()
                assert got[0] == E and got[1] == nrm, (got, E, nrm)
                assert rel_err(got[0], E_ref) <= tol_energy(dtype), (got[0], E_ref)
                assert abs(got[1] - 1.0) <= (1e-12 if dtype == _lib.VQE_C128 else 1e-5)
                d_out.fill_(float("nan"))
                torch.cuda.synchronize()
    finally:
        for n, h, c, s, th, E_ref in handles:
            s.free()
            _lib.vqe_circuit_free(c)
            _lib.vqe_hamiltonian_free(h)


def test_noalloc_rejects_host_memory_and_missing_tables():
    """Host-side checks only (nothing is launched): d_out must be device
    memory, and the Hamiltonian's tables must already be on the device."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    n = 10
    (x, z, w), arr, th, _ = _case(n, 5, synth.chain_bonds(5), 4.0, 23)
    h = _lib.vqe_hamiltonian_create(n, x, z, w)
    s = Dev(n, _lib.VQE_C128)
    d_out = torch.zeros(2, dtype=torch.float64, device="cuda")
    host = np.zeros(2)
    try:
        with pytest.raises(_lib.VqeError) as e:
            _lib.vqe_expect_pauli_noalloc(s.h, h, d_out.data_ptr())
        assert e.value.code == _lib.VQE_ERR_STATE
        _lib.vqe_expect_pauli(s.h, h, _lib.EXPECT_GROUPED)
        with pytest.raises(_lib.VqeError) as e:
            _lib.vqe_expect_pauli_noalloc(s.h, h, host.ctypes.data)
        assert e.value.code == _lib.VQE_ERR_ARG
        _lib.vqe_expect_pauli_noalloc(s.h, h, d_out.data_ptr())
        torch.cuda.synchronize()
        assert float(d_out[1].cpu()) == 1.0
    finally:
        s.free()
        _lib.vqe_hamiltonian_free(h)
