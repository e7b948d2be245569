"""Specialised window kernels (straight-line code generated per pass and
compiled at run time) against the CPU FP64 oracle and against the
interpreted kernels, through the C ABI.

Same tolerances as the interpreted path (test_gpu_parity); the two kernel
forms differ only in the rounding of fused multiply-adds, so their results
agree to complex128 1e-12 / complex64 1e-5 (energies, relative) and
complex128 1e-11 / complex64 1e-4 (gradients, relative to max(|g|_inf, 1)).
"""
import numpy as np
import pytest

import synth
from oracle import grad as ogr, hamiltonian as oham, statevector as osv
from paper_2402_11878_amd import _lib, ansatz, hamiltonians as lham

from gpu_util import Dev, oracle_gates, rel_err, say, tol_energy
from test_host import random_circuit

pytestmark = pytest.mark.gpu

DT = {"c64": _lib.VQE_C64, "c128": _lib.VQE_C128}
AMP_TOL = {_lib.VQE_C64: 2e-5, _lib.VQE_C128: 1e-12}
GRAD_TOL = {_lib.VQE_C64: 1e-4, _lib.VQE_C128: 1e-9}
FORM_E_TOL = {_lib.VQE_C64: 1e-5, _lib.VQE_C128: 1e-12}
FORM_G_TOL = {_lib.VQE_C64: 1e-4, _lib.VQE_C128: 1e-11}


@pytest.fixture(autouse=True)
def _restore_mode():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    prev = _lib.vqe_set_specialize(_lib.SPECIALIZE_AUTO)
    yield
    _lib.vqe_set_specialize(prev)


def _random_pauli_sum(n, n_terms, seed):
    rng = np.random.default_rng(seed)
    H = {}
    for _ in range(n_terms):
        s = tuple(rng.choice(list("IXYZ"), size=n, p=[0.4, 0.2, 0.2, 0.2]))
        H[s] = H.get(s, 0.0) + float(rng.normal())
    H[tuple("I" * n)] = 0.3
    return H


def test_mode_switch_and_errors():
    assert _lib.vqe_set_specialize(_lib.SPECIALIZE_ALWAYS) == _lib.SPECIALIZE_AUTO
    assert _lib.vqe_set_specialize(_lib.SPECIALIZE_NEVER) == _lib.SPECIALIZE_ALWAYS
    with pytest.raises(_lib.VqeError):
        _lib.vqe_set_specialize(7)
    assert _lib.vqe_set_specialize(_lib.SPECIALIZE_AUTO) == _lib.SPECIALIZE_NEVER


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n,kind,seed", [(3, "random", 31), (6, "random", 32), (9, "layered", 33),
                                         (11, "random", 34), (13, "layered", 35), (14, "random", 36)])
def test_state_specialised(n, kind, seed, dt):
    """Forward passes (every window size 1..5, every lane-split mode that the
    dtype uses, LDS-staged passes stay interpreted) match the oracle state."""
    dtype = DT[dt]
    if kind == "layered":
        arr, P = ansatz.layered(n, 3), 6 * n
    else:
        arr, P = random_circuit(n, 60 + 5 * n, seed)
    th = synth.theta(seed, max(P, 1))[:P]
    say(f"case specialised state n={n} {kind} seed={seed} {dt}")
    ref = osv.run(n, oracle_gates(arr), th)
    _lib.vqe_set_specialize(_lib.SPECIALIZE_ALWAYS)
    c = _lib.vqe_circuit_create(n, arr)
    s = Dev(n, dtype)
    try:
        _lib.vqe_state_set_basis(s.h, 0)
        _lib.vqe_apply_circuit(s.h, c, th)
        got = s.read()
        assert np.max(np.abs(got - ref)) <= AMP_TOL[dtype]
    finally:
        s.free()
        _lib.vqe_circuit_free(c)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n,kind,seed", [(5, "random", 41), (8, "random", 42), (10, "layered", 43),
                                         (12, "random", 44), (14, "layered", 45)])
def test_adjoint_specialised(n, kind, seed, dt):
    """Energy and adjoint gradient with specialised forward and reverse passes
    against the oracle adjoint, and against the interpreted kernels."""
    dtype = DT[dt]
    if kind == "layered":
        arr, P = ansatz.layered(n, 4), 8 * n
    else:
        arr, P = random_circuit(n, 80, seed)
    th = synth.theta(seed, P)
    og = oracle_gates(arr)
    H = _random_pauli_sum(n, 30, seed)
    say(f"case specialised adjoint n={n} {kind} seed={seed} {dt}")
    E_ref, g_ref = ogr.adjoint(n, og, th, H)
    x, z, w = oham.to_masks(H)
    h = _lib.vqe_hamiltonian_create(n, x, z, w)
    c = _lib.vqe_circuit_create(n, arr)
    s, l = Dev(n, dtype), Dev(n, dtype)
    try:
        _lib.vqe_set_specialize(_lib.SPECIALIZE_ALWAYS)
        E, g = _lib.vqe_energy_grad(s.h, l.h, c, th, h)
        gscale = max(np.max(np.abs(g_ref)), 1.0)
        assert rel_err(E, E_ref) <= tol_energy(dtype)
        assert np.max(np.abs(g - g_ref)) / gscale <= GRAD_TOL[dtype]
        # same call again: identical bits (cached kernels, fixed reduction order)
        E2, g2 = _lib.vqe_energy_grad(s.h, l.h, c, th, h)
        assert E2 == E and np.array_equal(g2, g)
        _lib.vqe_set_specialize(_lib.SPECIALIZE_NEVER)
        Ei, gi = _lib.vqe_energy_grad(s.h, l.h, c, th, h)
        assert rel_err(E, Ei) <= FORM_E_TOL[dtype]
        assert np.max(np.abs(g - gi)) / max(np.max(np.abs(gi)), 1.0) <= FORM_G_TOL[dtype]
    finally:
        s.free(), l.free()
        _lib.vqe_circuit_free(c)
        _lib.vqe_hamiltonian_free(h)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_auto_mode_at_20_qubits(dt):
    """At the auto threshold (20 qubits) the default mode runs specialised
    kernels; energy and gradient match the interpreted kernels."""
    dtype = DT[dt]
    n = _lib.SPECIALIZE_AUTO_MIN_QUBITS
    arr = ansatz.layered(n, 2)
    P = 4 * n
    th = synth.theta(7, P)
    x, z, w = lham.hubbard(n // 2, synth.chain_bonds(n // 2), 1.0, 4.0)
    h = _lib.vqe_hamiltonian_create(n, x, z, w)
    c = _lib.vqe_circuit_create(n, arr)
    s, l = Dev(n, dtype), Dev(n, dtype)
    say(f"case specialised auto n={n} {dt}")
    try:
        E, g = _lib.vqe_energy_grad(s.h, l.h, c, th, h)
        _lib.vqe_set_specialize(_lib.SPECIALIZE_NEVER)
        Ei, gi = _lib.vqe_energy_grad(s.h, l.h, c, th, h)
        assert rel_err(E, Ei) <= FORM_E_TOL[dtype]
        assert np.max(np.abs(g - gi)) / max(np.max(np.abs(gi)), 1.0) <= FORM_G_TOL[dtype]
    finally:
        s.free(), l.free()
        _lib.vqe_circuit_free(c)
        _lib.vqe_hamiltonian_free(h)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_prepare_then_evaluate(dt):
    """Kernels compiled ahead by vqe_circuit_prepare serve the evaluation:
    same energy and gradient bits as an evaluation that compiles on first use."""
    dtype = DT[dt]
    n = 11
    arr, P = random_circuit(n, 90, 77)
    th = synth.theta(77, P)
    H = _random_pauli_sum(n, 20, 77)
    x, z, w = oham.to_masks(H)
    h = _lib.vqe_hamiltonian_create(n, x, z, w)
    _lib.vqe_set_specialize(_lib.SPECIALIZE_ALWAYS)
    c1 = _lib.vqe_circuit_create(n, arr)
    c2 = _lib.vqe_circuit_create(n, arr)
    s, l = Dev(n, dtype), Dev(n, dtype)
    say(f"case prepare n={n} {dt}")
    try:
        _lib.vqe_circuit_prepare(c1, dtype)
        _lib.vqe_circuit_prepare(c1, dtype)  # second call: already loaded
        E1, g1 = _lib.vqe_energy_grad(s.h, l.h, c1, th, h)
        E2, g2 = _lib.vqe_energy_grad(s.h, l.h, c2, th, h)
        assert E1 == E2 and np.array_equal(g1, g2)
    finally:
        s.free(), l.free()
        _lib.vqe_circuit_free(c1)
        _lib.vqe_circuit_free(c2)
        _lib.vqe_hamiltonian_free(h)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_sheared_rotations_at_any_angle_with_checkpoints(dt):
    """The specialised reverse kernels un-apply RY and RZ as three shears
    after a half turn for |angle| > pi, which flips the sign of psi and lam
    together; after a checkpoint restore only lam carries the flips and the
    host corrects the gradient sign.  Excitation gates at the same angles
    (matrix form) share the passes.  Angles in (-4 pi, 4 pi) (most rotations
    take the half turn) and multiples of pi / 2 (the range edges), with 0, 1
    and 3 checkpoints: every gradient against the oracle, and the checkpoint
    counts against each other."""
    dtype = DT[dt]
    n = 12
    arr, P = ansatz.layered(n, 4), 8 * n
    rnd, P2 = random_circuit(n, 40, 91)
    rnd["param_index"][rnd["param_index"] >= 0] += P
    exc, P3 = ansatz.excitations(n, 4)  # excitations keep the matrix form: no half turns there
    exc["param_index"][exc["param_index"] >= 0] += P + P2
    arr = np.concatenate([arr, rnd, exc])
    P += P2 + P3
    rng = np.random.default_rng(92)
    th = rng.uniform(-4 * np.pi, 4 * np.pi, P)
    th[::5] = (np.pi / 2) * rng.integers(-8, 9, size=len(th[::5]))
    H = _random_pauli_sum(n, 30, 93)
    x, z, w = oham.to_masks(H)
    E_ref, g_ref = ogr.adjoint(n, oracle_gates(arr), th, H)
    gscale = max(np.max(np.abs(g_ref)), 1.0)
    h = _lib.vqe_hamiltonian_create(n, x, z, w)
    c = _lib.vqe_circuit_create(n, arr)
    s, l = Dev(n, dtype), Dev(n, dtype)
    cks = [Dev(n, dtype) for _ in range(3)]
    say(f"case sheared rotations n={n} {dt}")
    try:
        _lib.vqe_set_specialize(_lib.SPECIALIZE_ALWAYS)
        res = []
        for k in (0, 1, 3):
            E, g = _lib.vqe_energy_grad(s.h, l.h, c, th, h, ckpt=[d.h for d in cks[:k]])
            assert rel_err(E, E_ref) <= tol_energy(dtype), (k, E, E_ref)
            assert np.max(np.abs(g - g_ref)) / gscale <= GRAD_TOL[dtype], (k, np.max(np.abs(g - g_ref)) / gscale)
            res.append(g)
        for g in res[1:]:
            assert np.max(np.abs(g - res[0])) / gscale <= (1e-12 if dtype == _lib.VQE_C128 else 2e-5)
    finally:
        for d in [s, l] + cks:
            d.free()
        _lib.vqe_circuit_free(c)
        _lib.vqe_hamiltonian_free(h)
