"""GPU checks at full scale (28-32 qubits), where the oracle cannot hold the
state.  Each value is pinned by something the oracle computes without a
state vector:
  * one ansatz layer: Clifford conjugation of each Pauli term through the CNOT
    ladder and the per-qubit Bloch vectors (closed form, any n);
  * angles that are multiples of pi/2: the circuit is Clifford and a
    stabiliser tableau gives every <P> exactly; parameter shifts of pi/2 stay
    Clifford, so the exact gradient follows from two tableau runs;
  * theta = 0: E = sum of the x = 0 weights;
  * complex64 against complex128 on generic angles (1e-5 energy, 1e-4 gradient).
These sizes also exercise launches in which every thread (direct windows) or
every wave (LDS-staged windows) handles several cosets.
"""
import math

import numpy as np
import pytest

import synth
from oracle import closed_forms as cf, hamiltonian as oham
from paper_2402_11878_amd import _lib, ansatz, hamiltonians as lham

from gpu_util import Dev, oracle_gates, rel_err, say

pytestmark = pytest.mark.gpu


def _lattice_ham(rows, cols, U=4.0):
    bonds = synth.snake_bonds(rows, cols, False)
    lat = synth.Lattice(rows * cols, tuple(bonds), 1.0, U)
    return lham.from_lattice(lat)


@pytest.fixture(scope="module")
def ham30():
    x, z, w = _lattice_ham(3, 5)
    return x, z, w


def _energy_from(vals, w):
    return math.fsum(float(wi) * v for wi, v in zip(w, vals))


def test_one_layer_closed_form_30q(ham30):
    n = 30
    x, z, w = ham30
    th = synth.theta(31, 2 * n)
    want = _energy_from([cf.one_layer_expectation(n, th[:n], th[n:], int(a), int(b)) for a, b in zip(x, z)], w)
    h = _lib.vqe_hamiltonian_create(n, x, z, w)
    c = _lib.vqe_circuit_create(n, ansatz.layered(n, 1))
    for dt, tol in ((_lib.VQE_C128, 1e-10), (_lib.VQE_C64, 1e-5)):
        say(f"case one-layer 30q dtype={dt}")
        s = Dev(n, dt)
        try:
            _lib.vqe_state_set_basis(s.h, 0)
            _lib.vqe_apply_circuit(s.h, c, th)
            for mode in (_lib.EXPECT_GROUPED, _lib.EXPECT_PER_TERM):
                E, nrm = _lib.vqe_expect_pauli(s.h, h, mode)
                assert rel_err(E, want) <= tol, (mode, E, want)
        finally:
            s.free()
    _lib.vqe_circuit_free(c)
    _lib.vqe_hamiltonian_free(h)


def test_clifford_energy_and_gradient_30q(ham30):
    n, L = 30, 3
    x, z, w = ham30
    rng = np.random.default_rng(3)
    th = rng.choice([0.0, math.pi / 2, -math.pi / 2, math.pi], size=2 * n * L)
    arr = ansatz.layered(n, L)
    og = oracle_gates(arr)
    terms = list(zip(x.tolist(), z.tolist()))
    E_ref = _energy_from(cf.clifford_expectations(n, og, th, terms), w)
    ks = [0, 5, 2 * n + 7, 2 * n * L - 1, n + 3]
    g_ref = {}
    for k in ks:
        tp, tm = th.copy(), th.copy()
        tp[k] += math.pi / 2
        tm[k] -= math.pi / 2
        g_ref[k] = 0.5 * (_energy_from(cf.clifford_expectations(n, og, tp, terms), w)
                          - _energy_from(cf.clifford_expectations(n, og, tm, terms), w))
    h = _lib.vqe_hamiltonian_create(n, x, z, w)
    c = _lib.vqe_circuit_create(n, arr)
    for dt, te, tg in ((_lib.VQE_C128, 1e-10, 1e-9), (_lib.VQE_C64, 1e-5, 1e-4)):
        say(f"case clifford 30q dtype={dt}")
        s, l = Dev(n, dt), Dev(n, dt)
        try:
            E, g = _lib.vqe_energy_grad(s.h, l.h, c, th, h)
            assert rel_err(E, E_ref) <= te, (E, E_ref)
            gs = max(max(abs(v) for v in g_ref.values()), 1.0)
            for k in ks:
                assert abs(g[k] - g_ref[k]) / gs <= tg, (k, g[k], g_ref[k])
        finally:
            s.free(), l.free()
    _lib.vqe_circuit_free(c)
    _lib.vqe_hamiltonian_free(h)


def test_c64_vs_c128_generic_30q(ham30):
    n, L = 30, 2
    x, z, w = ham30
    th = synth.theta(32, 2 * n * L)
    h = _lib.vqe_hamiltonian_create(n, x, z, w)
    c = _lib.vqe_circuit_create(n, ansatz.layered(n, L))
    out = {}
    for dt in (_lib.VQE_C128, _lib.VQE_C64):
        say(f"case generic 30q dtype={dt}")
        s, l = Dev(n, dt), Dev(n, dt)
        ck = Dev(n, dt)
        try:
            out[dt] = _lib.vqe_energy_grad(s.h, l.h, c, th, h, ckpt=[ck.h])
            E_grp, _ = _lib.vqe_expect_pauli(s.h, h, _lib.EXPECT_GROUPED)
            # psi was un-applied back to |0...0>: E = sum of the x = 0 weights
            assert rel_err(E_grp, float(w[x == 0].sum())) <= (1e-9 if dt == _lib.VQE_C128 else 1e-5)
        finally:
            s.free(), l.free(), ck.free()
    E128, g128 = out[_lib.VQE_C128]
    E64, g64 = out[_lib.VQE_C64]
    assert rel_err(E64, E128) <= 1e-5
    assert np.max(np.abs(g64 - g128)) / max(np.max(np.abs(g128)), 1.0) <= 1e-4
    _lib.vqe_circuit_free(c)
    _lib.vqe_hamiltonian_free(h)


def test_bench_configuration_32q_clifford():
    """The benchmark step at its full size and in its launch configuration:
    32-qubit 4x4 Hubbard (145 terms, lam = H psi by window passes), 8-layer
    ansatz (23 specialised passes per sweep), complex128 with one checkpoint
    and complex64 with four, on Clifford angles (multiples of pi/2, about 2 %
    of them odd).  The stabiliser tableau gives the exact energy and, from two
    runs per parameter at +-pi/2 (still Clifford), the exact gradient of all
    512 parameters."""
    wl = synth.WORKLOADS["hubbard4x4"]
    n, L = wl.n_qubits, wl.layers
    x, z, w = lham.from_lattice(wl.lattice)
    arr = ansatz.layered(n, L)
    og = oracle_gates(arr)
    terms = list(zip(x.tolist(), z.tolist()))
    P = 2 * n * L
    rng = np.random.default_rng(5)
    th = np.where(rng.random(P) < 0.02, rng.choice([math.pi / 2, -math.pi / 2], size=P),
                  rng.choice([0.0, math.pi], size=P))

    def energy(t):
        return _energy_from(cf.clifford_expectations(n, og, t, terms), w)

    E_ref = energy(th)
    g_ref = np.zeros(P)
    for k in range(P):
        tp, tm = th.copy(), th.copy()
        tp[k] += math.pi / 2
        tm[k] -= math.pi / 2
        g_ref[k] = 0.5 * (energy(tp) - energy(tm))
    assert np.count_nonzero(g_ref) >= 3 and E_ref != float(w[(x == 0) & (z == 0)].sum())
    h = _lib.vqe_hamiltonian_create(n, x, z, w)
    c = _lib.vqe_circuit_create(n, arr)
    try:
        assert len(_lib.vqe_hamiltonian_plan(h)) == 4
        for dt, n_ck, te, tg in ((_lib.VQE_C128, 1, 1e-10, 1e-9), (_lib.VQE_C64, 4, 1e-5, 1e-4)):
            say(f"case bench configuration 32q dtype={dt} checkpoints={n_ck}")
            bufs = [Dev(n, dt) for _ in range(2 + n_ck)]
            try:
                E, g = _lib.vqe_energy_grad(bufs[0].h, bufs[1].h, c, th, h, ckpt=[b.h for b in bufs[2:]])
                assert rel_err(E, E_ref) <= te, (E, E_ref)
                gs = max(np.max(np.abs(g_ref)), 1.0)
                assert np.max(np.abs(g - g_ref)) / gs <= tg, np.max(np.abs(g - g_ref))
            finally:
                for b in bufs:
                    b.free()
    finally:
        _lib.vqe_circuit_free(c)
        _lib.vqe_hamiltonian_free(h)
