"""Batched mid-size items (above the LDS limit of the small-state kernel, up
to VQE_BATCH_MAX_QUBITS_MID qubits): tile passes over 10-qubit windows with
the states in device memory, one launch per pass index for the whole batch,
against the CPU FP64 oracle; bitwise independence of an item from its batch;
mixed small and mid-size batches; the per-request path as a cross-check at
20 and 24 qubits.

Tolerances as in test_gpu_batch: energies 1e-10 (complex128) / 1e-5
(complex64) relative; gradients 1e-9 / 1e-4 relative to max(|g_ref|_inf, 1).
"""
import numpy as np
import pytest

import synth
from oracle import grad as ogr, hamiltonian as oham
from paper_2402_11878_amd import _lib, ansatz, hamiltonians as lham

from gpu_util import Dev, oracle_gates, rel_err, say
from test_host import random_circuit

pytestmark = pytest.mark.gpu

TOL = {_lib.VQE_C128: (1e-10, 1e-9), _lib.VQE_C64: (1e-5, 1e-4)}


def _problem(kind, n, seed):
    if kind == "chain":
        lat = synth.Lattice(n // 2, tuple(synth.chain_bonds(n // 2)), 1.0, 4.0)
        x, z, w = lham.from_lattice(lat)
        arr, P = ansatz.layered(n, 3), 6 * n
    elif kind == "molecule":
        h, g = synth.molecule_integrals(n // 2, seed)
        x, z, w = lham.molecule(h, g)
        arr, P = ansatz.layered(n, 2), 4 * n
    elif kind == "excitation":
        h, g = synth.molecule_integrals(n // 2, seed)
        x, z, w = lham.molecule(h, g)
        arr, P = ansatz.excitations(n, 4)
        rnd, P2 = random_circuit(n, 30, seed)
        rnd["param_index"][rnd["param_index"] >= 0] += P
        arr, P = np.concatenate([arr, rnd]), P + P2
    else:
        arr, P = random_circuit(n, 80, seed)
        lat = synth.Lattice(n // 2, tuple(synth.chain_bonds(n // 2)), 1.0, 2.0)
        x, z, w = lham.from_lattice(lat)
    return arr, x, z, w, synth.theta(seed, P)


def _grad_err(g, ref):
    return float(np.max(np.abs(g - ref)) / max(float(np.max(np.abs(ref))), 1.0))


@pytest.fixture(scope="module")
def mid_items():
    import torch
    assert torch.cuda.is_available()
    probs = [("chain", 14, 1), ("molecule", 14, 2), ("random", 15, 3), ("excitation", 14, 4), ("chain", 16, 5),
             ("random", 13, 6)]
    out = []
    for kind, n, seed in probs:
        arr, x, z, w, th = _problem(kind, n, seed)
        say(f"case mid oracle kind={kind} n={n} seed={seed}")
        E_ref, g_ref = ogr.adjoint(n, oracle_gates(arr), th, oham.from_masks(n, x, z, w))
        out.append(dict(kind=kind, n=n, c=_lib.vqe_circuit_create(n, arr), h=_lib.vqe_hamiltonian_create(n, x, z, w),
                        th=th, E=E_ref, g=g_ref))
    yield out
    for d in out:
        _lib.vqe_circuit_free(d["c"])
        _lib.vqe_hamiltonian_free(d["h"])


@pytest.mark.parametrize("dt", [_lib.VQE_C128, _lib.VQE_C64])
def test_mid_batch_matches_oracle_and_is_order_independent(mid_items, dt):
    import torch
    say(f"case mid batch dtype={dt}")
    b = _lib.vqe_batch_create(dt, torch.cuda.current_stream().cuda_stream)
    try:
        items = [(d["c"], d["h"], d["th"]) for d in mid_items]
        mixed = _lib.vqe_batch_energy_grad(b, items)
        te, tg = TOL[dt]
        for d, (E, g) in zip(mid_items, mixed):
            assert rel_err(E, d["E"]) <= te, (d["kind"], d["n"], E, d["E"])
            assert _grad_err(g, d["g"]) <= tg, (d["kind"], d["n"], _grad_err(g, d["g"]))
        for i, it in enumerate(items):
            (E1, g1), = _lib.vqe_batch_energy_grad(b, [it])
            assert E1 == mixed[i][0] and np.array_equal(g1, mixed[i][1]), (i, E1, mixed[i][0])
        rev = _lib.vqe_batch_energy_grad(b, items[::-1] + items[:2])
        for i in range(len(items)):
            E2, g2 = rev[len(items) - 1 - i]
            assert E2 == mixed[i][0] and np.array_equal(g2, mixed[i][1])
        E3, g3 = rev[len(items)]
        assert E3 == mixed[0][0] and np.array_equal(g3, mixed[0][1])
    finally:
        _lib.vqe_batch_free(b)


def test_small_and_mid_items_in_one_call(mid_items):
    """Small items (whole state in LDS) and mid-size items in one call give
    the bits each path gives alone."""
    import torch
    dt = _lib.VQE_C64
    arr, x, z, w, th = _problem("chain", 8, 11)
    c = _lib.vqe_circuit_create(8, arr)
    h = _lib.vqe_hamiltonian_create(8, x, z, w)
    b = _lib.vqe_batch_create(dt, torch.cuda.current_stream().cuda_stream)
    try:
        small = (c, h, th)
        mids = [(d["c"], d["h"], d["th"]) for d in mid_items[:3]]
        both = _lib.vqe_batch_energy_grad(b, [mids[0], small, mids[1], mids[2], small])
        (Es, gs), = _lib.vqe_batch_energy_grad(b, [small])
        alone = _lib.vqe_batch_energy_grad(b, mids)
        for k in (1, 4):
            assert both[k][0] == Es and np.array_equal(both[k][1], gs)
        for k, j in ((0, 0), (2, 1), (3, 2)):
            assert both[k][0] == alone[j][0] and np.array_equal(both[k][1], alone[j][1])
    finally:
        _lib.vqe_batch_free(b)
        _lib.vqe_circuit_free(c)
        _lib.vqe_hamiltonian_free(h)


@pytest.mark.parametrize("n,kind", [(18, "chain"), (20, "random"), (24, "chain")])
def test_mid_batch_at_size_against_per_request_path(n, kind):
    """At 18 qubits against the oracle; at 20 and 24 qubits (where the
    oracle's adjoint takes minutes) against the per-request complex128 path,
    itself checked against the oracle elsewhere.  Two items of the same
    problem with different angles in one batch, complex128 and complex64."""
    import torch
    arr, x, z, w, th = _problem(kind, n, 40 + n)
    th2 = synth.theta(80 + n, len(th))
    c = _lib.vqe_circuit_create(n, arr)
    h = _lib.vqe_hamiltonian_create(n, x, z, w)
    refs = []
    try:
        if n <= 18:
            say(f"case mid size oracle n={n}")
            H = oham.from_masks(n, x, z, w)
            refs = [ogr.adjoint(n, oracle_gates(arr), t, H) for t in (th, th2)]
        else:
            say(f"case mid size per-request n={n}")
            psi, lam = Dev(n, _lib.VQE_C128), Dev(n, _lib.VQE_C128)
            try:
                for t in (th, th2):
                    E, g = _lib.vqe_energy_grad(psi.h, lam.h, c, t, h)
                    refs.append((E, np.array(g)))
            finally:
                psi.free()
                lam.free()
        for dt in (_lib.VQE_C128, _lib.VQE_C64):
            say(f"case mid size batch n={n} dtype={dt}")
            b = _lib.vqe_batch_create(dt, torch.cuda.current_stream().cuda_stream)
            try:
                res = _lib.vqe_batch_energy_grad(b, [(c, h, th), (c, h, th2)])
            finally:
                _lib.vqe_batch_free(b)
            te, tg = TOL[dt]
            for (E, g), (E_ref, g_ref) in zip(res, refs):
                assert rel_err(E, E_ref) <= te, (n, dt, E, E_ref)
                assert _grad_err(g, g_ref) <= tg, (n, dt, _grad_err(g, g_ref))
    finally:
        _lib.vqe_circuit_free(c)
        _lib.vqe_hamiltonian_free(h)


def test_mid_batch_limits():
    import torch
    for n, dt in ((25, _lib.VQE_C64), (25, _lib.VQE_C128)):
        c = _lib.vqe_circuit_create(n, ansatz.layered(n, 1))
        h = _lib.vqe_hamiltonian_create(n, np.array([0], np.uint64), np.array([1], np.uint64), np.array([1.0]))
        h2 = _lib.vqe_hamiltonian_create(n - 1, np.array([0], np.uint64), np.array([1], np.uint64), np.array([1.0]))
        b = _lib.vqe_batch_create(dt, torch.cuda.current_stream().cuda_stream)
        try:
            with pytest.raises(_lib.VqeError):
                _lib.vqe_batch_energy_grad(b, [(c, h, np.zeros(2 * n))])
            c2 = _lib.vqe_circuit_create(n - 1, ansatz.layered(n - 1, 1))
            try:
                with pytest.raises(_lib.VqeError):  # Hamiltonian of another size
                    _lib.vqe_batch_energy_grad(b, [(c2, h, np.zeros(2 * (n - 1)))])
                (E, g), = _lib.vqe_batch_energy_grad(b, [(c2, h2, np.zeros(2 * (n - 1)))])
                assert abs(E - 1.0) < 1e-6 and np.all(np.abs(g) < 1e-6)  # <0|Z_0|0> = 1, flat at theta = 0
            finally:
                _lib.vqe_circuit_free(c2)
        finally:
            _lib.vqe_batch_free(b)
            _lib.vqe_circuit_free(c)
            _lib.vqe_hamiltonian_free(h)
            _lib.vqe_hamiltonian_free(h2)


def _pauli_sum_masks(n, n_terms, seed, max_flip, long_x=False):
    """Random Pauli sum as (x, z, w) masks: each term flips (X or Y) at most
    max_flip qubits, with Z on some others, so Y counts are odd and even
    (complex and real folded coefficients); long_x adds X on every qubit,
    which no window holds."""
    rng = np.random.default_rng(seed)
    x, z, w = [], [], []
    for _ in range(n_terms):
        flips = rng.choice(n, size=int(rng.integers(0, max_flip + 1)), replace=False)
        xm = 0
        zm = int(rng.integers(0, 1 << n)) & int(rng.integers(0, 1 << n))
        for q in flips:
            xm |= 1 << int(q)
            if rng.random() < 0.5:
                zm |= 1 << int(q)     # Y on q
            else:
                zm &= ~(1 << int(q))  # X on q
        x.append(xm), z.append(zm), w.append(float(rng.normal()))
    if long_x:
        x.append((1 << n) - 1), z.append(0), w.append(0.7)
    return np.array(x, np.uint64), np.array(z, np.uint64), np.array(w)


@pytest.mark.parametrize("dt", [_lib.VQE_C128, _lib.VQE_C64])
def test_mid_batch_complex_and_uncovered_hamiltonians(dt):
    """lam = H psi of mid-size items in both forms: window passes with
    complex folded coefficients (terms with odd Y counts), and the tile
    kernel for a Hamiltonian with an X mask no window can hold; against the
    oracle, and bitwise the same alone and together."""
    import torch
    n = 14
    arr, P = ansatz.layered(n, 2), 4 * n
    probs = [_pauli_sum_masks(n, 60, 21, 4), _pauli_sum_masks(n, 40, 22, 3, long_x=True)]
    assert any(bin(int(a) & int(b)).count("1") % 2 for a, b in zip(probs[0][0], probs[0][1]))  # odd Y
    items, refs, hs = [], [], []
    c = _lib.vqe_circuit_create(n, arr)
    try:
        for k, (x, z, w) in enumerate(probs):
            h = _lib.vqe_hamiltonian_create(n, x, z, w)
            hs.append(h)
            th = synth.theta(60 + k, P)
            items.append((c, h, th))
            refs.append(ogr.adjoint(n, oracle_gates(arr), th, oham.from_masks(n, x, z, w)))
        say(f"case mid complex/uncovered dtype={dt}")
        b = _lib.vqe_batch_create(dt, torch.cuda.current_stream().cuda_stream)
        try:
            both = _lib.vqe_batch_energy_grad(b, items)
            alone = [_lib.vqe_batch_energy_grad(b, [it])[0] for it in items]
        finally:
            _lib.vqe_batch_free(b)
        te, tg = TOL[dt]
        for (E, g), (E1, g1), (E_ref, g_ref) in zip(both, alone, refs):
            assert E == E1 and np.array_equal(g, g1)
            assert rel_err(E, E_ref) <= te, (dt, E, E_ref)
            assert _grad_err(g, g_ref) <= tg, (dt, _grad_err(g, g_ref))
    finally:
        for h in hs:
            _lib.vqe_hamiltonian_free(h)
        _lib.vqe_circuit_free(c)
