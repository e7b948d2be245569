"""Batched small-state kernel (whole state in LDS, one workgroup per item)
against the oracle, and bitwise independence of an item from its batch."""
import numpy as np
import pytest

import synth
from oracle import grad as ogr, hamiltonian as oham
from paper_2402_11878_amd import _lib, ansatz, hamiltonians as lham

from gpu_util import oracle_gates, rel_err, say
from test_host import random_circuit

pytestmark = pytest.mark.gpu


def _problem(kind, n, seed):
    if kind == "chain":
        lat = synth.Lattice(n // 2, tuple(synth.chain_bonds(n // 2)), 1.0, 4.0)
        x, z, w = lham.from_lattice(lat)
        arr, P = ansatz.layered(n, 3), 6 * n
    elif kind == "molecule":
        h, g = synth.molecule_integrals(n // 2, seed)
        x, z, w = lham.molecule(h, g)
        arr, P = ansatz.layered(n, 2), 4 * n
    else:
        arr, P = random_circuit(n, 50, seed)
        lat = synth.Lattice(n // 2, tuple(synth.chain_bonds(n // 2)), 1.0, 2.0)
        x, z, w = lham.from_lattice(lat)
    th = synth.theta(seed, P)
    return arr, x, z, w, th


@pytest.fixture(scope="module")
def handles():
    import torch
    assert torch.cuda.is_available()
    probs = [("chain", 4, 1), ("molecule", 6, 2), ("random", 8, 3), ("chain", 12, 4), ("molecule", 8, 5),
             ("random", 5, 6), ("chain", 2, 7)]
    out = []
    for kind, n, seed in probs:
        arr, x, z, w, th = _problem(kind, n, seed)
        c = _lib.vqe_circuit_create(n, arr)
        h = _lib.vqe_hamiltonian_create(n, x, z, w)
        E_ref, g_ref = ogr.adjoint(n, oracle_gates(arr), th, oham.from_masks(n, x, z, w))
        out.append(dict(kind=kind, n=n, c=c, h=h, th=th, E=E_ref, g=g_ref))
    yield out
    for d in out:
        _lib.vqe_circuit_free(d["c"])
        _lib.vqe_hamiltonian_free(d["h"])


@pytest.mark.parametrize("dt", [_lib.VQE_C128, _lib.VQE_C64])
def test_batch_matches_oracle_and_is_order_independent(handles, dt):
    import torch
    say(f"case batch dtype={dt}")
    b = _lib.vqe_batch_create(dt, torch.cuda.current_stream().cuda_stream)
    try:
        items = [(d["c"], d["h"], d["th"]) for d in handles]
        mixed = _lib.vqe_batch_energy_grad(b, items)
        te, tg = (1e-10, 1e-9) if dt == _lib.VQE_C128 else (1e-5, 1e-4)
        for d, (E, g) in zip(handles, mixed):
            assert rel_err(E, d["E"]) <= te, (d["kind"], d["n"], E, d["E"])
            assert np.max(np.abs(g - d["g"])) / max(np.max(np.abs(d["g"])), 1.0) <= tg
        # alone, reversed and duplicated mixes: identical bits
        for i, it in enumerate(items):
            (E1, g1), = _lib.vqe_batch_energy_grad(b, [it])
            assert E1 == mixed[i][0] and np.array_equal(g1, mixed[i][1])
        rev = _lib.vqe_batch_energy_grad(b, items[::-1] + items[:3])
        for i in range(len(items)):
            E2, g2 = rev[len(items) - 1 - i]
            assert E2 == mixed[i][0] and np.array_equal(g2, mixed[i][1])
    finally:
        _lib.vqe_batch_free(b)


def test_batch_rejects_states_above_the_mid_size_limit():
    import torch
    n = _lib.BATCH_MAX_QUBITS_MID + 1
    c = _lib.vqe_circuit_create(n, ansatz.layered(n, 1))
    h = _lib.vqe_hamiltonian_create(n, np.array([0], np.uint64), np.array([1], np.uint64), np.array([1.0]))
    b = _lib.vqe_batch_create(_lib.VQE_C64, torch.cuda.current_stream().cuda_stream)
    try:
        with pytest.raises(_lib.VqeError):
            _lib.vqe_batch_energy_grad(b, [(c, h, np.zeros(2 * n))])
    finally:
        _lib.vqe_batch_free(b)
        _lib.vqe_circuit_free(c)
        _lib.vqe_hamiltonian_free(h)
