"""Host-side tests of the library (no GPU needed).

* libvqe.so loads and exports every function declared in include/vqe.h;
* the library's bit-mask Jordan-Wigner equals the oracle's string JW
  (masks bit-exact, coefficients within 1e-14);
* vqe_slim_hamiltonian selects exactly the oracle's terms;
* the fused pass plan is a valid reordering of the circuit (checked by running
  both orders in the oracle) and respects the window limits;
* C ABI argument checking.
"""
import math
import os
import re

import numpy as np
import pytest

import synth
from oracle import hamiltonian as oham, slim as oslim, statevector as osv
from paper_2402_11878_amd import _lib, ansatz, hamiltonians as lham

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_header_symbols():
    hdr = open(os.path.join(ROOT, "include", "vqe.h")).read()
    declared = set(re.findall(r"^(?:const char\*|int)\s+(vqe_\w+)\s*\(", hdr, flags=re.M))
    assert len(declared) >= 20
    L = _lib.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(_lib.exported_symbols())


def test_binding_constants_match_header():
    """Every #define VQE_<NAME> <int> of the header that the binding mirrors
    (as <NAME> or VQE_<NAME>) has the same value there."""
    hdr = open(os.path.join(ROOT, "include", "vqe.h")).read()
    defs = dict(re.findall(r"^#define\s+VQE_(\w+)\s+(-?\d+)\b", hdr, flags=re.M))
    checked = 0
    for name, val in defs.items():
        for py in (name, "VQE_" + name):
            if hasattr(_lib, py):
                assert getattr(_lib, py) == int(val), py
                checked += 1
    assert checked >= 15


def _oracle_masks(H):
    return oham.to_masks(H)


@pytest.mark.parametrize("name", ["hubbard1d_6", "hubbard2x7", "hubbard4x4"])
def test_jw_hubbard_matches_oracle(name):
    lat = synth.WORKLOADS[name].lattice
    ox, oz, ow = _oracle_masks(oham.hubbard(lat.n_sites, list(lat.bonds), lat.t, lat.U))
    lx, lz, lw = lham.from_lattice(lat)
    assert np.array_equal(ox, lx) and np.array_equal(oz, lz)
    assert np.max(np.abs(ow - lw)) <= 1e-14


@pytest.mark.parametrize("sites,bonds", [(1, []), (2, [(0, 1)]), (5, synth.snake_bonds(1, 5, True))])
def test_jw_small_lattices_match_oracle(sites, bonds):
    ox, oz, ow = _oracle_masks(oham.hubbard(sites, bonds, 1.0, 3.0))
    lx, lz, lw = lham.hubbard(sites, bonds, 1.0, 3.0)
    assert np.array_equal(ox, lx) and np.array_equal(oz, lz)
    assert np.max(np.abs(ow - lw)) <= 1e-14


@pytest.mark.parametrize("n_orb,seed", [(1, 3), (2, 0), (3, 1), (4, 2)])
def test_jw_molecule_matches_oracle(n_orb, seed):
    h, g = synth.molecule_integrals(n_orb, seed)
    ox, oz, ow = _oracle_masks(oham.molecule(h, g))
    lx, lz, lw = lham.molecule(h, g)
    assert np.array_equal(ox, lx) and np.array_equal(oz, lz)
    assert np.max(np.abs(ow - lw)) <= 1e-14


def test_hamiltonian_tables_group_counts():
    for name, terms, groups in (("hubbard1d_6", 39, 11), ("hubbard2x7", 127, 43), ("hubbard4x4", 145, 49)):
        wl = synth.WORKLOADS[name]
        x, z, w = lham.from_lattice(wl.lattice)
        h = _lib.vqe_hamiltonian_create(wl.n_qubits, x, z, w)
        nt, ng, idw = _lib.vqe_hamiltonian_info(h)
        _lib.vqe_hamiltonian_free(h)
        assert (nt, ng) == (terms, groups)
        assert abs(idw - wl.lattice.n_sites * wl.lattice.U / 4) < 1e-12


def _slim_inputs(seed, ties):
    rng = np.random.default_rng(seed)
    n = 300
    x = rng.integers(0, 1 << 12, size=n).astype(np.uint64)
    z = rng.integers(0, 1 << 12, size=n).astype(np.uint64)
    w = rng.normal(size=n) * 10.0 ** rng.uniform(-7, 0, size=n)
    if ties:
        w = np.round(w * 8) / 8
        w[w == 0] = -0.125
    x[0] = z[0] = 0
    x[5] = z[5] = 0          # a repeated identity entry
    return x, z, w


@pytest.mark.parametrize("seed,ties", [(0, False), (1, True), (2, True), (3, False)])
def test_slim_matches_oracle_bit_exact(seed, ties):
    x, z, w = _slim_inputs(seed, ties)
    ths = [0.0, 1e-6, 1e-4, 1e-3, 0.125, float(abs(w[17])), float(abs(w[42]))]
    for th in ths:
        keep, nk, dropped = _lib.vqe_slim_hamiltonian(x, z, w, _lib.SLIM_THRESHOLD, th)
        ok, od = oslim.threshold(x, z, w, th)
        assert np.array_equal(keep, ok) and nk == int(ok.sum()) and dropped == od
    for pct in (0, 10, 25, 60, 70, 80, 90, 100):
        keep, nk, dropped = _lib.vqe_slim_hamiltonian(x, z, w, _lib.SLIM_REMOVE_PERCENT, pct)
        ok, od = oslim.remove_percent(x, z, w, pct)
        assert np.array_equal(keep, ok) and dropped == od
    for lim in (0.0, 1e-5, 1e-3, 0.5, 3.0, 1e9):
        keep, nk, dropped = _lib.vqe_slim_hamiltonian(x, z, w, _lib.SLIM_BUDGET, lim)
        ok, od = oslim.budget(x, z, w, lim)
        assert np.array_equal(keep, ok) and dropped == od
    for cnt in (0, 1, 7, 150, 297, 298, 299, 1000):
        keep, nk, dropped = _lib.vqe_slim_hamiltonian(x, z, w, _lib.SLIM_KEEP_TOP, cnt)
        ok, od = oslim.keep_top(x, z, w, cnt)
        assert np.array_equal(keep, ok) and nk == int(ok.sum()) and dropped == od


def test_cutoff_search_keeps_floor_of_tenths():
    """Algorithm 1 keeps the top N x ratio terms: with N = 23 non-identity
    terms, k tenths keep floor(23 k / 10) of them (2, 4, 6, 9, 11, 13, 16, 18,
    20, 23), not the ceiling that removing floor(N (10 - k) / 10) would give."""
    from paper_2402_11878_amd import vqe
    rng = np.random.default_rng(4)
    x = np.concatenate([[0], rng.integers(1, 1 << 8, size=23)]).astype(np.uint64)
    z = rng.integers(0, 1 << 8, size=24).astype(np.uint64)
    z[0] = 0                                   # term 0 is the identity
    w = rng.normal(size=24)
    kept = [vqe.kept_terms(x, z, w, k)[1] - 1 for k in range(1, 11)]
    assert kept == [2, 4, 6, 9, 11, 13, 16, 18, 20, 23]
    assert kept != [int(np.ceil(23 * k / 10)) for k in range(1, 11)]


def test_slim_molecule_counts_monotone():
    h, g = synth.molecule_integrals(4, 0)
    x, z, w = lham.molecule(h, g)
    prev = len(w) + 1
    for th in (0.0, 1e-6, 1e-4, 1e-3, 1e-2):
        keep, nk, dropped = _lib.vqe_slim_hamiltonian(x, z, w, _lib.SLIM_THRESHOLD, th)
        assert nk <= prev
        prev = nk


def test_slim_argument_errors():
    x = np.zeros(2, np.uint64)
    w = np.ones(2)
    with pytest.raises(_lib.VqeError):
        _lib.vqe_slim_hamiltonian(x, x, w, 7, 0.1)
    with pytest.raises(_lib.VqeError):
        _lib.vqe_slim_hamiltonian(x, x, w, _lib.SLIM_REMOVE_PERCENT, 12.5)
    with pytest.raises(_lib.VqeError):
        _lib.vqe_slim_hamiltonian(x, x, w, _lib.SLIM_KEEP_TOP, 2.5)
    with pytest.raises(_lib.VqeError):
        _lib.vqe_slim_hamiltonian(x, x, w, _lib.SLIM_THRESHOLD, -1.0)
    with pytest.raises(_lib.VqeError):
        _lib.vqe_slim_hamiltonian(x, x, np.array([1.0, np.nan]), _lib.SLIM_THRESHOLD, 0.1)


def _oracle_gates(arr):
    names = {0: "RY", 1: "RZ", 2: "RX", 3: "H", 4: "X", 5: "CNOT", 6: "CZ"}
    out = []
    for g in arr:
        k = int(g["kind"])
        if k in (7, 8):
            qs = (int(g["q0"]), int(g["q1"])) + ((int(g["q2"]), int(g["q3"])) if k == 8 else ())
            out.append(("SEXC" if k == 7 else "DEXC", qs, -1, int(g["param_index"]), float(g["angle"])))
        else:
            out.append((names[k], int(g["q0"]), int(g["q1"]), int(g["param_index"]), float(g["angle"])))
    return out


def random_circuit(n, n_gates, seed):
    rng = np.random.default_rng(seed)
    gates = []
    p = 0
    for _ in range(n_gates):
        k = int(rng.integers(0, 7))
        q0 = int(rng.integers(0, n))
        q1 = int(rng.integers(0, n - 1)) if n > 1 else 0
        if q1 >= q0:
            q1 += 1
        if k in (5, 6) and n < 2:
            k = 0
        if k in (0, 1, 2):
            if rng.random() < 0.7:
                gates.append((k, q0, 0, p, 0.0))
                p += 1
            else:
                gates.append((k, q0, 0, -1, float(rng.uniform(-3, 3))))
        elif k in (5, 6):
            gates.append((k, q0, q1, -1, 0.0))
        else:
            gates.append((k, q0, 0, -1, 0.0))
    return ansatz.gates_array(gates), p


@pytest.fixture
def specialize_mode():
    """Sets the kernel form for one test (plans differ: windows <= 5 qubits
    interpreted, <= 7 specialised) and restores the default afterwards."""
    modes = []

    def set_mode(m):
        modes.append(_lib.vqe_set_specialize(m))
    yield set_mode
    if modes:
        _lib.vqe_set_specialize(modes[0])


@pytest.mark.parametrize("mode,kmax", [(_lib.SPECIALIZE_NEVER, 5), (_lib.SPECIALIZE_ALWAYS, 7)])
@pytest.mark.parametrize("n,kind,seed", [(8, "layered", 0), (13, "layered", 1), (7, "random", 2), (9, "random", 3),
                                         (1, "random", 4), (2, "random", 5)])
def test_plan_is_valid_reordering(n, kind, seed, mode, kmax, specialize_mode):
    specialize_mode(mode)
    if kind == "layered":
        arr = ansatz.layered(n, 3)
        P = 6 * n
    else:
        arr, P = random_circuit(n, 80, seed)
    c = _lib.vqe_circuit_create(n, arr)
    try:
        og = _oracle_gates(arr)
        th = synth.theta(seed, max(P, 1))
        ref = osv.run(n, og, th)
        for dtype in (_lib.VQE_C64, _lib.VQE_C128):
            order = []
            p = 0
            while True:
                try:
                    qubits, idx = _lib.vqe_circuit_pass(c, dtype, p)
                except _lib.VqeError:
                    break
                assert 1 <= len(qubits) <= min(kmax, n)
                for gi in idx:
                    g = og[gi]
                    assert g[1] in qubits
                    if g[0] in ("CNOT", "CZ"):
                        assert g[2] in qubits
                order += idx
                p += 1
            assert sorted(order) == list(range(len(og)))
            got = osv.run(n, [og[i] for i in order], th)
            assert np.max(np.abs(got - ref)) < 1e-12
    finally:
        _lib.vqe_circuit_free(c)


def test_circuit_prepare_host_paths(specialize_mode):
    """vqe_circuit_prepare: bad dtype is an argument error; with interpreted
    kernels it is a no-op that needs no device; with specialised kernels and
    no device it reports the missing device."""
    c = _lib.vqe_circuit_create(6, ansatz.layered(6, 2))
    try:
        with pytest.raises(_lib.VqeError) as e:
            _lib.vqe_circuit_prepare(c, 7)
        assert e.value.code == _lib.VQE_ERR_ARG
        specialize_mode(_lib.SPECIALIZE_NEVER)
        _lib.vqe_circuit_prepare(c, _lib.VQE_C64)
        if _lib.vqe_device_count() == 0:
            specialize_mode(_lib.SPECIALIZE_ALWAYS)
            with pytest.raises(_lib.VqeError) as e:
                _lib.vqe_circuit_prepare(c, _lib.VQE_C128)
            assert e.value.code == _lib.VQE_ERR_DEVICE
    finally:
        _lib.vqe_circuit_free(c)


def test_plan_pass_counts_beat_layerwise(specialize_mode):
    """Layer-by-layer fusion needs ceil((n-1)/(K-1)) passes per layer for the
    CNOT ladder; the planner pipelines layers.  Interpreted plans (K <= 5)
    and specialised plans (K <= 7) of the layered ansatz, pass counts of the
    planner as built (regression values)."""
    expect = {(20, 8): (25, 15), (28, 16): (74, 43), (32, 8): (41, 23)}
    for (n, L), (n_interp, n_spec) in expect.items():
        c = _lib.vqe_circuit_create(n, ansatz.layered(n, L))
        specialize_mode(_lib.SPECIALIZE_NEVER)
        _, np_i = _lib.vqe_circuit_info(c)
        specialize_mode(_lib.SPECIALIZE_ALWAYS)
        _, np_s = _lib.vqe_circuit_info(c)
        _lib.vqe_circuit_free(c)
        assert np_i <= L * math.ceil((n - 1) / 4) and np_i <= n_interp
        assert np_s <= L * math.ceil((n - 1) / 6) and np_s <= n_spec


def test_abi_argument_errors():
    g = ansatz.layered(4, 1)
    with pytest.raises(_lib.VqeError) as e:
        _lib.vqe_circuit_create(41, g)
    assert e.value.code == _lib.VQE_ERR_ARG
    bad = g.copy()
    bad[0]["q0"] = 9
    with pytest.raises(_lib.VqeError):
        _lib.vqe_circuit_create(4, bad)
    bad = g.copy()
    bad[-1]["param_index"] = 3          # CNOT cannot take a parameter
    with pytest.raises(_lib.VqeError):
        _lib.vqe_circuit_create(4, bad)
    with pytest.raises(_lib.VqeError):
        _lib.vqe_hamiltonian_create(3, np.array([8], np.uint64), np.array([0], np.uint64), np.array([1.0]))
    with pytest.raises(_lib.VqeError):
        _lib.vqe_hamiltonian_create(3, np.array([1], np.uint64), np.array([0], np.uint64), np.array([np.inf]))
    if _lib.vqe_device_count() == 0:
        with pytest.raises(_lib.VqeError) as e:
            _lib.vqe_state_alloc(4, _lib.VQE_C64)
        assert e.value.code == _lib.VQE_ERR_DEVICE
    with pytest.raises(_lib.VqeError):
        _lib.vqe_state_alloc(4, 7)


def test_molecule_10_slimming_matches_golden():
    """Library Jordan-Wigner + slimming of the 20-qubit molecule-shaped
    Hamiltonian against the oracle's stored counts per cutoff threshold
    (tests/golden/molecule_10.json, written from oracle/ only)."""
    import json
    with open(os.path.join(ROOT, "tests", "golden", "molecule_10.json")) as f:
        ref = json.load(f)
    wl = synth.WORKLOADS["molecule_10"]
    h, g = synth.molecule_integrals(wl.n_orb, wl.integral_seed)
    x, z, w = lham.molecule(h, g)
    assert len(w) == ref["n_terms_full"]
    assert abs(w[(x == 0) & (z == 0)].sum() - ref["identity"]) <= 1e-12
    for key, r in ref["thresholds"].items():
        keep, n_kept, dropped = _lib.vqe_slim_hamiltonian(x, z, w, _lib.SLIM_THRESHOLD, float(key))
        k = keep == 1
        assert n_kept == r["n_terms"]
        assert len(set(x[k].tolist())) == r["n_groups"]
        assert abs(dropped - r["dropped_abs_sum"]) <= 1e-12 * max(1.0, r["dropped_abs_sum"])


# ------------------------------------------------------------------ excitation gates (eq. 5)
@pytest.mark.parametrize("n,ne,layers", [(4, 2, 1), (8, 4, 1), (10, 4, 2)])
def test_excitation_builder_matches_oracle(n, ne, layers):
    """The library's S/D ansatz (after the X gates of the Hartree-Fock
    reference) is the oracle's gate list."""
    arr, P = ansatz.excitations(n, ne, layers)
    og = _oracle_gates(arr)
    assert og[:ne] == [("X", q, 0, -1, 0.0) for q in range(ne)]
    ref = osv.excitation_ansatz(n, ne, layers)
    assert [(k, tuple(q), p) for (k, q, _, p, _) in og[ne:]] == [(k, tuple(q), p) for (k, q, _, p, _) in ref]
    assert P == len(ref)


@pytest.mark.parametrize("n,ne,seed", [(6, 2, 0), (8, 4, 1), (9, 3, 2)])
def test_excitation_plan_is_valid_reordering(n, ne, seed, specialize_mode):
    """Specialised plans of circuits mixing excitation gates with the other
    kinds are valid reorderings (windows hold all qubits of every gate); the
    default form plans them specialised at any size, the interpreted form
    reports them unsupported."""
    exc, P = ansatz.excitations(n, ne)
    rnd, P2 = random_circuit(n, 40, seed)
    rnd["param_index"][rnd["param_index"] >= 0] += P
    arr = np.concatenate([exc, rnd])
    og = _oracle_gates(arr)
    th = synth.theta(seed, P + P2)
    ref = osv.run(n, og, th)
    c = _lib.vqe_circuit_create(n, arr)
    try:
        specialize_mode(_lib.SPECIALIZE_AUTO)
        order, p = [], 0
        while True:
            try:
                qubits, idx = _lib.vqe_circuit_pass(c, _lib.VQE_C128, p)
            except _lib.VqeError:
                break
            assert 1 <= len(qubits) <= min(_lib.MAX_WINDOW, n)
            for gi in idx:
                kind, q0, q1, _, _ = og[gi]
                need = q0 if isinstance(q0, tuple) else ((q0, q1) if kind in ("CNOT", "CZ") else (q0,))
                assert set(need) <= set(qubits)
            order += idx
            p += 1
        assert sorted(order) == list(range(len(og)))
        got = osv.run(n, [og[i] for i in order], th)
        assert np.max(np.abs(got - ref)) < 1e-12
        specialize_mode(_lib.SPECIALIZE_NEVER)
        with pytest.raises(_lib.VqeError) as e:
            _lib.vqe_circuit_pass(c, _lib.VQE_C128, 0)
        assert e.value.code == _lib.VQE_ERR_UNSUPPORTED
    finally:
        _lib.vqe_circuit_free(c)


def test_excitation_gate_argument_errors():
    bad = ansatz.gates_array([(_lib.GATE_DEXC, (0, 1, 2, 1), 0, 0.0)])
    with pytest.raises(_lib.VqeError) as e:
        _lib.vqe_circuit_create(4, bad)
    assert e.value.code == _lib.VQE_ERR_ARG
    bad = ansatz.gates_array([(_lib.GATE_SEXC, (0, 4), 0, 0.0)])
    with pytest.raises(_lib.VqeError):
        _lib.vqe_circuit_create(4, bad)
    ok = ansatz.gates_array([(_lib.GATE_SEXC, (3, 0), -1, 0.4), (_lib.GATE_DEXC, (0, 1, 2, 3), 0, 0.0)])
    c = _lib.vqe_circuit_create(4, ok)
    assert _lib.vqe_circuit_info(c)[0] == 1
    _lib.vqe_circuit_free(c)


def test_cutoff_ratio_rule():
    """Algorithm 1 read as: first k in 10, 9, ..., 1 with |E_k - E_10| >=
    delta_E returns (k + 1)/10; none returns 0.1 (energies given per tenth)."""
    from paper_2402_11878_amd.vqe import cutoff_ratio
    E = {10: -1.0, 9: -1.0, 8: -0.9999, 7: -0.999, 6: -0.99, 5: -0.9, 4: -0.5, 3: -0.4, 2: -0.3, 1: -0.2}
    calls = []

    def f(k):
        calls.append(k)
        return E[k]
    assert cutoff_ratio(f, 5e-4) == 0.8          # k = 7 is the first miss
    assert calls == [10, 9, 8, 7]
    assert cutoff_ratio(lambda k: E[k], 1e-5) == 0.9   # k = 8 misses
    assert cutoff_ratio(lambda k: E[k], 10.0) == 0.1   # never
    assert cutoff_ratio(lambda k: E[k], 0.0) == 1.1    # |E_10 - E_10| >= 0 at once


@pytest.mark.parametrize("name,th", [("hubbard4x4", None), ("hubbard2x7", None), ("molecule_10", 1e-3),
                                     ("molecule_10", 0.0)])
def test_hamiltonian_window_plan_valid(name, th):
    """Window form of H psi: windows of HPSI_WINDOW_QUBITS qubits holding qubits
    0..2, every X mask inside some window, chosen only when (3 m - 1) S <
    (D + 2) S."""
    wl = synth.WORKLOADS[name]
    if wl.kind == "molecule":
        h, g = synth.molecule_integrals(wl.n_orb, wl.integral_seed)
        x, z, w = lham.molecule(h, g)
        keep, _, _ = _lib.vqe_slim_hamiltonian(x, z, w, _lib.SLIM_THRESHOLD, th)
        x, z, w = x[keep == 1], z[keep == 1], w[keep == 1]
    else:
        x, z, w = lham.from_lattice(wl.lattice)
    h = _lib.vqe_hamiltonian_create(wl.n_qubits, x, z, w)
    try:
        wins = _lib.vqe_hamiltonian_plan(h)
    finally:
        _lib.vqe_hamiltonian_free(h)
    D = len(set((np.unique(x) >> 10).tolist()) - {0})
    assert wins, "expected the window form for this Hamiltonian"
    assert 3 * len(wins) - 1 < D + 2
    for W in wins:
        assert bin(W).count("1") == _lib.HPSI_WINDOW_QUBITS and W & 0b111 == 0b111 and W < (1 << wl.n_qubits)
    for xm in np.unique(x).tolist():
        assert any(int(xm) & ~W == 0 for W in wins)


def test_hamiltonian_window_plan_splits_classes():
    """One X group with 700 distinct z patterns on 14 qubits: its terms fall
    into more classes (equal in-window z bits) than one pass holds (512), so
    the window takes two passes over the same qubits."""
    n = 14
    rng = np.random.default_rng(11)
    xs = [1] * 700 + [1 << 10, 1 << 11, 1 << 12, 1 << 13, (1 << 10) | (1 << 13)] * 4
    zs = list(rng.choice(1 << n, 700, replace=False)) + list(rng.integers(0, 1 << n, 20))
    x, z = np.array(xs, np.uint64), np.array(zs, np.uint64)
    h = _lib.vqe_hamiltonian_create(n, x, z, rng.normal(size=len(xs)))
    try:
        plan = _lib.vqe_hamiltonian_plan(h)
    finally:
        _lib.vqe_hamiltonian_free(h)
    assert len(plan) == 2 and plan[0] == plan[1]
    high = 0b1111 << 10  # every x lies in qubits 0 and 10..13
    assert plan[0] & (high | 0b111) == high | 0b111 and bin(plan[0]).count("1") == _lib.HPSI_WINDOW_QUBITS
    assert 512 < len({int(zi) & plan[0] for zi in z[:700]}) <= 1024


def test_hamiltonian_window_plan_small_n():
    """At the window size (13 qubits) one window holds every qubit (one pass,
    2 S); below it H psi keeps the tile form."""
    k = _lib.HPSI_WINDOW_QUBITS
    wl = synth.WORKLOADS["hubbard1d_6"]
    x, z, w = lham.from_lattice(wl.lattice)
    h = _lib.vqe_hamiltonian_create(k, x, z, w)  # the 12-qubit chain on k qubits (the top ones idle)
    assert _lib.vqe_hamiltonian_plan(h) == [(1 << k) - 1]
    _lib.vqe_hamiltonian_free(h)
    h = _lib.vqe_hamiltonian_create(k - 1, x, z, w)
    assert _lib.vqe_hamiltonian_plan(h) == []
    _lib.vqe_hamiltonian_free(h)
    h = _lib.vqe_hamiltonian_create(10, np.array([1, 3], np.uint64), np.array([0, 2], np.uint64), np.array([1.0, 0.5]))
    assert _lib.vqe_hamiltonian_plan(h) == []
    _lib.vqe_hamiltonian_free(h)


def test_hamiltonian_window_plan_deterministic_and_compact():
    """The window cover is a deterministic function of the Hamiltonian (its
    restarts use a fixed seeded stream) and keeps the pass counts reached by
    the multi-start greedy: 4 for the 32-qubit Hubbard step, 4 at 28 qubits,
    at most 20 for the 32-qubit molecule-shaped Hamiltonian slimmed at 1e-3
    (its groups spread so that no window overflows one pass's classes)."""
    cases = [("hubbard4x4", None, 4), ("hubbard2x7", None, 4), ("molecule_16", 1e-3, 20)]
    for name, th, most in cases:
        wl = synth.WORKLOADS[name]
        if wl.kind == "molecule":
            h1, g2 = synth.molecule_integrals(wl.n_orb, wl.integral_seed)
            x, z, w = lham.molecule(h1, g2)
            keep, _, _ = _lib.vqe_slim_hamiltonian(x, z, w, _lib.SLIM_THRESHOLD, th)
            x, z, w = x[keep == 1], z[keep == 1], w[keep == 1]
        else:
            x, z, w = lham.from_lattice(wl.lattice)
        plans = []
        for _ in range(2):
            h = _lib.vqe_hamiltonian_create(wl.n_qubits, x, z, w)
            try:
                plans.append(_lib.vqe_hamiltonian_plan(h))
            finally:
                _lib.vqe_hamiltonian_free(h)
        assert plans[0] == plans[1], name
        assert 1 <= len(plans[0]) <= most, (name, len(plans[0]))
