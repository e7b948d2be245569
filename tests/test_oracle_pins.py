"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a worked closed form, a textbook
result, an invariant of the mathematics, or brute force.  A mistake anywhere in
the oracle (a dropped term, a wrong sign, a swapped index, a transposed
operand) should fail at least one of them.
"""
import math

import numpy as np
import pytest

import synth
from oracle import closed_forms as cf
from oracle import ed, expect, grad, hamiltonian as ham, slim
from oracle import statevector as sv


# ------------------------------------------------------------------ Hamiltonians
def test_jw_two_site_hubbard_worked_form():
    """2-site Hubbard (4 qubits) written out by hand (Sec. II-B, eqs. 1-4):
    I: U/2; Z_j: -U/4; Z0Z1, Z2Z3: +U/4; X0Z1X2, Y0Z1Y2, X1Z2X3, Y1Z2Y3: -t/2."""
    t, U = 1.3, 4.7
    H = ham.hubbard(2, [(0, 1)], t, U)
    want = {
        "IIII": U / 2, "ZIII": -U / 4, "IZII": -U / 4, "IIZI": -U / 4, "IIIZ": -U / 4,
        "ZZII": U / 4, "IIZZ": U / 4,
        "XZXI": -t / 2, "YZYI": -t / 2, "IXZX": -t / 2, "IYZY": -t / 2,
    }
    got = {"".join(k): v for k, v in H.items()}
    assert set(got) == set(want)
    for k in want:
        assert abs(got[k] - want[k]) < 1e-14, k


@pytest.mark.parametrize("name,terms,groups", [
    ("hubbard1d_6", 39, 11), ("hubbard2x7", 127, 43), ("hubbard4x4", 145, 49)])
def test_hubbard_counts_closed_form(name, terms, groups):
    """Terms = 4E + 3N + 1 and X-groups = 2E + 1 for E bonds and N sites."""
    lat = synth.WORKLOADS[name].lattice
    E, N = len(lat.bonds), lat.n_sites
    assert (4 * E + 3 * N + 1, 2 * E + 1) == (terms, groups)
    H = ham.hubbard(lat.n_sites, list(lat.bonds), lat.t, lat.U)
    x, z, w = ham.to_masks(H)
    assert len(w) == terms
    assert len(set(x.tolist())) == groups


def test_two_site_hubbard_ed_closed_forms():
    """Global ground energy -t at U=4 (one electron); -2t at U=0 (free fermions);
    half-filling singlet (U - sqrt(U^2+16t^2))/2 is an eigenvalue."""
    H4 = ham.hubbard(2, [(0, 1)], 1.0, 4.0)
    ev = np.linalg.eigvalsh(ed.dense(H4, 4))
    assert abs(ev[0] - (-1.0)) < 1e-12
    assert np.min(np.abs(ev - (4 - math.sqrt(32)) / 2)) < 1e-12
    H0 = ham.hubbard(2, [(0, 1)], 1.0, 0.0)
    assert abs(ed.ground_energy(H0, 4) - (-2.0)) < 1e-12


@pytest.mark.parametrize("sites,bonds", [
    (4, synth.chain_bonds(4)), (6, synth.chain_bonds(6)), (6, synth.snake_bonds(2, 3, False))])
def test_free_fermion_energy_matches_ed(sites, bonds):
    """At U = 0, ED over the full Fock space equals twice the sum of the negative
    single-particle hopping levels."""
    H = ham.hubbard(sites, bonds, 1.0, 0.0)
    n = 2 * sites
    assert abs(ed.ground_energy(H, n) - ed.free_fermion_energy(sites, bonds, 1.0)) < 1e-9


def test_dense_and_sparse_matrices_agree():
    """Kronecker-built dense H equals the signed-permutation sparse H."""
    H = ham.hubbard(3, synth.chain_bonds(3), 1.0, 2.5)
    D = ed.dense(H, 6)
    S = ed.sparse(H, 6).toarray()
    assert np.max(np.abs(D - S)) < 1e-13
    assert np.max(np.abs(D - D.conj().T)) < 1e-13


def test_molecule_one_orbital_spectrum():
    """One spatial orbital: H = h (n_up + n_dn) + g n_up n_dn, spectrum {0, h, h, 2h+g}."""
    h = np.array([[0.7]])
    g = np.full((1, 1, 1, 1), 0.3)
    H = ham.molecule(h, g)
    ev = np.sort(np.linalg.eigvalsh(ed.dense(H, 2)))
    assert np.allclose(ev, np.sort([0.0, 0.7, 0.7, 2 * 0.7 + 0.3]), atol=1e-13)


def test_molecule_symmetries():
    """Molecule-shaped H is Hermitian and conserves particle number and S_z."""
    h, g = synth.molecule_integrals(3, seed=5)
    H = ham.molecule(h, g)
    n = 6
    D = ed.dense(H, n)
    assert np.max(np.abs(D - D.conj().T)) < 1e-13
    b = np.arange(1 << n)
    occ = np.array([[(bb >> j) & 1 for j in range(n)] for bb in b])
    Nop = np.diag(occ.sum(1)).astype(float)
    Sz = np.diag(occ[:, 0::2].sum(1) - occ[:, 1::2].sum(1)).astype(float)
    assert np.max(np.abs(D @ Nop - Nop @ D)) < 1e-12
    assert np.max(np.abs(D @ Sz - Sz @ D)) < 1e-12


def test_molecule_matches_one_body_diagonal():
    """With g = 0, H = sum_pq h_pq a+_p a_q: its single-particle block is h (per spin)."""
    h, _ = synth.molecule_integrals(3, seed=2)
    H = ham.molecule(h, np.zeros((3, 3, 3, 3)))
    D = ed.dense(H, 6)
    one = [1 << j for j in range(0, 6, 2)]           # one up electron in orbital p
    block = D[np.ix_(one, one)]
    assert np.max(np.abs(block - h)) < 1e-13


def test_restricted_matrix_is_a_block_of_the_dense_matrix():
    """P H P on a sector equals the rows and columns of the Kronecker-built
    dense H at those basis states, for a particle-conserving molecule-shaped
    H and for an arbitrary Pauli sum (which leaks out of the sector)."""
    h, g = synth.molecule_integrals(4, seed=9)
    H = ham.molecule(h, g)
    basis = ed.sector_basis(8, 2, 1)
    assert len(basis) == 6 * 4 and all(bin(b).count("1") == 3 for b in basis)
    D = ed.dense(H, 8)
    assert np.max(np.abs(ed.restricted(H, 8, basis) - D[np.ix_(basis, basis)])) < 1e-14
    rng = np.random.default_rng(2)
    Hr = {tuple(rng.choice(list("IXYZ"), size=6)): float(rng.normal()) for _ in range(25)}
    b6 = ed.sector_basis(6, 1, 2)
    assert np.max(np.abs(ed.restricted(Hr, 6, b6) - ed.dense(Hr, 6)[np.ix_(b6, b6)])) < 1e-14


def test_mask_round_trip():
    H = ham.hubbard(3, synth.chain_bonds(3), 1.0, 3.0)
    x, z, w = ham.to_masks(H)
    back = ham.from_masks(6, x, z, w)
    assert back == H


# ------------------------------------------------------------------ simulator
@pytest.mark.parametrize("t,p", [(0.3, -1.1), (2.9, 0.4), (-1.7, 2.2)])
def test_single_qubit_bloch(t, p):
    """RZ(p) RY(t)|0> has Bloch vector (sin t cos p, sin t sin p, cos t)."""
    psi = sv.run(1, [("RY", 0, -1, 0, 0.0), ("RZ", 0, -1, 1, 0.0)], [t, p])
    vals = [expect.expect_term_masks(psi, 1, x, z).real for (x, z) in ((1, 0), (1, 1), (0, 1))]
    assert np.allclose(vals, cf.bloch_ry_rz(t, p), atol=1e-14)


def test_cnot_truth_table():
    """CNOT(0 -> 1): |00>->|00>, |01>->|11>, |10>->|10>, |11>->|01> (bit 0 = control)."""
    for b, want in ((0, 0), (1, 3), (2, 2), (3, 1)):
        psi = sv.apply_cnot(sv.basis_state(2, b), 2, 0, 1)
        assert psi[want] == 1.0


@pytest.mark.parametrize("n", [3, 7, 11])
def test_ladder_prefix_xor(n):
    """The ascending CNOT ladder maps |b> to |M b>, (M b)_j = b_0 ^ ... ^ b_j."""
    gates = [("CNOT", q, q + 1, -1, 0.0) for q in range(n - 1)]
    rng = np.random.default_rng(n)
    for b in rng.integers(0, 1 << n, size=8):
        psi = sv.run(n, gates, [], psi=sv.basis_state(n, int(b)))
        assert psi[cf.ladder_map(int(b), n)] == 1.0


@pytest.mark.parametrize("n", [4, 9])
def test_one_layer_closed_form(n):
    """One ansatz layer: <P> from Clifford conjugation of P through the ladder and
    the per-qubit Bloch vectors equals the simulated value."""
    rng = np.random.default_rng(7 + n)
    th = rng.uniform(-math.pi, math.pi, size=2 * n)
    psi = sv.run(n, sv.layered_ansatz(n, 1), th)
    for _ in range(25):
        x, z = int(rng.integers(0, 1 << n)), int(rng.integers(0, 1 << n))
        want = cf.one_layer_expectation(n, th[:n], th[n:], x, z)
        got = expect.expect_term_masks(psi, n, x, z).real
        assert abs(got - want) < 1e-12


@pytest.mark.parametrize("n,layers", [(5, 6), (8, 4)])
def test_clifford_tableau_matches_simulation(n, layers):
    """Angles in {0, +-pi/2, pi}: stabiliser-tableau <P> equals the simulated value."""
    rng = np.random.default_rng(n * 10 + layers)
    th = rng.choice([0.0, math.pi / 2, -math.pi / 2, math.pi], size=2 * n * layers)
    gates = sv.layered_ansatz(n, layers)
    psi = sv.run(n, gates, th)
    terms = [(int(rng.integers(0, 1 << n)), int(rng.integers(0, 1 << n))) for _ in range(40)]
    terms += [(0, 1 << q) for q in range(n)]
    want = cf.clifford_expectations(n, gates, th, terms)
    for (x, z), w in zip(terms, want):
        assert abs(expect.expect_term_masks(psi, n, x, z).real - w) < 1e-12


def test_norm_and_inverse():
    """Unitary gates preserve the norm; applying U then U^dag returns |0...0>."""
    n = 8
    gates = sv.layered_ansatz(n, 3)
    th = synth.theta(3, 2 * n * 3)
    psi = sv.run(n, gates, th)
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-12
    for g in reversed(gates):
        sv.apply_gate(psi, n, g, th, inverse=True)
    assert abs(psi[0] - 1.0) < 1e-12
    assert np.max(np.abs(psi[1:])) < 1e-12


def test_theta_zero_energy():
    """At theta = 0 the state stays |0...0>: E = sum of w over the x = 0 terms."""
    lat = synth.WORKLOADS["hubbard1d_6"].lattice
    H = ham.hubbard(lat.n_sites, list(lat.bonds), lat.t, lat.U)
    n = 12
    psi = sv.run(n, sv.layered_ansatz(n, 2), np.zeros(4 * n))
    E, _ = expect.energy(psi, n, H)
    x, z, w = ham.to_masks(H)
    assert abs(E - math.fsum(w[x == 0])) < 1e-12


def test_expectation_routes_agree():
    """Per-qubit sigma route and the vectorised b^x route give the same <P>."""
    n = 7
    psi = sv.run(n, sv.layered_ansatz(n, 2), synth.theta(11, 4 * n))
    rng = np.random.default_rng(0)
    for _ in range(30):
        s = tuple(rng.choice(list("IXYZ"), size=n))
        x, z = expect.string_masks(s)
        a = expect.expect_term_gates(psi, n, s)
        b = expect.expect_term_masks(psi, n, x, z)
        assert abs(a - b) < 1e-13


def test_variational_bound_config0():
    """E(theta) >= E_0 (ED) for the 12-qubit 6-site chain at random angles."""
    wl = synth.WORKLOADS["hubbard1d_6"]
    lat = wl.lattice
    H = ham.hubbard(lat.n_sites, list(lat.bonds), lat.t, lat.U)
    E0 = ed.ground_energy(H, 12)
    assert E0 >= ed.free_fermion_energy(lat.n_sites, list(lat.bonds), lat.t) - 1e-9
    for s in range(3):
        th = synth.theta(s, wl.n_params)
        E, norm = expect.energy(sv.run(12, sv.layered_ansatz(12, wl.layers), th), 12, H)
        assert E >= E0 - 1e-10
        assert abs(norm - 1) < 1e-12


# ------------------------------------------------------------------ gradients
def test_gradients_three_ways():
    """Parameter shift (exact), central differences and the adjoint sweep agree."""
    n, layers = 6, 2
    H = ham.hubbard(3, synth.chain_bonds(3), 1.0, 4.0)
    gates = sv.layered_ansatz(n, layers)
    th = synth.theta(4, 2 * n * layers)
    E, g_adj = grad.adjoint(n, gates, th, H)
    ps = grad.param_shift(n, gates, th, H)
    fd = grad.finite_diff(n, gates, th, H, indices=range(0, 24, 5))
    g_ps = np.array([ps[k] for k in range(len(th))])
    assert np.max(np.abs(g_adj - g_ps)) < 1e-12
    for k, v in fd.items():
        assert abs(v - g_ps[k]) < 1e-7
    assert abs(E - expect.energy(sv.run(n, gates, th), n, H)[0]) < 1e-13


def test_parameter_shift_single_rotation_closed_form():
    """E = <Z> after RY(t): cos t, derivative -sin t."""
    H = {("Z",): 1.0}
    for t in (0.3, -2.0):
        g = grad.param_shift(1, [("RY", 0, -1, 0, 0.0)], [t], H)[0]
        assert abs(g + math.sin(t)) < 1e-14


# ------------------------------------------------------------------ slimming
def _rand_terms(seed, n_terms=200, ties=False):
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 1 << 10, size=n_terms).astype(np.uint64)
    z = rng.integers(0, 1 << 10, size=n_terms).astype(np.uint64)
    w = rng.normal(size=n_terms) * 10.0 ** rng.uniform(-6, 0, size=n_terms)
    if ties:
        w = np.round(w * 4) / 4 + 0.0
        w[w == 0] = 0.25
    x[0] = z[0] = 0
    return x, z, w


@pytest.mark.parametrize("seed,ties", [(0, False), (1, True), (2, True)])
def test_slim_threshold_bruteforce(seed, ties):
    """Keep iff |w| >= Th, identity always kept; dropped sum bounds |dE| (Sec. II-D)."""
    x, z, w = _rand_terms(seed, ties=ties)
    for th in (0.0, 1e-4, 0.25, float(np.abs(w[5]))):
        keep, dropped = slim.threshold(x, z, w, th)
        want = np.array([1 if (i == 0 or abs(w[i]) >= th) else 0 for i in range(len(w))])
        assert np.array_equal(keep, want)
        assert abs(dropped - math.fsum(abs(v) for v in w[want == 0])) < 1e-12
    keep0, d0 = slim.threshold(x, z, w, 0.0)
    assert keep0.all() and d0 == 0.0


@pytest.mark.parametrize("seed,ties", [(3, False), (4, True)])
def test_slim_remove_percent_and_budget(seed, ties):
    x, z, w = _rand_terms(seed, ties=ties)
    N = len(w) - 1
    for pct in (0, 10, 33, 70, 100):
        keep, dropped = slim.remove_percent(x, z, w, pct)
        assert int((keep == 0).sum()) == (N * pct) // 100
        if 0 < pct < 100:       # every dropped |w| <= every kept non-identity |w|
            assert np.abs(w[keep == 0]).max() <= np.abs(w[1:][keep[1:] == 1]).min()
    for lim in (0.0, 1e-3, 0.5, 1e9):
        keep, s = slim.budget(x, z, w, lim)
        assert s <= lim
        assert keep[0] == 1
        kept = np.abs(w[1:][keep[1:] == 1])
        if len(kept):
            assert s + kept.min() > lim     # the next term would exceed the budget


@pytest.mark.parametrize("seed,ties", [(5, False), (6, True)])
def test_slim_keep_top_bruteforce(seed, ties):
    """Keep-top mode keeps exactly the K non-identity terms of largest |w|
    (ties by x, then z), and the identity; the dropped sum is the rest's |w|."""
    x, z, w = _rand_terms(seed, ties=ties)
    N = len(w) - 1
    for K in (0, 1, 17, N - 1, N, N + 5):
        keep, dropped = slim.keep_top(x, z, w, K)
        assert keep[0] == 1 and int(keep[1:].sum()) == min(K, N)
        key = lambda i: (-abs(w[i]), int(x[i]), int(z[i]))
        ranked = sorted(range(1, N + 1), key=key)
        assert set(np.nonzero(keep[1:])[0] + 1) == set(ranked[:K])
        assert abs(dropped - math.fsum(abs(w[i]) for i in ranked[K:])) < 1e-12


def test_slim_energy_bound():
    """|E_full - E_slim| <= sum of dropped |w| for a normalised state (Sec. II-D)."""
    h, g = synth.molecule_integrals(3, seed=1)
    H = ham.molecule(h, g)
    x, z, w = ham.to_masks(H)
    n = 6
    psi = sv.run(n, sv.layered_ansatz(n, 3), synth.theta(9, 36))
    E_full, _ = expect.energy_masks(psi, n, x, z, w)
    for th in (1e-4, 1e-3, 1e-2, 1e-1):
        keep, dropped = slim.threshold(x, z, w, th)
        k = keep == 1
        E_slim, _ = expect.energy_masks(psi, n, x[k], z[k], w[k])
        assert slim.dropped_bound_check(E_full, E_slim, dropped)


# ------------------------------------------------------------------ excitation gates (eq. 5)
_P2 = {"I": np.eye(2), "X": np.array([[0, 1], [1, 0]]), "Y": np.array([[0, -1j], [1j, 0]]),
       "Z": np.diag([1.0, -1.0]),
       "+": np.array([[0, 0], [1, 0]]),    # |1><0| (raise the occupation)
       "-": np.array([[0, 1], [0, 0]])}    # |0><1| (lower it)


def _kron_ops(n, ops):
    """Operator with ops[q] on qubit q (identity elsewhere); qubit n-1 leftmost."""
    from functools import reduce
    return reduce(np.kron, [_P2[ops.get(q, "I")] for q in reversed(range(n))]).astype(np.complex128)


def test_single_excitation_is_exp_of_pauli_generator():
    """SEXC(t) on (p, q) = expm(-i t G / 2) with G = (X_p Y_q - Y_p X_q)/2,
    built from Pauli matrices (scipy's expm, not the oracle's pair loop)."""
    from scipy.linalg import expm
    n = 3
    rng = np.random.default_rng(5)
    for (p, q) in ((0, 1), (2, 0), (0, 2)):
        G = 0.5 * (_kron_ops(n, {p: "X", q: "Y"}) - _kron_ops(n, {p: "Y", q: "X"}))
        for t in (0.7, -2.1):
            psi = rng.normal(size=8) + 1j * rng.normal(size=8)
            ref = expm(-0.5j * t * G) @ psi
            got = sv.apply_excitation(psi.copy(), n, sv.SEXC, (p, q), t)
            assert np.max(np.abs(got - ref)) < 1e-13


def test_double_excitation_is_exp_of_ladder_generator():
    """DEXC(t) on (p, q, r, s) = expm(t K / 2) with K = s-_p s-_q s+_r s+_s - h.c.
    (|1100> <-> |0011> on those qubits), built from ladder matrices."""
    from scipy.linalg import expm
    n = 5
    rng = np.random.default_rng(6)
    for (p, q, r, s) in ((0, 1, 2, 3), (4, 1, 0, 3), (2, 4, 1, 0)):
        K = _kron_ops(n, {p: "-", q: "-", r: "+", s: "+"})
        K = K - K.conj().T
        for t in (1.1, -0.4):
            psi = rng.normal(size=32) + 1j * rng.normal(size=32)
            ref = expm(0.5 * t * K) @ psi
            got = sv.apply_excitation(psi.copy(), n, sv.DEXC, (p, q, r, s), t)
            assert np.max(np.abs(got - ref)) < 1e-13


def test_excitation_closed_forms_and_conservation():
    """On basis states: SEXC(t)|b_p=1,b_q=0> = cos(t/2)|..> + sin(t/2)|b_p=0,b_q=1>;
    DEXC on |1100> likewise; every excitation circuit keeps particle number and
    the up/down counts (spin-orbital 2i + sigma)."""
    n, t = 6, 0.9
    c, s = math.cos(t / 2), math.sin(t / 2)
    psi = sv.apply_excitation(sv.basis_state(n, 0b000100), n, sv.SEXC, (2, 5), t)
    assert abs(psi[0b000100] - c) < 1e-15 and abs(psi[0b100000] - s) < 1e-15
    assert abs(np.linalg.norm(psi) - 1) < 1e-15
    psi = sv.apply_excitation(sv.basis_state(n, 0b000011), n, sv.DEXC, (0, 1, 4, 5), t)
    assert abs(psi[0b000011] - c) < 1e-15 and abs(psi[0b110000] - s) < 1e-15
    gates = sv.excitation_ansatz(8, 4, layers=2)
    th = synth.theta(3, len(gates))
    psi = sv.run(8, gates, th, psi=sv.basis_state(8, sv.hartree_fock_index(4)))
    idx = np.arange(256)
    up = np.array([bin(b & 0x55).count("1") for b in idx])
    dn = np.array([bin(b & 0xAA).count("1") for b in idx])
    assert np.sum(np.abs(psi[(up != 2) | (dn != 2)]) ** 2) < 1e-28
    assert abs(np.linalg.norm(psi) - 1) < 1e-14


def test_excitation_gradients_three_ways():
    """Four-term parameter shift (Anselmetti et al. 2021), central differences
    and the adjoint sweep agree for an S/D circuit from the Hartree-Fock state."""
    n, ne = 8, 4
    h, g = synth.molecule_integrals(4, 3)
    H = ham.molecule(h, g)
    gates = sv.excitation_ansatz(n, ne)
    th = synth.theta(8, len(gates)) * 0.5
    psi0 = sv.basis_state(n, sv.hartree_fock_index(ne))
    gates_hf = [("X", q, -1, -1, 0.0) for q in range(ne)] + gates
    E, g_adj = grad.adjoint(n, gates_hf, th, H)
    ps = grad.param_shift(n, gates_hf, th, H)
    fd = grad.finite_diff(n, gates_hf, th, H, indices=range(0, len(th), 4))
    g_ps = np.array([ps[k] for k in range(len(th))])
    assert np.max(np.abs(g_adj - g_ps)) < 1e-12
    for k, v in fd.items():
        assert abs(v - g_adj[k]) < 1e-7
    assert abs(E - expect.energy(sv.run(n, gates, th, psi=psi0), n, H)[0]) < 1e-13


def test_excitation_vqe_reaches_sector_ground_state():
    """2 electrons in 2 spatial orbitals (4 qubits, one up and one down): the
    S/D ansatz from Hartree-Fock spans the real states of that sector, so
    minimising E(theta) reaches the lowest eigenvalue of H restricted to the
    sector (dense diagonalisation); every theta stays above it."""
    from scipy.optimize import minimize
    n, ne = 4, 2
    h, g = synth.molecule_integrals(2, 11)
    H = ham.molecule(h, g)
    M = ed.dense(H, n)
    sector = [b for b in range(16) if bin(b & 0x5).count("1") == 1 and bin(b & 0xA).count("1") == 1]
    E0 = np.linalg.eigvalsh(M[np.ix_(sector, sector)]).min()
    gates = [("X", q, -1, -1, 0.0) for q in range(ne)] + sv.excitation_ansatz(n, ne)
    P = 1 + max(gt[3] for gt in gates)
    f = lambda t: expect.energy(sv.run(n, gates, t), n, H)[0]
    for seed in range(3):
        assert f(synth.theta(seed, P)) >= E0 - 1e-12
    best = minimize(f, np.zeros(P) + 0.1, method="BFGS", options={"gtol": 1e-10})
    assert abs(best.fun - E0) < 1e-9


def _random_unitary(k, rng):
    a = rng.normal(size=(1 << k, 1 << k)) + 1j * rng.normal(size=(1 << k, 1 << k))
    q, r = np.linalg.qr(a)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _random_state(n, rng):
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("q0,k", [(0, 5), (2, 3), (4, 2)])
def test_dense_window_contiguous_is_kron(q0, k):
    """On qubits q0 .. q0+k-1 in ascending order the dense window is the full
    operator I (x) U (x) I (numpy kron, most significant factor first)."""
    n = 7
    rng = np.random.default_rng(20 + q0)
    U = _random_unitary(k, rng)
    psi = _random_state(n, rng)
    full = np.kron(np.kron(np.eye(1 << (n - q0 - k)), U), np.eye(1 << q0))
    got = sv.apply_dense(psi.copy(), n, list(range(q0, q0 + k)), U)
    assert np.max(np.abs(got - full @ psi)) <= 1e-13


def test_dense_window_product_and_permutation():
    """Any qubit order: a Kronecker product of 2x2 matrices (pattern bit i on
    qubits[i]) equals one 2x2 per qubit; a permutation matrix of CNOT between
    pattern bits equals the CNOT on their qubits; a unitary keeps the norm."""
    n, qubits = 8, [6, 1, 7, 3, 4]
    rng = np.random.default_rng(7)
    singles = [_random_unitary(1, rng) for _ in qubits]
    U = np.array([[1.0 + 0j]])
    for m in singles:  # bit i of the pattern is factor i counted from the right
        U = np.kron(m, U)
    psi = _random_state(n, rng)
    want = psi.copy()
    for q, m in zip(qubits, singles):
        sv.apply_1q(want, n, q, m)
    assert np.max(np.abs(sv.apply_dense(psi.copy(), n, qubits, U) - want)) <= 1e-13
    P = np.zeros((32, 32))
    for p in range(32):
        P[p ^ (((p >> 3) & 1) << 1), p] = 1.0  # control pattern bit 3, target bit 1
    want = sv.apply_cnot(psi.copy(), n, qubits[3], qubits[1])
    assert np.max(np.abs(sv.apply_dense(psi.copy(), n, qubits, P) - want)) == 0.0
    W = _random_unitary(5, rng)
    assert abs(np.linalg.norm(sv.apply_dense(psi.copy(), n, qubits, W)) - 1.0) <= 1e-13


# ------------------------------------------------------------------ gates beyond RY / RZ / CNOT
def _bloch(psi):
    """(<X>, <Y>, <Z>) of a one-qubit state read off its two amplitudes:
    2 Re(a* b), 2 Im(a* b), |a|^2 - |b|^2."""
    a, b = psi[0], psi[1]
    ab = np.conj(a) * b
    return (2 * ab.real, 2 * ab.imag, abs(a) ** 2 - abs(b) ** 2)


def _rand_state(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("t", [0.3, 2.9, -1.7])
def test_rx_bloch_vector(t):
    """RX(t)|0> = exp(-i t X/2)|0> rotates the Bloch vector about x: (0, -sin t, cos t)."""
    psi = sv.run(1, [("RX", 0, -1, 0, 0.0)], [t])
    assert np.allclose(_bloch(psi), (0.0, -math.sin(t), math.cos(t)), atol=1e-15)


def test_rx_is_ry_conjugated_by_rz():
    """A rotation about x is the rotation about y conjugated by RZ(pi/2):
    RX(t) = RZ(-pi/2) RY(t) RZ(pi/2) exactly (the RZ phases cancel), on any qubit
    of a random state; RY and RZ are pinned by their Bloch vectors."""
    n = 5
    for q, t in ((0, 0.7), (3, -2.3), (4, 1.9)):
        psi = _rand_state(n, 40 + q)
        a = sv.run(n, [("RX", q, -1, 0, 0.0)], [t], psi=psi)
        b = sv.run(n, [("RZ", q, -1, -1, math.pi / 2), ("RY", q, -1, 0, 0.0),
                       ("RZ", q, -1, -1, -math.pi / 2)], [t], psi=psi)
        assert np.max(np.abs(a - b)) < 1e-14


def test_x_and_hadamard_closed_forms():
    """X|0> = |1>, X|1> = |0>; H|0> = (|0>+|1>)/sqrt2 (Bloch (1,0,0)),
    H|1> = (|0>-|1>)/sqrt2 (Bloch (-1,0,0)); H = X RY(pi/2) exactly
    (RY(pi/2) = [[1,-1],[1,1]]/sqrt2, then X swaps the rows); H^2 = I and
    H Z H = X on a random state."""
    assert np.array_equal(sv.run(1, [("X", 0, -1, -1, 0.0)], [], psi=sv.basis_state(1, 0)), [0, 1])
    assert np.array_equal(sv.run(1, [("X", 0, -1, -1, 0.0)], [], psi=sv.basis_state(1, 1)), [1, 0])
    h0 = sv.run(1, [("H", 0, -1, -1, 0.0)], [], psi=sv.basis_state(1, 0))
    h1 = sv.run(1, [("H", 0, -1, -1, 0.0)], [], psi=sv.basis_state(1, 1))
    assert np.allclose(_bloch(h0), (1, 0, 0), atol=1e-15)
    assert np.allclose(_bloch(h1), (-1, 0, 0), atol=1e-15)
    assert np.allclose(h0, [2 ** -0.5, 2 ** -0.5], atol=1e-16)
    assert np.allclose(h1, [2 ** -0.5, -(2 ** -0.5)], atol=1e-16)
    n = 4
    for q in range(n):
        psi = _rand_state(n, 50 + q)
        a = sv.run(n, [("H", q, -1, -1, 0.0)], [], psi=psi)
        b = sv.run(n, [("RY", q, -1, -1, math.pi / 2), ("X", q, -1, -1, 0.0)], [], psi=psi)
        assert np.max(np.abs(a - b)) < 1e-15
        assert np.max(np.abs(sv.run(n, [("H", q, -1, -1, 0.0)], [], psi=a) - psi)) < 1e-15
        # H Z H = X: <psi|H Z H|psi> = <psi|X_q|psi>, Z and X by their masks
        zq = expect.expect_term_masks(a, n, 0, 1 << q)
        xq = expect.expect_term_masks(psi, n, 1 << q, 0)
        assert abs(zq - xq) < 1e-14


def test_cz_truth_table_and_cnot_identity():
    """CZ multiplies |11> by -1 and leaves |00>, |01>, |10> unchanged; it is
    symmetric in its qubits and equals H_t CNOT(c -> t) H_t."""
    for b in range(4):
        psi = sv.apply_cz(sv.basis_state(2, b), 2, 0, 1)
        want = sv.basis_state(2, b) * (-1.0 if b == 3 else 1.0)
        assert np.array_equal(psi, want)
    n = 5
    for (c, t) in ((0, 1), (4, 1), (2, 3)):
        psi = _rand_state(n, 60 + c + t)
        a = sv.run(n, [("CZ", c, t, -1, 0.0)], [], psi=psi)
        b = sv.run(n, [("CZ", t, c, -1, 0.0)], [], psi=psi)
        h = sv.run(n, [("H", t, -1, -1, 0.0), ("CNOT", c, t, -1, 0.0), ("H", t, -1, -1, 0.0)], [], psi=psi)
        assert np.max(np.abs(a - b)) == 0.0
        assert np.max(np.abs(a - h)) < 1e-15


# ------------------------------------------------------------------ two-body term of eq. (1)
def test_molecule_two_electron_slater_condon():
    """Two spatial orbitals, generic h and 8-fold-symmetric chemist integrals
    g_pqrs = (pq|rs).  The diagonal of H on a determinant is the textbook
    Slater-Condon energy: sum of h_ii over occupied spin-orbitals plus, per
    occupied pair, the Coulomb integral J_ij = (ii|jj) minus the exchange
    integral K_ij = (ij|ji) when the two spins are equal.  So (spin-orbital
    2p + sigma):
      |0up 1up>, |0dn 1dn>:  h00 + h11 + J - K
      |0up 1dn>, |0dn 1up>:  h00 + h11 + J
      |0up 0dn>:             2 h00 + (00|00);  |1up 1dn>: 2 h11 + (11|11)
      |0up 0dn 1up>:         2 h00 + h11 + (00|00) + 2 J - K
    and the triplet energy h00 + h11 + J - K is an eigenvalue three times in
    the two-electron sector (S_z = 1, 0, -1)."""
    rng = np.random.default_rng(3)
    a = rng.normal(size=(2, 2))
    h = a + a.T
    g = np.zeros((2, 2, 2, 2))
    for p in range(2):
        for q in range(2):
            for r in range(2):
                for s in range(2):
                    key = tuple(sorted((tuple(sorted((p, q))), tuple(sorted((r, s))))))
                    g[p, q, r, s] = {((0, 0), (0, 0)): 0.61, ((0, 0), (0, 1)): 0.13,
                                     ((0, 0), (1, 1)): 0.47, ((0, 1), (0, 1)): 0.19,
                                     ((0, 1), (1, 1)): -0.08, ((1, 1), (1, 1)): 0.55}[key]
    J, K = g[0, 0, 1, 1], g[0, 1, 1, 0]
    assert abs(J - K) > 0.2                 # exchange and Coulomb distinguishable
    D = ed.dense(ham.molecule(h, g), 4)
    bit = lambda *so: sum(1 << s for s in so)
    want = {
        bit(0, 2): h[0, 0] + h[1, 1] + J - K, bit(1, 3): h[0, 0] + h[1, 1] + J - K,
        bit(0, 3): h[0, 0] + h[1, 1] + J, bit(1, 2): h[0, 0] + h[1, 1] + J,
        bit(0, 1): 2 * h[0, 0] + g[0, 0, 0, 0], bit(2, 3): 2 * h[1, 1] + g[1, 1, 1, 1],
        bit(0, 1, 2): 2 * h[0, 0] + h[1, 1] + g[0, 0, 0, 0] + 2 * J - K,
        bit(0): h[0, 0], bit(2): h[1, 1],
    }
    for b, e in want.items():
        assert abs(D[b, b] - e) < 1e-14, (bin(b), D[b, b], e)
    two = [b for b in range(16) if bin(b).count("1") == 2]
    ev = np.linalg.eigvalsh(D[np.ix_(two, two)])
    trip = h[0, 0] + h[1, 1] + J - K
    assert int(np.sum(np.abs(ev - trip) < 1e-12)) == 3


# ------------------------------------------------------------------ terms with an odd number of Y
def _random_pauli_sum(n, n_terms, seed):
    """Hermitian Pauli sum over arbitrary strings, odd numbers of Y included
    (JW images of real integrals never hold those, so the phases i and -i of
    eq. 3's Y = iXZ are only exercised here)."""
    rng = np.random.default_rng(seed)
    H = {}
    for _ in range(n_terms):
        s = tuple(rng.choice(list("IXYZ"), size=n))
        H[s] = H.get(s, 0.0) + float(rng.normal())
    assert any(s.count("Y") % 2 == 1 for s in H)
    return H


def test_hamiltonian_apply_and_sparse_match_kron_with_odd_y():
    """H psi of the oracle (signed permutations per term) and the sparse
    matrix equal the Kronecker-built dense H for strings with odd Y counts."""
    n = 5
    H = _random_pauli_sum(n, 30, 8)
    D = ed.dense(H, n)
    psi = _rand_state(n, 9)
    assert np.max(np.abs(expect.apply_hamiltonian(psi, n, H) - D @ psi)) < 1e-13
    assert np.max(np.abs(ed.sparse(H, n).toarray() - D)) < 1e-14
    E, _ = expect.energy(psi, n, H)
    assert abs(E - float(np.vdot(psi, D @ psi).real)) < 1e-13


def test_gradients_three_ways_all_gate_kinds():
    """Adjoint, parameter shift and central differences agree on a random
    circuit of RX, RY, RZ, H, X, CNOT and CZ gates against a Pauli sum with odd
    Y counts; the energy equals <psi|D|psi> with the Kronecker-built D."""
    n = 4
    rng = np.random.default_rng(12)
    gates, k = [], 0
    for _ in range(14):
        kind = str(rng.choice(["RX", "RY", "RZ", "H", "X", "CNOT", "CZ"]))
        q0 = int(rng.integers(0, n))
        if kind in ("CNOT", "CZ"):
            q1 = int((q0 + 1 + rng.integers(0, n - 1)) % n)
            gates.append((kind, q0, q1, -1, 0.0))
        elif kind in ("RX", "RY", "RZ"):
            gates.append((kind, q0, -1, k, 0.0))
            k += 1
        else:
            gates.append((kind, q0, -1, -1, 0.0))
    assert any(g[0] == "RX" for g in gates)
    H = _random_pauli_sum(n, 12, 13)
    th = rng.uniform(-math.pi, math.pi, size=k)
    E, g_adj = grad.adjoint(n, gates, th, H)
    ps = grad.param_shift(n, gates, th, H)
    fd = grad.finite_diff(n, gates, th, H)
    g_ps = np.array([ps[i] for i in range(k)])
    g_fd = np.array([fd[i] for i in range(k)])
    assert np.max(np.abs(g_adj - g_ps)) < 1e-12
    assert np.max(np.abs(g_fd - g_ps)) < 1e-7
    psi = sv.run(n, gates, th)
    assert abs(E - float(np.vdot(psi, ed.dense(H, n) @ psi).real)) < 1e-13


def test_energy_is_a_rayleigh_quotient():
    """Eq. 7 divides by <psi|psi>: scaling psi by any non-zero c leaves E
    unchanged and multiplies the reported norm by |c|^2 (both energy routes)."""
    n = 5
    H = _random_pauli_sum(n, 20, 14)
    x, z, w = ham.to_masks(H)
    psi = _rand_state(n, 15)
    E1, n1 = expect.energy(psi, n, H)
    E2, n2 = expect.energy((1.7 - 0.4j) * psi, n, H)
    E3, _ = expect.energy_masks(0.3j * psi, n, x, z, w)
    assert abs(n1 - 1.0) < 1e-14 and abs(n2 - abs(1.7 - 0.4j) ** 2) < 1e-13
    assert abs(E1 - E2) < 1e-13 and abs(E1 - E3) < 1e-13
