"""GPU: the autograd Function, and the serving loop on the device — every
served result equals the same request run alone, bit for bit, and matches the
oracle."""
import numpy as np
import pytest

import synth
from oracle import grad as ogr, hamiltonian as oham
from paper_2402_11878_amd import _lib, hamiltonians as lham
from paper_2402_11878_amd.core import Circuit, Hamiltonian

from gpu_util import oracle_gates, rel_err, say

pytestmark = pytest.mark.gpu


def _chain(n, U=4.0):
    lat = synth.Lattice(n // 2, tuple(synth.chain_bonds(n // 2)), 1.0, U)
    return lham.from_lattice(lat)


def test_energy_fn_autograd():
    import torch
    from paper_2402_11878_amd.autograd import EnergyFn, Workspace
    say("case autograd")
    n, L = 10, 3
    x, z, w = _chain(n)
    H = Hamiltonian(n, x, z, w)
    C = Circuit.layered(n, L)
    th = torch.tensor(synth.theta(8, C.n_params), dtype=torch.float64, requires_grad=True)
    ws = Workspace()
    E = EnergyFn.apply(th, H, C, "c128", 0, ws)
    E.backward()
    E_ref, g_ref = ogr.adjoint(n, oracle_gates(C.gates), th.detach().numpy(), oham.from_masks(n, x, z, w))
    assert rel_err(E.item(), E_ref) <= 1e-10
    assert np.max(np.abs(th.grad.numpy() - g_ref)) <= 1e-9 * max(np.max(np.abs(g_ref)), 1)
    # chain rule through a downstream expression
    th2 = th.detach().clone().requires_grad_(True)
    loss = 3.0 * EnergyFn.apply(th2, H, C, "c128", 0, ws) ** 2
    loss.backward()
    assert np.max(np.abs(th2.grad.numpy() - 6.0 * E_ref * g_ref)) <= 1e-8 * max(abs(6 * E_ref), 1)
    # no gradient wanted: the forward sweep and the grouped energy only
    from paper_2402_11878_amd.autograd import energy
    with torch.no_grad():
        E1 = energy(th, H, C, "c128", 0, ws)
    E2 = EnergyFn.apply(th.detach(), H, C, "c128", 0, ws)
    assert not E1.requires_grad and not E2.requires_grad
    assert rel_err(E1.item(), E_ref) <= 1e-10 and rel_err(E2.item(), E_ref) <= 1e-10
    ws.clear()


def _serve(ex, budget, insts, reqs, n_workers):
    from paper_2402_11878_amd.serving import Server
    srv = Server(ex, budget, n_workers=n_workers)
    for i, (n, C, H, *_r) in enumerate(insts):
        srv.add_instance(i, n, C, H)
    futs = srv.submit_many(reqs)
    out = [f.result(timeout=120) for f in futs]
    srv.close()
    return srv, out


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_served_equals_alone(dt):
    """Every request in a burst served concurrently (small ones batched into
    one launch, large ones overlapping on worker streams, a budget that
    forces evictions and re-admissions) equals the same request run alone,
    bit for bit, and matches the oracle."""
    from paper_2402_11878_amd.serving import GpuExecutor
    say(f"case serving {dt}")
    specs = [(8, 2, 0), (12, 3, 1), (14, 2, 2), (16, 2, 3), (10, 4, 4), (18, 1, 5)]
    insts = []
    for n, L, seed in specs:
        x, z, w = _chain(n)
        insts.append((n, Circuit.layered(n, L), Hamiltonian(n, x, z, w), x, z, w, seed))
    ex = GpuExecutor(dt, n_ckpt=1)
    reqs = [(i, synth.theta(100 * i + k, insts[i][1].n_params)) for k in range(3) for i in range(len(insts))]
    amp = 8 if dt == "c64" else 16
    footprints = [3 * amp * (1 << n) for n, *_r in insts if n > ex.small_n_max]   # psi, lam, 1 checkpoint
    # alone: one request at a time, everything fits
    alone = []
    for i, th in reqs:
        _, (res,) = _serve(ex, 64 << 20, insts, [(i, th)], 1)
        alone.append(res)
    # mix: the whole burst in flight at once, budget below the summed footprints
    budget = max(footprints) + min(footprints)
    assert budget < sum(footprints)
    srv, mixed = _serve(ex, budget, insts, reqs, 4)
    ex.close()
    assert max(srv.batches) >= 2, srv.batches          # several small requests in one launch
    assert srv.max_concurrent >= 2                     # work in flight together
    assert srv.evictions >= 1 and srv.peak_used <= budget
    for (E1, g1), (E2, g2) in zip(alone, mixed):
        assert E1 == E2 and np.array_equal(g1, g2)
    # and against the oracle
    te, tg = (1e-10, 1e-9) if dt == "c128" else (1e-5, 1e-4)
    for (i, th), (E, g) in list(zip(reqs, mixed))[:len(insts)]:
        n, C, H, x, z, w, seed = insts[i]
        E_ref, g_ref = ogr.adjoint(n, oracle_gates(C.gates), th, oham.from_masks(n, x, z, w))
        assert rel_err(E, E_ref) <= te
        assert np.max(np.abs(g - g_ref)) / max(np.max(np.abs(g_ref)), 1) <= tg


def test_served_c64_without_checkpoints_at_20_qubits():
    """The form the served stream runs: complex64, no checkpoints, a 20-qubit
    instance (specialised kernels) beside small batched ones; each result
    against the oracle and against the same request alone."""
    from paper_2402_11878_amd.serving import GpuExecutor
    say("case serving c64 n_ckpt=0 20q")
    specs = [(20, 2), (12, 2), (10, 3)]
    insts = []
    for n, L in specs:
        x, z, w = _chain(n)
        insts.append((n, Circuit.layered(n, L), Hamiltonian(n, x, z, w), x, z, w))
    ex = GpuExecutor("c64", n_ckpt=0)
    reqs = [(i, synth.theta(500 + 10 * i + k, insts[i][1].n_params)) for k in range(2) for i in range(len(insts))]
    _, mixed = _serve(ex, 1 << 30, insts, reqs, 2)
    alone = [_serve(ex, 1 << 30, insts, [r], 1)[1][0] for r in reqs]
    ex.close()
    for (E1, g1), (E2, g2) in zip(alone, mixed):
        assert E1 == E2 and np.array_equal(g1, g2)
    for (i, th), (E, g) in list(zip(reqs, mixed))[:len(insts)]:
        n, C, H, x, z, w = insts[i]
        E_ref, g_ref = ogr.adjoint(n, oracle_gates(C.gates), th, oham.from_masks(n, x, z, w))
        assert rel_err(E, E_ref) <= 1e-5
        assert np.max(np.abs(g - g_ref)) / max(np.max(np.abs(g_ref)), 1) <= 1e-4


def test_cu_masked_stream_gives_the_same_bits():
    """An evaluation on a stream restricted to 32 compute units (vqe_stream_create
    with a CU mask) gives bitwise the result of the same evaluation on an
    ordinary stream: the kernels and their reduction order do not depend on
    where the blocks run."""
    import torch
    say("case cu-masked stream")
    n = 16
    x, z, w = _chain(n)
    H = Hamiltonian(n, x, z, w)
    C = Circuit.layered(n, 3)
    th = synth.theta(77, C.n_params)
    res = []
    streams = [_lib.vqe_stream_create(range(32)), _lib.vqe_stream_create()]
    try:
        for st in streams:
            bufs = [torch.empty(1 << n, dtype=torch.complex128, device="cuda") for _ in range(2)]
            hs = [_lib.vqe_state_alloc(n, _lib.VQE_C128, b.data_ptr(), b.numel() * 16, st) for b in bufs]
            try:
                res.append(_lib.vqe_energy_grad(hs[0], hs[1], C.handle, th, H.handle))
            finally:
                for h in hs:
                    _lib.vqe_state_free(h)
    finally:
        torch.cuda.synchronize()
        for st in streams:
            _lib.vqe_stream_destroy(st)
    (E1, g1), (E2, g2) = res
    assert E1 == E2 and np.array_equal(g1, g2)
    E_ref, g_ref = ogr.adjoint(n, oracle_gates(C.gates), th, oham.from_masks(n, x, z, w))
    assert rel_err(E1, E_ref) <= 1e-10


def test_served_with_lanes_equals_alone():
    """Serving with a mid-size lane and 32 compute units reserved for the
    batched and mid-size lanes: every result equals the same request served
    alone without lanes, bit for bit."""
    from paper_2402_11878_amd.serving import GpuExecutor
    say("case serving with lanes")
    specs = [(10, 2), (12, 3), (16, 2), (18, 2), (20, 1), (22, 1)]
    insts = []
    for n, L in specs:
        x, z, w = _chain(n)
        insts.append((n, Circuit.layered(n, L), Hamiltonian(n, x, z, w), x, z, w))
    reqs = [(i, synth.theta(900 + 10 * i + k, insts[i][1].n_params)) for k in range(2) for i in range(len(insts))]
    ex0 = GpuExecutor("c64", n_ckpt=0)
    alone = [_serve(ex0, 1 << 30, insts, [r], 1)[1][0] for r in reqs]
    ex0.close()
    ex = GpuExecutor("c64", n_ckpt=0, reserve_cus=32, mid_n_max=18, big_streams=2)
    from paper_2402_11878_amd.serving import Server
    srv = Server(ex, 1 << 30, n_workers=2, mid_n_max=18, mid_workers=1)
    for i, (n, C, H, *_r) in enumerate(insts):
        srv.add_instance(i, n, C, H)
    mixed = [f.result(timeout=120) for f in srv.submit_many(reqs)]
    srv.close()
    ex.close()
    for (E1, g1), (E2, g2) in zip(alone, mixed):
        assert E1 == E2 and np.array_equal(g1, g2)


def test_served_with_mid_batches_and_chunks():
    """The served stream's default form: mid-size requests up to 16 qubits
    batched (tile passes), 18-20 qubits on the mid worker, larger ones
    submitted in chunks of 3 passes.  Batched results equal the same items
    batched alone (the batch path's own bits) and match the oracle within the
    complex64 tolerance; worker results equal the request served alone."""
    from paper_2402_11878_amd.serving import GpuExecutor, Server
    import torch
    say("case serving with mid batches and chunks")
    specs = [(10, 2), (14, 2), (16, 3), (16, 2), (18, 2), (22, 1)]
    insts = []
    for n, L in specs:
        x, z, w = _chain(n)
        insts.append((n, Circuit.layered(n, L), Hamiltonian(n, x, z, w), x, z, w))
    reqs = [(i, synth.theta(1300 + 10 * i + k, insts[i][1].n_params)) for k in range(2) for i in range(len(insts))]
    ex0 = GpuExecutor("c64", n_ckpt=0)
    alone = [_serve(ex0, 1 << 30, insts, [r], 1)[1][0] for r in reqs]
    ex0.close()
    ex = GpuExecutor("c64", n_ckpt=0, mid_n_max=20, chunk_passes=3)
    srv = Server(ex, 1 << 30, n_workers=2, mid_n_max=20, mid_workers=1, mid_batch=True, mid_batch_n_max=16)
    for i, (n, C, H, *_r) in enumerate(insts):
        srv.add_instance(i, n, C, H)
    mixed = [f.result(timeout=120) for f in srv.submit_many(reqs)]
    srv.close()
    b = _lib.vqe_batch_create(_lib.VQE_C64, torch.cuda.current_stream().cuda_stream)
    try:
        for (i, th), (E1, g1), (E2, g2) in zip(reqs, alone, mixed):
            n, C, H, x, z, w = insts[i]
            if 13 < n <= 16:
                (Eb, gb), = _lib.vqe_batch_energy_grad(b, [(C.handle, H.handle, th)])
                assert E2 == Eb and np.array_equal(g2, gb)
                assert rel_err(E2, E1) <= 1e-5
            else:
                assert E1 == E2 and np.array_equal(g1, g2)
    finally:
        _lib.vqe_batch_free(b)
        ex.close()
    assert sum(srv.mid_batches) == 6
    for (i, th), (E, g) in list(zip(reqs, mixed))[:len(insts)]:
        n, C, H, x, z, w = insts[i]
        E_ref, g_ref = ogr.adjoint(n, oracle_gates(C.gates), th, oham.from_masks(n, x, z, w))
        assert rel_err(E, E_ref) <= 1e-5
        assert np.max(np.abs(g - g_ref)) / max(np.max(np.abs(g_ref)), 1) <= 1e-4
