"""Scheduler tests of the serving loop on the CPU, with a mock executor that
sleeps instead of launching kernels and checks the HBM budget itself."""
import threading
import time

import numpy as np
import pytest

from paper_2402_11878_amd.serving import Server, percentile


class MockExecutor:
    def __init__(self, budget, small_n_max=12, fail_theta=None, dur=0.02):
        self.budget = budget
        self.small_n_max = small_n_max
        self.fail_theta = fail_theta
        self.dur = dur
        self.resident = 0
        self.lock = threading.Lock()
        self.running = 0
        self.max_running = 0
        self.order = []

    def is_small(self, inst):
        return inst.n <= self.small_n_max

    def footprint(self, inst):
        return 0 if self.is_small(inst) else 3 * 8 * (1 << inst.n)

    def make_resident(self, inst):
        with self.lock:
            self.resident += inst.footprint
            assert self.resident <= self.budget, "budget exceeded"
        inst.state = "buffers"

    def release(self, inst):
        with self.lock:
            self.resident -= inst.footprint
        inst.state = None

    def _result(self, theta):
        if self.fail_theta is not None and theta[0] == self.fail_theta:
            raise RuntimeError("injected failure")
        return float(np.sum(theta)), 2 * theta

    def run_one(self, inst, theta):
        assert inst.state == "buffers"
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)
            self.order.append(inst.iid)
        time.sleep(self.dur * (1 + (inst.n - 12) / 8))
        with self.lock:
            self.running -= 1
        return self._result(theta)

    def run_batch(self, items):
        time.sleep(self.dur)
        out = []
        for inst, th in items:
            try:
                out.append(self._result(th))
            except Exception as e:
                out.append(e)
        return out

    def run_mid_batch(self, items):
        for inst, _ in items:
            assert inst.state is None and not self.is_small(inst)  # batched: no resident buffers
        with self.lock:
            self.mid_sizes = getattr(self, "mid_sizes", []) + [len(items)]
        return self.run_batch(items)


def _server(ex, budget, **kw):
    return Server(ex, budget, **kw)


def test_results_and_budget():
    budget = 3 * 8 * (1 << 20) * 2        # room for two 20-qubit instances
    ex = MockExecutor(budget)
    srv = _server(ex, budget, n_workers=3)
    for i, n in enumerate([12, 16, 20, 20, 20, 12]):
        srv.add_instance(i, n, None, None)
    futs = [(i, k, srv.submit(i, np.full(3, float(10 * i + k)))) for k in range(4) for i in range(6)]
    for i, k, f in futs:
        E, g = f.result(timeout=20)
        assert E == 3 * (10 * i + k)
    srv.close()
    assert srv.peak_used <= budget
    assert ex.resident == 0
    assert ex.max_running >= 2                 # large requests overlapped


def test_small_requests_are_batched_while_busy():
    ex = MockExecutor(1 << 30, dur=0.05)
    srv = _server(ex, 1 << 30, n_workers=1, max_batch=64)
    for i in range(10):
        srv.add_instance(i, 12, None, None)
    futs = [srv.submit(i % 10, np.array([float(i)])) for i in range(40)]
    for f in futs:
        f.result(timeout=20)
    srv.close()
    assert max(srv.batches) > 1
    assert sum(srv.batches) == 40


def test_continuous_admission():
    """Requests that arrive while others are running start before those finish."""
    budget = 1 << 30
    ex = MockExecutor(budget, dur=0.2)
    srv = _server(ex, budget, n_workers=4)
    for i in range(4):
        srv.add_instance(i, 16, None, None)
    f0 = srv.submit(0, np.zeros(2))
    time.sleep(0.05)
    f1 = srv.submit(1, np.zeros(2))
    f1.result(timeout=10)
    f0.result(timeout=10)
    srv.close()
    r0, r1 = srv.completed[0], srv.completed[1]
    assert ex.max_running == 2


def test_failure_isolation():
    ex = MockExecutor(1 << 30, fail_theta=-1.0)
    srv = _server(ex, 1 << 30, n_workers=2)
    srv.add_instance(0, 12, None, None)
    srv.add_instance(1, 16, None, None)
    good = [srv.submit(i % 2, np.array([float(i)])) for i in range(6)]
    bad = [srv.submit(0, np.array([-1.0])), srv.submit(1, np.array([-1.0]))]
    more = [srv.submit(i % 2, np.array([float(i)])) for i in range(6)]
    for f in good + more:
        assert f.result(timeout=10)[0] >= 0
    for f in bad:
        with pytest.raises(RuntimeError):
            f.result(timeout=10)
    srv.close()


def test_no_starvation_of_large_instance():
    """A 20-qubit instance needing the whole budget runs although smaller
    instances keep the memory busy."""
    big = 3 * 8 * (1 << 20)
    budget = big
    ex = MockExecutor(budget, dur=0.01)
    srv = _server(ex, budget, n_workers=3, max_wait=0.1)
    srv.add_instance(0, 20, None, None)
    for i in range(1, 4):
        srv.add_instance(i, 16, None, None)
    stop = threading.Event()

    def spam():
        k = 0
        while not stop.is_set():
            srv.submit(1 + k % 3, np.zeros(1))
            k += 1
            time.sleep(0.002)

    t = threading.Thread(target=spam)
    t.start()
    time.sleep(0.05)
    f = srv.submit(0, np.ones(1))
    f.result(timeout=10)
    stop.set()
    t.join()
    srv.close()
    assert srv.peak_used <= budget


def test_oversized_instance_rejected():
    ex = MockExecutor(1 << 20)
    srv = _server(ex, 1 << 20)
    with pytest.raises(ValueError):
        srv.add_instance(0, 20, None, None)
    srv.close()


def test_percentile_matches_numpy():
    rng = np.random.default_rng(0)
    v = rng.exponential(size=101).tolist()
    for q in (50, 90, 99):
        assert abs(percentile(v, q) - np.percentile(v, q)) < 1e-12


def test_burst_is_batched_and_evictions_counted():
    """A burst queued with submit_many reaches the batch loop together (one
    launch holds several small requests); a budget below the summed
    footprints makes the workers evict idle instances and re-admit them."""
    budget = 3 * 8 * (1 << 16) * 2       # two 16-qubit instances at a time
    ex = MockExecutor(budget, dur=0.01)
    srv = _server(ex, budget, n_workers=3)
    for i, n in enumerate([12, 12, 12, 16, 16, 16, 16]):
        srv.add_instance(i, n, None, None)
    items = [(i, np.full(2, float(10 * i + k))) for k in range(3) for i in range(7)]
    futs = srv.submit_many(items)
    for (i, th), f in zip(items, futs):
        assert f.result(timeout=20)[0] == 2 * th[0]
    srv.close()
    assert max(srv.batches) >= 2
    assert srv.evictions >= 1
    assert srv.peak_used <= budget and ex.resident == 0


def test_mid_lane_is_not_blocked_by_large_requests():
    """With a mid lane, mid-size requests are served by their own worker while
    every large worker is busy with long requests."""
    ex = MockExecutor(1 << 34, dur=0.2)
    srv = _server(ex, 1 << 34, n_workers=1, mid_n_max=20, mid_workers=1)
    srv.add_instance(0, 28, None, None)
    srv.add_instance(1, 16, None, None)
    fl = srv.submit(0, np.ones(1))
    time.sleep(0.02)
    fm = srv.submit(1, np.ones(1))
    fm.result(timeout=10)
    assert not fl.done()            # the mid request finished while the large one still ran
    fl.result(timeout=10)
    srv.close()


def test_mid_batch_lane_batches_queued_mid_requests():
    """With mid_batch, queued mid-size requests are launched together by a
    batch loop of their own: no resident state, no footprint, one launch
    for a burst; small and large requests keep their own paths."""
    budget = 3 * 8 * (1 << 24)            # one 24-qubit instance
    ex = MockExecutor(budget, dur=0.05)
    srv = _server(ex, budget, n_workers=1, mid_n_max=20, mid_batch=True)
    sizes = [12, 16, 16, 18, 20, 20, 24]
    for i, n in enumerate(sizes):
        srv.add_instance(i, n, None, None)
    items = [(i, np.full(2, float(10 * i + k))) for k in range(2) for i in range(len(sizes))]
    futs = srv.submit_many(items)
    for (i, th), f in zip(items, futs):
        assert f.result(timeout=20)[0] == 2 * th[0]
    srv.close()
    assert sum(srv.mid_batches) == 2 * 5 and max(srv.mid_batches) >= 2
    assert ex.mid_sizes == srv.mid_batches
    assert all(srv.instances[i].footprint == 0 for i in range(5))
    assert srv.instances[6].footprint > 0 and srv.peak_used <= budget and ex.resident == 0


def test_mid_batch_split_by_size():
    """mid_batch_n_max splits the mid lane: requests up to it are batched,
    larger mid-size ones go to the mid workers (resident state)."""
    ex = MockExecutor(1 << 34, dur=0.02)
    srv = _server(ex, 1 << 34, n_workers=1, mid_n_max=20, mid_workers=1, mid_batch=True, mid_batch_n_max=16)
    for i, n in enumerate([14, 16, 18, 20, 24]):
        srv.add_instance(i, n, None, None)
    items = [(i, np.full(2, float(10 * i + k))) for k in range(3) for i in range(5)]
    for (i, th), f in zip(items, srv.submit_many(items)):
        assert f.result(timeout=20)[0] == 2 * th[0]
    srv.close()
    assert sum(srv.mid_batches) == 6
    assert [srv.instances[i].footprint == 0 for i in range(5)] == [True, True, False, False, False]
    with pytest.raises(ValueError):
        _server(ex, 1 << 34, mid_n_max=20, mid_workers=0, mid_batch=True, mid_batch_n_max=16)


def test_energy_fn_runs_the_adjoint_only_for_a_gradient(monkeypatch):
    """autograd.energy / EnergyFn call the energy + gradient entry point only
    when theta needs a gradient; otherwise the forward sweep and the grouped
    energy (library calls stubbed: this checks the dispatch on the host)."""
    import torch
    from paper_2402_11878_amd import _lib, autograd

    calls = []

    class FakeState:
        def __init__(self, k):
            self.handle = k

    class FakeWs:
        def get(self, n, dtype, n_ckpt, count=None):
            return [FakeState(k) for k in range(2 + n_ckpt if count is None else count)]

    class FakeCircuit:
        n, handle = 4, "C"

    class FakeHamiltonian:
        handle = "H"

    def grad(psi, lam, c, th, h, ckpt=()):
        calls.append("grad")
        return 1.5, np.arange(len(th), dtype=np.float64)

    monkeypatch.setattr(_lib, "vqe_energy_grad", grad)
    monkeypatch.setattr(_lib, "vqe_state_set_basis", lambda s, b: calls.append("basis"))
    monkeypatch.setattr(_lib, "vqe_apply_circuit", lambda s, c, th: calls.append("circuit"))
    monkeypatch.setattr(_lib, "vqe_expect_pauli", lambda s, h, mode: (calls.append("energy"), (2.5, 1.0))[1])
    ws, C, H = FakeWs(), FakeCircuit(), FakeHamiltonian()

    th = torch.zeros(3, dtype=torch.float64, requires_grad=True)
    E = autograd.energy(th, H, C, "c128", 0, ws)
    assert calls == ["grad"] and E.item() == 1.5
    E.backward()
    assert th.grad.tolist() == [0.0, 1.0, 2.0]

    for run in (lambda: autograd.energy(th.detach(), H, C, "c128", 0, ws),
                lambda: autograd.EnergyFn.apply(th.detach(), H, C, "c128", 0, ws)):
        calls.clear()
        E = run()
        assert calls == ["basis", "circuit", "energy"] and E.item() == 2.5 and not E.requires_grad
    calls.clear()
    with torch.no_grad():
        E = autograd.energy(th, H, C, "c128", 0, ws)
    assert calls == ["basis", "circuit", "energy"] and E.item() == 2.5


def test_workspace_grows_entries_on_demand(monkeypatch):
    """Workspace.get allocates only the states asked for and reuses them: an
    energy-only call takes psi alone, a later gradient call adds lam (and
    checkpoints) to the same entry (allocation stubbed)."""
    import types
    import torch
    from paper_2402_11878_amd import autograd

    made = []

    class FakeState:
        def __init__(self, n, dtype):
            made.append((n, dtype))

        def free(self):
            made.append("free")

    monkeypatch.setattr(autograd, "State", FakeState)
    monkeypatch.setattr(torch.cuda, "current_stream", lambda: types.SimpleNamespace(cuda_stream=7))
    ws = autograd.Workspace()
    (psi,) = ws.get(20, "c128", 0, count=1)
    assert made == [(20, "c128")]
    psi2, lam = ws.get(20, "c128", 0)
    assert psi2 is psi and len(made) == 2
    assert ws.get(20, "c128", 0, count=1)[0] is psi and len(made) == 2
    assert len(ws.get(20, "c128", 2)) == 4 and len(made) == 6  # another entry: psi, lam, 2 checkpoints
    ws.clear()
    assert made.count("free") == 6
