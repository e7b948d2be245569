"""Continuous-batching request loop for energy + gradient evaluations.

Many optimiser instances (each a circuit, a Hamiltonian and a qubit count)
send evaluation requests theta -> (E(theta), dE/dtheta); the paper ran the
independent circuit runs of an optimiser iteration concurrently on separate
node groups (Sec. II-C).  Here they share one GPU:

  * small requests (n <= the LDS limit of the batched kernel) are collected
    while the device is busy and launched together, one workgroup per
    request (vqe_batch_energy_grad);
  * large requests run on worker threads, each instance on its own HIP stream
    with its state vectors (psi, lam, checkpoints) resident in HBM, so
    several instances' kernels overlap on the device;
  * optionally, mid-size requests (up to `mid_n_max` qubits) form a lane of
    their own, so that they never queue behind large ones on the host:
    either dedicated workers running them one at a time, or (`mid_batch`) a
    second batch loop that launches every queued mid-size request together
    (the tile passes of vqe_batch_energy_grad, one launch per pass index);
    the GPU executor can also reserve a few compute units for the batched
    and mid-size lanes (streams with CU masks), so that their short kernels
    do not wait for the compute units that the persistent kernels of large
    requests hold;
  * an instance becomes resident only while the summed footprint of resident
    instances stays within the HBM budget; idle resident instances are
    evicted least-recently-used first;
  * requests are served oldest first; a request that has waited longer than
    `max_wait` blocks admission of younger ones until it runs (no
    starvation);
  * a failing request resolves its own future with the error and the loop
    carries on.
Each result depends only on its request (fixed kernels and reduction order),
so it is bitwise the same whatever else is in flight.

The executor is pluggable: ``GpuExecutor`` drives libvqe.so; tests drive the
scheduler with a mock executor on the CPU.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Instance:
    iid: int
    n: int
    circuit: object
    hamiltonian: object
    footprint: int = 0
    resident: bool = False
    busy: bool = False
    last_used: float = 0.0
    state: object = None


@dataclass
class Request:
    inst: Instance
    theta: np.ndarray
    submit_t: float
    future: Future = field(default_factory=Future)
    start_t: float = 0.0   # when a worker or a batch launch took it
    done_t: float = 0.0


def percentile(values, q):
    """q-th percentile (0..100) by linear interpolation between order statistics."""
    v = sorted(values)
    if not v:
        return float("nan")
    pos = (len(v) - 1) * q / 100.0
    lo = int(np.floor(pos))
    hi = min(lo + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (pos - lo)


class Server:
    def __init__(self, executor, budget_bytes, n_workers=4, max_batch=64, max_wait=2.0, clock=time.perf_counter,
                 mid_n_max=None, mid_workers=1, mid_batch=False, mid_batch_n_max=None):
        self.ex = executor
        # requests of more than the batch limit and at most mid_n_max qubits go to the mid lane: with
        # mid_batch, those of at most mid_batch_n_max qubits (default: all of them) to its batch loop,
        # the others to its workers
        self.mid_n_max = mid_n_max if (mid_n_max is not None and (mid_workers > 0 or mid_batch)) else None
        self.mid_batch = bool(mid_batch) and self.mid_n_max is not None
        self.mid_batch_n_max = (min(mid_batch_n_max, self.mid_n_max) if mid_batch_n_max is not None
                                else self.mid_n_max) if self.mid_batch else None
        if self.mid_batch and self.mid_batch_n_max < self.mid_n_max and mid_workers < 1:
            raise ValueError("mid_batch_n_max below mid_n_max needs mid_workers >= 1")
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.max_wait = max_wait
        self.clock = clock
        self.instances = {}
        self.used = 0
        self.peak_used = 0
        self._cv = threading.Condition()
        self._small = collections.deque()
        self._large = collections.deque()
        self._mid = collections.deque()
        self._midb = collections.deque()
        self._closing = False
        self.completed = []
        self.batches = []          # sizes of the launched batches of small requests
        self.mid_batches = []      # ... of mid-size requests (mid_batch)
        self.evictions = 0         # resident instances released to admit others
        self.max_concurrent = 0
        self._running = 0
        self._threads = [threading.Thread(target=self._batch_loop, args=(self._small, self.ex.run_batch,
                                                                         self.batches), daemon=True)]
        self._threads += [threading.Thread(target=self._worker_loop, args=(self._large,), daemon=True)
                          for _ in range(n_workers)]
        if self.mid_batch:
            self._threads.append(threading.Thread(target=self._batch_loop, args=(self._midb, self.ex.run_mid_batch,
                                                                                self.mid_batches), daemon=True))
        if self.mid_n_max is not None and (not self.mid_batch or self.mid_batch_n_max < self.mid_n_max):
            self._threads += [threading.Thread(target=self._worker_loop, args=(self._mid,), daemon=True)
                              for _ in range(mid_workers)]
        for t in self._threads:
            t.start()

    # ------------------------------------------------------------ client side
    def add_instance(self, iid, n, circuit, hamiltonian):
        inst = Instance(iid, n, circuit, hamiltonian)
        inst.footprint = 0 if self._batched(inst) else self.ex.footprint(inst)
        if not self._batched(inst) and inst.footprint > self.budget:
            raise ValueError(f"instance {iid} needs {inst.footprint} bytes, more than the budget {self.budget}")
        prepare = getattr(self.ex, "prepare", None)
        if prepare is not None and not self._batched(inst):
            prepare(inst)  # kernel compilation stays out of the instance's first request
        with self._cv:
            self.instances[iid] = inst
        return inst

    def submit(self, iid, theta):
        return self.submit_many([(iid, theta)])[0]

    def submit_many(self, items):
        """Queues a burst of requests [(iid, theta), ...] at once (one lock
        hold, so the loops see all of them together); returns their futures."""
        reqs = [Request(self.instances[iid], np.asarray(theta, dtype=np.float64), self.clock())
                for iid, theta in items]
        with self._cv:
            if self._closing:
                raise RuntimeError("server is closed")
            for req in reqs:
                self._queue_of(req.inst).append(req)
            self._cv.notify_all()
        return [r.future for r in reqs]

    def close(self):
        with self._cv:
            self._closing = True
            self._cv.notify_all()
        for t in self._threads:
            t.join()
        for inst in self.instances.values():
            if inst.resident:
                self.ex.release(inst)
                inst.resident = False

    def _queue_of(self, inst):
        if self.ex.is_small(inst):
            return self._small
        if self.mid_batch and inst.n <= self.mid_batch_n_max:
            return self._midb
        if self.mid_n_max is not None and inst.n <= self.mid_n_max:
            return self._mid
        return self._large

    def _batched(self, inst):
        """Served by a batch launch (no resident state of its own)."""
        return self.ex.is_small(inst) or (self.mid_batch and inst.n <= self.mid_batch_n_max)

    def latencies(self):
        return [r.done_t - r.submit_t for r in self.completed]

    # ------------------------------------------------------------ internals
    def _finish(self, req, result=None, error=None):
        req.done_t = self.clock()
        with self._cv:
            self.completed.append(req)
        if error is not None:
            req.future.set_exception(error)
        else:
            req.future.set_result(result)

    def _batch_loop(self, queue, run, sizes):
        """Launches everything queued (up to max_batch) as one batch, again and
        again; requests queued meanwhile form the next batch."""
        while True:
            with self._cv:
                while not queue and not self._closing:
                    self._cv.wait()
                if not queue and self._closing:
                    return
                batch = [queue.popleft() for _ in range(min(self.max_batch, len(queue)))]
                t_start = self.clock()
                for r in batch:
                    r.start_t = t_start
                self._running += 1
                self.max_concurrent = max(self.max_concurrent, self._running)
            sizes.append(len(batch))
            try:
                results = run([(r.inst, r.theta) for r in batch])
            except Exception as e:  # the whole launch failed: fail its requests, keep serving
                results = [e] * len(batch)
            with self._cv:
                self._running -= 1
            for r, res in zip(batch, results):
                if isinstance(res, Exception):
                    self._finish(r, error=res)
                else:
                    self._finish(r, result=res)

    def _admit(self, inst):
        """Make inst resident if the budget allows (evicting idle instances). Caller holds the lock."""
        if inst.resident:
            return True
        need = inst.footprint
        if self.used + need > self.budget:
            idle = sorted((i for i in self.instances.values() if i.resident and not i.busy),
                          key=lambda i: i.last_used)
            for victim in idle:
                if self.used + need <= self.budget:
                    break
                self.ex.release(victim)
                victim.resident = False
                self.used -= victim.footprint
                self.evictions += 1
        if self.used + need > self.budget:
            return False
        self.ex.make_resident(inst)
        inst.resident = True
        self.used += need
        self.peak_used = max(self.peak_used, self.used)
        return True

    def _pick(self, queue):
        """Oldest runnable request of `queue` (caller holds the lock), or None."""
        now = self.clock()
        for k, req in enumerate(queue):
            if req.inst.busy:
                continue
            if self._admit(req.inst):
                del queue[k]
                return req
            if now - req.submit_t > self.max_wait:
                return None          # the old request waits for memory: admit nobody younger
        return None

    def _worker_loop(self, queue):
        while True:
            with self._cv:
                while True:
                    if self._closing and not queue:
                        return
                    req = self._pick(queue)
                    if req is not None:
                        break
                    self._cv.wait(timeout=0.05)
                req.inst.busy = True
                req.start_t = self.clock()
                self._running += 1
                self.max_concurrent = max(self.max_concurrent, self._running)
            try:
                res = self.ex.run_one(req.inst, req.theta)
                err = None
            except Exception as e:
                res, err = None, e
            with self._cv:
                req.inst.busy = False
                req.inst.last_used = self.clock()
                self._running -= 1
                self._cv.notify_all()
            self._finish(req, result=res, error=err)


class GpuExecutor:
    """Runs requests with libvqe.so: batched LDS kernel for small states, the
    fused-pass adjoint path on per-instance streams for large ones.

    reserve_cus > 0 splits the compute units: the batched launches and the
    instances of at most mid_n_max qubits run on streams restricted to the
    first reserve_cus compute units, larger instances on big_streams
    streams restricted to the others (vqe_stream_create with a CU mask).
    Batched mid-size requests (run_mid_batch) have a batch handle and stream
    of their own.  chunk_passes > 0 submits the evaluations of instances
    above mid_n_max qubits in chunks of that many window passes (about one
    ansatz layer at 3), waiting for each chunk before queueing the next, so
    that kernels of other lanes start between chunks."""

    def __init__(self, dtype="c64", n_ckpt=0, small_n_max=None, reserve_cus=0, mid_n_max=20, big_streams=3,
                 chunk_passes=0):
        import torch

        from . import _lib
        self.torch, self.L = torch, _lib
        self.dtype = _lib.VQE_C64 if dtype == "c64" else _lib.VQE_C128
        self.tdtype = torch.complex64 if self.dtype == _lib.VQE_C64 else torch.complex128
        self.amp = 8 if self.dtype == _lib.VQE_C64 else 16
        self.n_ckpt = n_ckpt
        lim = _lib.BATCH_MAX_QUBITS[self.dtype]
        self.small_n_max = lim if small_n_max is None else min(small_n_max, lim)
        self.mid_n_max = mid_n_max
        self.chunk_passes = int(chunk_passes)
        self._own_streams = []
        self._rr = 0
        if reserve_cus > 0:
            ncu = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
            if not 0 < reserve_cus < ncu:
                raise ValueError(f"reserve_cus must be in (0, {ncu})")
            fast = _lib.vqe_stream_create(range(reserve_cus))
            fast2 = _lib.vqe_stream_create(range(reserve_cus))
            big = [_lib.vqe_stream_create(range(reserve_cus, ncu)) for _ in range(big_streams)]
            self._own_streams = [fast, fast2] + big
            self.batch_stream = torch.cuda.ExternalStream(fast)
            self.fast_stream = self.batch_stream
            self.mid_stream = torch.cuda.ExternalStream(fast2)
            self.big_streams = [torch.cuda.ExternalStream(b) for b in big]
        else:
            self.batch_stream = torch.cuda.Stream()
            self.mid_stream = torch.cuda.Stream()
            self.fast_stream = None
            self.big_streams = []
        self.batch = _lib.vqe_batch_create(self.dtype, self.batch_stream.cuda_stream)
        self.mid_batch = _lib.vqe_batch_create(self.dtype, self.mid_stream.cuda_stream)

    def _stream_for(self, inst):
        if self.fast_stream is None:
            return self.torch.cuda.Stream()
        if inst.n <= self.mid_n_max:
            return self.fast_stream
        self._rr = (self._rr + 1) % len(self.big_streams)
        return self.big_streams[self._rr]

    def is_small(self, inst):
        return inst.n <= self.small_n_max

    def prepare(self, inst):
        if not self.is_small(inst):
            self.L.vqe_circuit_prepare(inst.circuit.handle, self.dtype)

    def footprint(self, inst):
        # resident vectors: psi, lam and the checkpoints (8 * 2^n bytes per complex64 vector)
        return 0 if self.is_small(inst) else (2 + self.n_ckpt) * self.amp * (1 << inst.n)

    def make_resident(self, inst):
        torch, L = self.torch, self.L
        st = self._stream_for(inst)
        bufs = [torch.empty(1 << inst.n, dtype=self.tdtype, device="cuda") for _ in range(2 + self.n_ckpt)]
        hs = [L.vqe_state_alloc(inst.n, self.dtype, b.data_ptr(), b.numel() * b.element_size(), st.cuda_stream)
              for b in bufs]
        inst.state = (st, bufs, hs)

    def release(self, inst):
        st, bufs, hs = inst.state
        for h in hs:
            self.L.vqe_state_free(h)
        inst.state = None

    def run_one(self, inst, theta):
        st, bufs, hs = inst.state
        chunk = self.chunk_passes if inst.n > self.mid_n_max else 0
        return self.L.vqe_energy_grad(hs[0], hs[1], inst.circuit.handle, theta, inst.hamiltonian.handle,
                                      ckpt=hs[2:], chunk_passes=chunk)

    def run_batch(self, items):
        return self.L.vqe_batch_energy_grad(
            self.batch, [(inst.circuit.handle, inst.hamiltonian.handle, th) for inst, th in items])

    def run_mid_batch(self, items):
        return self.L.vqe_batch_energy_grad(
            self.mid_batch, [(inst.circuit.handle, inst.hamiltonian.handle, th) for inst, th in items])

    def close(self):
        if self.batch:
            self.L.vqe_batch_free(self.batch)
            self.batch = None
        if self.mid_batch:
            self.L.vqe_batch_free(self.mid_batch)
            self.mid_batch = None
        if self._own_streams:
            self.torch.cuda.synchronize()
            for st in self._own_streams:
                self.L.vqe_stream_destroy(st)
            self._own_streams = []
