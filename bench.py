#!/usr/bin/env python3
"""Benchmark: VQE energy + adjoint-gradient evaluations per second at 32 qubits.

One step = one pass of the whole hot path on one parameter vector: reset to
|0...0>, the fused forward ansatz sweeps (eq. 6), lam = H psi with the energy
(eq. 7) from the X-mask-grouped kernel, and the reverse sweep that un-applies
every gate from (psi, lam) while accumulating dE/dtheta for all parameters.

Workload (default): 2-D Fermi-Hubbard on a 4 x 4 open lattice, t = 1, U = 4,
Jordan-Wigner in snake order (32 qubits, 145 Pauli terms, 49 X-mask groups),
8 layers of [RY, RZ on every qubit; CNOT ladder] = 760 gates and 512
parameters drawn uniform in [-pi, pi) from seed 0.  The headline figure uses
a complex128 state (64 GiB per vector, psi + lam + one checkpoint); the same
step on a complex64 state (FP32 amplitudes, FP64 reductions) is reported
beside it, with its energy and gradient error against the complex128 result.

Prints one JSON line.  Inputs are synthetic and resident in HBM before the
timed region starts.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("kernels.hip", "dense.hip", "jit.cpp", "api.cpp", "plan.cpp", "vqe_internal.h")


def kernel_sources_sha256():
    """Digest of every source that shapes the window kernels (the interpreted
    kernels, the generator of the specialised ones, planning and lowering)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2402_11878_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel="window_rev", record="profiles/window_rev_hubbard4x4_32q_c128_traffic.txt"):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE record (copy-calibrated), or None when a kernel
    source has changed since the counters were taken."""
    path = os.path.join(ROOT, record)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if line.startswith("#") or ":" not in line:
            continue
        k, v = line.split(":", 1)
        kv[k.strip()] = v.strip()
    if kv.get("kernel") != kernel or kv.get("sources_sha256") != kernel_sources_sha256():
        return None
    return float(kv["traffic_bytes_per_launch"])


WORKLOAD_TEXT = {
    "hubbard1d_6": "1-D Fermi-Hubbard, 6 sites open, t=1, U=4",
    "hubbard2x7": "2-D Fermi-Hubbard 2x7, periodic along the long axis, t=1, U=8, JW snake order",
    "hubbard4x4": "2-D Fermi-Hubbard 4x4 open, t=1, U=4, JW snake order",
    "molecule_10": "molecule-shaped Hamiltonian, 10 spatial orbitals, integral seed 0",
    "molecule_16": "molecule-shaped Hamiltonian, 16 spatial orbitals, integral seed 0",
}


def workload_hamiltonian(wl, threshold):
    """(x, z, w) of a workload: lattice models as built, molecule-shaped ones
    slimmed at `threshold` (default: the workload's largest threshold)."""
    import synth
    from paper_2402_11878_amd import _lib as L, hamiltonians as hm
    if wl.kind != "molecule":
        return hm.from_lattice(wl.lattice), None
    h, g = synth.molecule_integrals(wl.n_orb, wl.integral_seed)
    x, z, w = hm.molecule(h, g)
    th = max(wl.thresholds) if threshold is None else threshold
    keep, _, _ = L.vqe_slim_hamiltonian(x, z, w, L.SLIM_THRESHOLD, th)
    m = keep == 1
    return (x[m], z[m], w[m]), th


def run_dtype(torch, L, core, wl, dtype, n_ckpt, steps, warmup, thetas, threshold=None):
    """Times `steps` energy+gradient evaluations, cycling through the rows of
    `thetas` (a workload's parameter batch); returns a result dict."""
    n = wl.n_qubits
    (x, z, w), th_used = workload_hamiltonian(wl, threshold)
    H = core.Hamiltonian(n, x, z, w)
    circ = core.Circuit.layered(n, wl.layers)
    tdt = torch.complex64 if dtype == L.VQE_C64 else torch.complex128
    bufs = [torch.empty(1 << n, dtype=tdt, device="cuda") for _ in range(2 + n_ckpt)]
    st = torch.cuda.current_stream()
    handles = [L.vqe_state_alloc(n, dtype, b.data_ptr(), b.numel() * b.element_size(), st.cuda_stream) for b in bufs]
    psi, lam, ck = handles[0], handles[1], handles[2:]
    name = "c64" if dtype == L.VQE_C64 else "c128"
    try:
        for i in range(warmup):
            log(f"[bench] {name} warmup step {i + 1}/{warmup}")
            E, g = L.vqe_energy_grad(psi, lam, circ.handle, thetas[i % len(thetas)], H.handle, ckpt=ck)
        torch.cuda.synchronize()
        L.vqe_profile_reset()
        L.vqe_profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        energies = []
        grads = []
        for i in range(steps):
            E, g = L.vqe_energy_grad(psi, lam, circ.handle, thetas[i % len(thetas)], H.handle, ckpt=ck)
            energies.append(E)
            grads.append(g)
            log(f"[bench] {name} step {i + 1}/{steps} E={E:.12f}")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.vqe_profile_enable(False)
        prof = {k: L.vqe_profile_read(k) for k in range(5)}
        L.vqe_profile_reset()
    finally:
        for hnd in handles:
            L.vqe_state_free(hnd)
        del bufs
        torch.cuda.empty_cache()
    sec = (t1 - t0) / steps
    return dict(name=name, sec=sec, E=energies[-1], grad=g, grads=grads, energies=energies, prof=prof,
                threshold=th_used,
                n_gates=len(circ.gates), n_passes_adj=circ.passes_count(dtype), n_terms=H.n_terms,
                n_groups=H.n_groups,
                state_bytes=(1 << n) * (8 if dtype == L.VQE_C64 else 16), n_ckpt=n_ckpt)


def _oracle_sample(job):
    """One oracle energy + adjoint gradient of the 20-qubit sample state of
    cpu_baseline (runs in a child process for the all-core figure); returns
    its duration in seconds."""
    import synth
    from oracle import grad as ogr, hamiltonian as oham, statevector as osv
    layers, seed = job
    ns = 20
    Hs = oham.hubbard(10, synth.snake_bonds(2, 5, False), 1.0, 4.0)
    gates = osv.layered_ansatz(ns, layers)
    th = synth.theta(seed, 2 * ns * layers)
    t0 = time.perf_counter()
    ogr.adjoint(ns, gates, th, Hs)
    return time.perf_counter() - t0


def cpu_baseline(wl_name):
    """The CPU oracle, as it stands, on a bounded sample of the workload.

    The 28- and 32-qubit states do not fit the oracle's NumPy temporaries on
    the host, so the sample is the same workload shape at 20 qubits: a 2 x 5
    open Hubbard lattice (t = 1, U = 4, snake order), the same ansatz with the
    workload's layer count, energy + adjoint gradient by the oracle's
    gate-by-gate reverse sweep (about 10 s for 8 layers on one core).  Its time
    is scaled to the workload's step by 2^(n-20) (state size) times the ratio
    of (3 gates + terms) (gate sweeps of psi forward and of psi, lam in
    reverse, plus one sweep per Hamiltonian term).  Measured twice: one
    evaluation on one core (latency), and one evaluation per host core at
    once, on different angle vectors, in child processes with one thread each
    (the all-core throughput, the value reported).  Must run before the
    process touches the GPU (the children are started from it).  Lattice
    workloads only.
    """
    import multiprocessing as mp
    import synth
    wl = synth.WORKLOADS[wl_name]
    ns, ls = 20, wl.layers
    n_gates = ls * (2 * ns + ns - 1)
    n_terms = 4 * len(synth.snake_bonds(2, 5, False)) + 3 * 10 + 1
    lat = wl.lattice
    T32 = 4 * len(lat.bonds) + 3 * lat.n_sites + 1
    G32 = wl.layers * (2 * wl.n_qubits + wl.n_qubits - 1)
    scale = 2.0 ** (wl.n_qubits - ns) * (3 * G32 + T32) / (3 * n_gates + n_terms)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    os.environ["OMP_NUM_THREADS"] = "1"
    ctx = mp.get_context("spawn")
    with ctx.Pool(1) as pool:                       # one core
        t1 = pool.map(_oracle_sample, [(ls, 0)])[0]
    with ctx.Pool(cores) as pool:                   # every core, different angles
        t0 = time.perf_counter()
        ts = pool.map(_oracle_sample, [(ls, 100 + i) for i in range(cores)], chunksize=1)
        t_all = time.perf_counter() - t0
    rate_all = cores / (t_all * scale)
    return dict(value=rate_all, unit="evals/s", cores=cores, kind="oracle",
                sample=(f"oracle energy+adjoint gradient of a 20-qubit 2x5 Hubbard lattice with the same ansatz at "
                        f"{ls} layers ({n_gates} gates): {cores} at once, one per host core on different angle vectors, "
                        f"took {t_all:.2f} s; scaled by 2^{wl.n_qubits - ns} x (3*gates+terms) ratio, {scale:.0f} in "
                        f"all, to the {wl.n_qubits}-qubit step"),
                one_core=dict(value=1.0 / (t1 * scale), sample_seconds=t1),
                all_core_seconds=t_all, per_process_seconds=[round(t, 2) for t in ts], host_cpus=os.cpu_count())


def serving_bench(args, fracs=(0.5, 0.8, 0.95), baseline=True, emit=True):
    """Served stream of 32 optimiser instances (complex64, adjoint gradients,
    continuous batching) against one-at-a-time complex128 per-term energies
    with parameter-shift gradients on the same GPU.  Returns the result dict
    (printed as one JSON line when emit)."""
    import torch
    import synth
    from paper_2402_11878_amd import _lib as L, hamiltonians as hm
    from paper_2402_11878_amd.core import Circuit, Hamiltonian
    from paper_2402_11878_amd.serving import GpuExecutor, Server, percentile

    n_inst = args.instances
    insts = []
    for i in range(n_inst):
        n, (kind, src), layers, rng = synth.serving_instance(i)
        if kind == "hubbard":
            x, z, w = hm.from_lattice(src)
        else:
            h, g = synth.molecule_integrals(*src)
            x, z, w = hm.molecule(h, g)
            keep, _, _ = L.vqe_slim_hamiltonian(x, z, w, L.SLIM_THRESHOLD, args.slim)
            k = keep.astype(bool)
            x, z, w = x[k], z[k], w[k]
        insts.append(dict(i=i, n=n, kind=kind, layers=layers, rng=rng, C=Circuit.layered(n, layers),
                          H=Hamiltonian(n, x, z, w)))
    log(f"[serving] {n_inst} instances built")
    t_build = time.perf_counter()
    ex = GpuExecutor("c64", n_ckpt=0, reserve_cus=args.reserve_cus, mid_n_max=args.mid_n_max,
                     chunk_passes=args.chunk_passes)
    budget = int(args.budget_gib * (1 << 30))

    def new_server():
        srv = Server(ex, budget, n_workers=args.workers,
                     mid_n_max=args.mid_n_max if (args.mid_workers or args.mid_batch) else None,
                     mid_workers=args.mid_workers, mid_batch=bool(args.mid_batch),
                     mid_batch_n_max=args.mid_batch_n_max or None)
        for d in insts:
            srv.add_instance(d["i"], d["n"], d["C"], d["H"])
        return srv

    def draw(d):
        return d["rng"].uniform(-np.pi, np.pi, size=d["C"].n_params)

    srv = new_server()
    for f in [srv.submit(d["i"], draw(d)) for d in insts]:      # warm-up, makes instances resident
        f.result()
    torch.cuda.synchronize()
    log(f"[serving] instances registered and warm ({time.perf_counter() - t_build:.1f} s)")
    # capacity: every instance submits `reps` requests at once
    reqs = [(d["i"], draw(d)) for _ in range(args.reps) for d in insts]
    t0 = time.perf_counter()
    for f in [srv.submit(i, th) for i, th in reqs]:
        f.result()
    cap = len(reqs) / (time.perf_counter() - t0)
    log(f"[serving] capacity {cap:.2f} evals/s")
    srv.close()
    loads = {}
    for frac in fracs:
        srv = new_server()
        for f in [srv.submit(d["i"], draw(d)) for d in insts]:
            f.result()
        srv.completed.clear()
        rate = frac * cap
        arr_rng = np.random.default_rng(int(frac * 100))
        order = arr_rng.integers(0, n_inst, size=args.requests)
        gaps = arr_rng.exponential(1.0 / rate, size=args.requests)
        futs = []
        t_start = time.perf_counter()
        t_next = t_start
        for k in range(args.requests):
            t_next += gaps[k]
            while time.perf_counter() < t_next:
                time.sleep(min(0.001, max(t_next - time.perf_counter(), 0)))
            d = insts[order[k]]
            futs.append(srv.submit(d["i"], draw(d)))
        t_last_arrival = time.perf_counter()
        for f in futs:
            f.result()
        t_end = time.perf_counter()
        lat = srv.latencies()
        # completions inside the arrival window measure the sustained rate; the drain after the
        # last arrival (the largest requests still running) is reported on its own
        in_window = sum(1 for r in srv.completed if r.done_t <= t_last_arrival)
        by_n, svc_n = {}, {}
        for r in srv.completed:
            by_n.setdefault(r.inst.n, []).append(r.done_t - r.submit_t)
            svc_n.setdefault(r.inst.n, []).append(r.done_t - r.start_t)
        loads[str(frac)] = dict(offered=rate, offered_measured=args.requests / (t_last_arrival - t_start),
                                achieved=len(futs) / (t_end - t_start),
                                achieved_in_window=in_window / (t_last_arrival - t_start),
                                drain_s=t_end - t_last_arrival,
                                p50_ms=percentile(lat, 50) * 1e3, p99_ms=percentile(lat, 99) * 1e3,
                                by_qubits={str(k): dict(count=len(v), p50_ms=percentile(v, 50) * 1e3,
                                                        p99_ms=percentile(v, 99) * 1e3,
                                                        service_p50_ms=percentile(svc_n[k], 50) * 1e3,
                                                        service_max_ms=max(svc_n[k]) * 1e3)
                                           for k, v in sorted(by_n.items())},
                                batches=len(srv.batches), mean_batch=float(np.mean(srv.batches)) if srv.batches else 0,
                                mid_batches=len(srv.mid_batches),
                                mean_mid_batch=float(np.mean(srv.mid_batches)) if srv.mid_batches else 0,
                                max_concurrent=srv.max_concurrent, evictions=srv.evictions)
        log(f"[serving] load {frac}: {loads[str(frac)]}")
        srv.close()
    ex.close()
    out = {
        "metric": "served energy+gradient evals/s (32 optimiser instances) and p50/p99 latency",
        "value": cap, "unit": "evals/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f32 state, f64 reductions", "data": "synthetic",
        "config": {"workload": f"{n_inst} instances: n in {{12,16,20,24,28}}, 1-D/2-D Hubbard and molecule-shaped "
                               f"(slimmed at {args.slim}) Hamiltonians, 4-16 layers, seeds 10000+i",
                   "workers": args.workers, "mid_workers": args.mid_workers, "mid_n_max": args.mid_n_max,
                   "mid_batch": bool(args.mid_batch), "mid_batch_n_max": args.mid_batch_n_max or None,
                   "chunk_passes": args.chunk_passes,
                   "reserve_cus": args.reserve_cus, "budget_gib": args.budget_gib, "requests_per_load": args.requests},
        "loads": loads,
    }
    if not baseline:
        if emit:
            print(json.dumps(out), flush=True)
        return out
    # baseline: complex128, per-term energy, parameter shift, one request at a time
    base_t = []
    acc = []
    for d in insts:
        n = d["n"]
        bufs = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
        st = torch.cuda.current_stream().cuda_stream
        s = L.vqe_state_alloc(n, L.VQE_C128, bufs.data_ptr(), bufs.numel() * 16, st)
        th = draw(d)
        L.vqe_circuit_prepare(d["C"].handle, L.VQE_C128)  # kernel compilation outside the timed region
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.vqe_state_set_basis(s, 0)
        L.vqe_apply_circuit(s, d["C"].handle, th)
        E_pt, _ = L.vqe_expect_pauli(s, d["H"].handle, L.EXPECT_PER_TERM)
        t_e = time.perf_counter() - t0
        base_t.append((2 * d["C"].n_params + 1) * t_e)
        if n <= 12:   # full baseline evaluation vs the served form at small n
            Eb, gb = L.vqe_energy_grad(s, None, d["C"].handle, th, d["H"].handle, method=L.GRAD_PARAM_SHIFT,
                                       expect_mode=L.EXPECT_PER_TERM)
            b = L.vqe_batch_create(L.VQE_C64, st)
            (Es, gs), = L.vqe_batch_energy_grad(b, [(d["C"].handle, d["H"].handle, th)])
            L.vqe_batch_free(b)
            acc.append(dict(n=n, energy_rel=abs(Es - Eb) / max(abs(Eb), 1),
                            grad_rel=float(np.max(np.abs(gs - gb)) / max(np.max(np.abs(gb)), 1))))
        L.vqe_state_free(s)
        del bufs
    torch.cuda.empty_cache()
    base_rate = 1.0 / float(np.mean(base_t))
    out["baseline_per_term_param_shift_f64"] = {"evals_per_s": base_rate,
                                                "method": "one request at a time: (2P+1) x measured per-term energy time"}
    out["speedup_vs_baseline"] = cap / base_rate
    out["accuracy_vs_baseline_small"] = acc
    if emit:
        print(json.dumps(out), flush=True)
    return out


def copy_calibration(args):
    """A plain device copy of known size (8 GiB read + 8 GiB written, 3 times):
    the reference that scales the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    nbytes = 8 << 30
    a = torch.zeros(nbytes // 16, dtype=torch.complex128, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 3
    print(json.dumps({"mode": "copy", "bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes,
                      "copies": 3, "gbs": 2 * nbytes / dt / 1e9}), flush=True)


def energy_bench(args):
    """The grouped energy-only sweep (vqe_expect_pauli, eq. 7) on the state
    of the workload's ansatz at its first parameter vector, for both state
    precisions: time per energy from the library's HIP events, the bytes it
    reads in units of S (one S per window pass, or (1 + D/2) S for the tile
    sweep) and Pauli terms per second; then the per-term form of the paper's
    evaluation order (one sweep per term, S each) on the same state."""
    import torch
    import synth
    from paper_2402_11878_amd import _lib as L, core

    wl = synth.WORKLOADS[args.workload]
    n = wl.n_qubits
    (x, z, w), th_used = workload_hamiltonian(wl, args.threshold)
    H = core.Hamiltonian(n, x, z, w)
    circ = core.Circuit.layered(n, wl.layers)
    theta = wl.thetas()[0]
    out = {"mode": "energy", "workload": wl.name, "n_qubits": n, "n_terms": H.n_terms, "n_groups": H.n_groups,
           "threshold": th_used, "reps": args.reps,
           "window_passes_lam": len(L.vqe_hamiltonian_plan(H.handle))}
    for dt, dtype, tdt in (("c128", L.VQE_C128, torch.complex128), ("c64", L.VQE_C64, torch.complex64)):
        if (dt == "c128" and args.skip_c128) or (dt == "c64" and args.skip_c64):
            continue
        buf = torch.empty(1 << n, dtype=tdt, device="cuda")
        st = torch.cuda.current_stream().cuda_stream
        s = L.vqe_state_alloc(n, dtype, buf.data_ptr(), buf.numel() * buf.element_size(), st)
        S = buf.numel() * buf.element_size()
        try:
            L.vqe_state_set_basis(s, 0)
            L.vqe_apply_circuit(s, circ.handle, theta)
            E0, _ = L.vqe_expect_pauli(s, H.handle, L.EXPECT_GROUPED)
            torch.cuda.synchronize()
            L.vqe_profile_reset()
            L.vqe_profile_enable(True)
            t0 = time.perf_counter()
            for i in range(args.reps):
                E, nrm = L.vqe_expect_pauli(s, H.handle, L.EXPECT_GROUPED)
                log(f"[energy] {dt} rep {i + 1}/{args.reps} E={E:.12f}")
            t1 = time.perf_counter()
            cnt, ms, nbytes = L.vqe_profile_read(L.KERNEL_EXPECT_HALF)
            L.vqe_profile_enable(False)
            L.vqe_profile_reset()
            r = {"energy": E, "sec_per_energy": (t1 - t0) / args.reps, "kernel_ms_per_energy": ms / args.reps,
                 "launches_per_energy": cnt / args.reps, "bytes_per_energy_in_S": nbytes / args.reps / S,
                 "gbs": nbytes / (ms * 1e-3) / 1e9, "frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                 "pauli_terms_per_s": H.n_terms / ((t1 - t0) / args.reps)}
            if args.per_term:
                L.vqe_profile_enable(True)
                t0 = time.perf_counter()
                Ep, _ = L.vqe_expect_pauli(s, H.handle, L.EXPECT_PER_TERM)
                t1 = time.perf_counter()
                cnt, ms, nbytes = L.vqe_profile_read(L.KERNEL_PER_TERM)
                L.vqe_profile_enable(False)
                L.vqe_profile_reset()
                r["per_term"] = {"energy": Ep, "sec_per_energy": t1 - t0, "sweeps": cnt,
                                 "gbs": nbytes / (ms * 1e-3) / 1e9, "pauli_terms_per_s": H.n_terms / (t1 - t0)}
            out[dt] = r
            log(f"[energy] {dt}: {r['kernel_ms_per_energy']:.1f} ms per energy, {r['bytes_per_energy_in_S']:.2f} S, "
                f"{r['gbs']:.0f} GB/s")
        finally:
            L.vqe_state_free(s)
            del buf
            torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def dense_bench(args):
    """Dense window on the matrix cores against the gate-by-gate window pass,
    at 32 qubits: one 5-qubit window applied as a dense 32 x 32 unitary
    (vqe_apply_dense: FP32 MFMA on complex64, FP64 MFMA on complex128) and the
    specialised window pass of vqe_apply_circuit for a 14-gate circuit on the
    same qubits (RY and RZ on each, a CNOT chain: one pass).  Both are timed
    with the library's HIP events; both move 2 S per pass."""
    import numpy as np
    import torch
    from paper_2402_11878_amd import _lib as L, ansatz

    n, qubits = 32, [8, 9, 10, 11, 12]
    gates = [(0, q, -1, 2 * i, 0.0) for i, q in enumerate(qubits)] + \
            [(1, q, -1, 2 * i + 1, 0.0) for i, q in enumerate(qubits)] + \
            [(5, a, b, -1, 0.0) for a, b in zip(qubits, qubits[1:])]
    rng = np.random.default_rng(5)
    theta = rng.uniform(-np.pi, np.pi, 2 * len(qubits))
    a = rng.normal(size=(32, 32)) + 1j * rng.normal(size=(32, 32))
    U, _ = np.linalg.qr(a)
    out = {"mode": "dense", "n_qubits": n, "qubits": qubits, "reps": args.reps,
           "note": "per pass; algorithmic bytes 2 S; dense flops 2^(n-5) x 64 x 64 x 2 real"}
    peaks = {"c64": 157.3, "c128": 78.6}  # dense MFMA TFLOP/s: FP32, FP64
    for dt, dtype, tdt in (("c64", L.VQE_C64, torch.complex64), ("c128", L.VQE_C128, torch.complex128)):
        buf = torch.zeros(1 << n, dtype=tdt, device="cuda")
        st = torch.cuda.current_stream().cuda_stream
        s = L.vqe_state_alloc(n, dtype, buf.data_ptr(), buf.numel() * buf.element_size(), st)
        c = L.vqe_circuit_create(n, ansatz.gates_array(gates))
        try:
            L.vqe_circuit_prepare(c, dtype)
            L.vqe_state_set_basis(s, 0)
            L.vqe_apply_circuit(s, c, theta)
            L.vqe_apply_dense(s, qubits, U)
            torch.cuda.synchronize()
            L.vqe_profile_enable(1)
            L.vqe_profile_reset()
            for _ in range(args.reps):
                L.vqe_apply_circuit(s, c, theta)
            for _ in range(args.reps):
                L.vqe_apply_dense(s, qubits, U)
            torch.cuda.synchronize()
            nf, msf, bf = L.vqe_profile_read(L.KERNEL_WINDOW_FWD)
            nd, msd, bd = L.vqe_profile_read(L.KERNEL_DENSE)
            L.vqe_profile_enable(0)
            flops = float(1 << (n - 5)) * 64 * 64 * 2
            out[dt] = {"window_fwd_ms": msf / nf, "window_fwd_gbs": bf / msf / 1e6, "window_passes": nf // args.reps,
                       "dense_ms": msd / nd, "dense_gbs": bd / msd / 1e6,
                       "dense_tflops": flops / (msd / nd) / 1e9, "mfma_peak_tflops": peaks[dt]}
            log(f"[dense] {dt}: window pass {msf / nf:.2f} ms, dense MFMA {msd / nd:.2f} ms")
        finally:
            L.vqe_circuit_free(c)
            L.vqe_state_free(s)
            del buf
            torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def batch_bench(args):
    """Mid-size requests batched (vqe_batch_energy_grad: tile passes, one
    launch per pass index for every item) against the same requests one at a
    time on the per-request path (vqe_energy_grad, fused window passes),
    complex64, for 14-24 qubits and batches of 1-16 items.  Items mix layer
    counts (4-16) and Hamiltonians (Hubbard chains and molecule-shaped,
    slimmed at --slim) as the served stream does.  Optionally restricted to
    the first --reserve-cus compute units (the serving lane's stream)."""
    import numpy as np
    import torch
    import synth
    from paper_2402_11878_amd import _lib as L, ansatz, hamiltonians as hm

    sizes = [int(v) for v in args.batch_sizes.split(",")]
    qubits = [int(v) for v in args.batch_qubits.split(",")]
    if args.reserve_cus > 0 and args.batch_masked:
        raw = L.vqe_stream_create(range(args.reserve_cus))
        stream = torch.cuda.ExternalStream(raw)
    else:
        raw, stream = None, torch.cuda.current_stream()
    out = {"mode": "batch", "dtype": "c64", "reps": args.reps,
           "cus": args.reserve_cus if raw else torch.cuda.get_device_properties(0).multi_processor_count,
           "note": "evals/s = items x reps / wall time of reps calls; per_request: the same items one at a time "
                   "(vqe_energy_grad, psi and lam resident, no checkpoints)"}
    with torch.cuda.stream(stream):
        for n in qubits:
            items = []
            for i in range(max(sizes)):
                layers = 4 + (3 * i) % 13
                if i % 2 == 0:
                    lat = synth.Lattice(n // 2, tuple(synth.chain_bonds(n // 2)), 1.0, 4.0)
                    x, z, w = hm.from_lattice(lat)
                else:
                    h, g = synth.molecule_integrals(n // 2, 500 + i)
                    x, z, w = hm.molecule(h, g)
                    keep, _, _ = L.vqe_slim_hamiltonian(x, z, w, L.SLIM_THRESHOLD, args.slim)
                    k = keep.astype(bool)
                    x, z, w = x[k], z[k], w[k]
                c = L.vqe_circuit_create(n, ansatz.layered(n, layers))
                hh = L.vqe_hamiltonian_create(n, x, z, w)
                th = np.random.default_rng(700 + i).uniform(-np.pi, np.pi, 2 * n * layers)
                items.append((c, hh, th))
            res = {}
            b = L.vqe_batch_create(L.VQE_C64, stream.cuda_stream)
            try:
                for B in sizes:
                    L.vqe_batch_energy_grad(b, items[:B])           # warm-up: buffers, table uploads
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(args.reps):
                        L.vqe_batch_energy_grad(b, items[:B])
                    dt = time.perf_counter() - t0
                    res[str(B)] = {"evals_per_s": B * args.reps / dt, "ms_per_call": dt / args.reps * 1e3}
            finally:
                L.vqe_batch_free(b)
            tdt = torch.complex64
            bufs = [torch.empty(1 << n, dtype=tdt, device="cuda") for _ in range(2)]
            hs = [L.vqe_state_alloc(n, L.VQE_C64, t.data_ptr(), t.numel() * 8, stream.cuda_stream) for t in bufs]
            try:
                B = max(sizes)
                for c, hh, th in items[:B]:
                    L.vqe_circuit_prepare(c, L.VQE_C64)
                    L.vqe_energy_grad(hs[0], hs[1], c, th, hh)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.reps):
                    for c, hh, th in items[:B]:
                        L.vqe_energy_grad(hs[0], hs[1], c, th, hh)
                dt = time.perf_counter() - t0
                res["per_request"] = {"evals_per_s": B * args.reps / dt, "ms_per_eval": dt / (B * args.reps) * 1e3}
            finally:
                for h_ in hs:
                    L.vqe_state_free(h_)
                del bufs
            for c, hh, _ in items:
                L.vqe_circuit_free(c)
                L.vqe_hamiltonian_free(hh)
            out[str(n)] = res
            log(f"[batch] n={n}: {res}")
    if raw:
        torch.cuda.synchronize()
        L.vqe_stream_destroy(raw)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="hubbard4x4",
                    help="hubbard4x4 (the 32-qubit step), hubbard2x7 (28 qubits, batch of 8 vectors), "
                         "molecule_16 (32 qubits), molecule_10, hubbard1d_6")
    ap.add_argument("--threshold", type=float, default=None,
                    help="slimming threshold of molecule-shaped workloads (default: the workload's largest)")
    ap.add_argument("--skip-c64", action="store_true")
    ap.add_argument("--skip-c128", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="step", choices=["step", "serving", "copy", "dense", "energy", "batch"],
                    help="step: the 32-qubit energy+gradient step (default); serving: the served stream; "
                         "copy: a plain 8 GiB device copy (counter calibration); dense: a 5-qubit window "
                         "as a dense unitary on the matrix cores against the gate-by-gate window pass; "
                         "energy: the grouped energy-only sweep of the workload; batch: mid-size requests "
                         "batched against one at a time")
    ap.add_argument("--per-term", action="store_true", help="energy mode: also time the per-term form once")
    ap.add_argument("--specialize", default="auto", choices=["never", "auto", "always"],
                    help="kernel form of the window passes (vqe_set_specialize): interpreted 5-qubit windows "
                         "(never), specialised 7-qubit windows from 20 qubits on (auto, the default), or always")
    ap.add_argument("--instances", type=int, default=32)
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--workers", type=int, default=3, help="serving: workers for large requests")
    ap.add_argument("--mid-workers", type=int, default=1,
                    help="serving: workers of the mid-size lane (0: mid-size requests share the large workers)")
    ap.add_argument("--mid-n-max", type=int, default=20, help="serving: largest qubit count of the mid-size lane")
    ap.add_argument("--reserve-cus", type=int, default=0,
                    help="serving: compute units reserved for the batched and mid-size lanes (0: none)")
    ap.add_argument("--mid-batch", type=int, default=1,
                    help="serving: 1 = the mid-size lane launches its queued requests together (tile passes)")
    ap.add_argument("--mid-batch-n-max", type=int, default=16,
                    help="serving with --mid-batch 1: largest qubit count batched (larger mid-size requests go "
                         "to the mid-size workers; 0: all of them batched)")
    ap.add_argument("--chunk-passes", type=int, default=3,
                    help="serving: submit large evaluations in chunks of this many window passes (0: at once)")
    ap.add_argument("--batch-sizes", default="1,4,16", help="batch mode: items per call")
    ap.add_argument("--batch-qubits", default="14,16,20,24", help="batch mode: qubit counts")
    ap.add_argument("--batch-masked", type=int, default=0,
                    help="batch mode: 1 = run on a stream restricted to the first --reserve-cus compute units")
    ap.add_argument("--no-serving", action="store_true", help="step mode: skip the short serving leg")
    ap.add_argument("--budget-gib", type=float, default=160.0)
    ap.add_argument("--slim", type=float, default=1e-3)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported (the library is "
              f"single-device; sharding over several GPUs is a design, not an implemented path)", file=sys.stderr)
        sys.exit(2)
    cpu = None
    if args.mode == "step" and not args.no_cpu_baseline:
        import synth
        if synth.WORKLOADS[args.workload].kind != "molecule":
            log("[bench] cpu baseline (oracle, before the GPU is touched) ...")
            cpu = cpu_baseline(args.workload)
    import torch
    import synth
    from paper_2402_11878_amd import _lib as L, core

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    L.lib()
    L.vqe_set_specialize({"never": L.SPECIALIZE_NEVER, "auto": L.SPECIALIZE_AUTO,
                          "always": L.SPECIALIZE_ALWAYS}[args.specialize])
    if args.mode == "serving":
        serving_bench(args)
        return
    if args.mode == "copy":
        copy_calibration(args)
        return
    if args.mode == "dense":
        dense_bench(args)
        return
    if args.mode == "batch":
        batch_bench(args)
        return
    if args.mode == "energy":
        energy_bench(args)
        return
    wl = synth.WORKLOADS[args.workload]
    thetas = wl.thetas()
    res = {}
    if not args.skip_c128:
        res["c128"] = run_dtype(torch, L, core, wl, L.VQE_C128, 1, args.steps, args.warmup, thetas, args.threshold)
    if not args.skip_c64:
        res["c64"] = run_dtype(torch, L, core, wl, L.VQE_C64, 4, args.steps, args.warmup, thetas, args.threshold)
    head = res["c128"] if "c128" in res else res["c64"]

    n_rev, ms_rev, b_rev = head["prof"][L.KERNEL_WINDOW_REV]
    avg_ms = ms_rev / max(n_rev, 1)
    bytes_per_launch = b_rev / max(n_rev, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    kernels = {}
    names = {0: "window_fwd", 1: "window_rev", 2: "hpsi", 3: "expect_grouped", 4: "expect_per_term"}
    for k, (cnt, ms, b) in head["prof"].items():
        if cnt:
            kernels[names[k]] = dict(launches=cnt, avg_ms=ms / cnt, gbs=(b / cnt) / (ms / cnt * 1e-3) / 1e9,
                                     frac=(b / cnt) / (ms / cnt * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                     share=ms / (head["sec"] * 1e3 * args.steps))
    out = {
        "metric": f"VQE energy+adjoint-grad evals/s at {wl.n_qubits}q",
        "value": 1.0 / head["sec"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["sec"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head["name"] == "c128" else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{wl.name}: {WORKLOAD_TEXT.get(wl.name, wl.kind)}, {wl.n_qubits} qubits, "
                        + (f"slimmed at |w| >= {head['threshold']:g}, " if head["threshold"] is not None else "")
                        + f"{head['n_terms']} Pauli terms / {head['n_groups']} X-groups; {wl.layers}-layer RY/RZ/CNOT "
                        f"ansatz ({head['n_gates']} gates, {wl.n_params} params, seed {wl.theta_seed}"
                        + (f", {len(thetas)} parameter vectors cycled" if len(thetas) > 1 else "") + "); "
                        f"{head['name']} state, {head['n_ckpt']} checkpoint(s); energy + adjoint gradient",
            "n_qubits": wl.n_qubits,
            "state": head["name"],
            "fused_passes_adjoint": head["n_passes_adj"],
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "window_rev (reverse fused pass on psi and lam)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic() if head["name"] == "c128" else None,
            "bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": avg_ms,
        },
        "kernels": kernels,
        "gates_per_s": head["n_gates"] / head["sec"],
        "pauli_terms_per_s": head["n_terms"] / head["sec"],
        "energy": head["E"],
    }
    if "c64" in res and "c128" in res:
        a, b = res["c64"], res["c128"]
        gs = max(np.max(np.abs(b["grad"])), 1.0)
        out["c64"] = dict(value=1.0 / a["sec"], ms_per_step=a["sec"] * 1e3,
                          energy_rel_err_vs_c128=abs(a["E"] - b["E"]) / max(abs(b["E"]), 1.0),
                          grad_err_vs_c128=float(np.max(np.abs(a["grad"] - b["grad"])) / gs),
                          n_ckpt=a["n_ckpt"],
                          window_rev_frac=(a["prof"][1][2] / a["prof"][1][0]) / (a["prof"][1][1] / a["prof"][1][0] * 1e-3)
                          / 1e9 / HBM_PEAK_GBS if a["prof"][1][0] else None)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    if not args.no_serving:
        log("[bench] serving leg ...")
        sv = serving_bench(args, fracs=(0.8,), baseline=False, emit=False)
        ld = sv["loads"]["0.8"]
        out["serving"] = {"capacity_evals_per_s": sv["value"], "load": 0.8, "offered": ld["offered"],
                          "achieved_in_window": ld["achieved_in_window"], "p50_ms": ld["p50_ms"],
                          "p99_ms": ld["p99_ms"], "requests": args.requests, "config": sv["config"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
