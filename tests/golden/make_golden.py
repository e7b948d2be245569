"""Writes stored expected values for the GPU parity tests, computed by the
CPU oracle only (oracle/ and the seeded inputs in synth/; nothing from the
GPU path).

  molecule_10.json   20-qubit molecule-shaped Hamiltonian (10 orbitals,
                     integral seed 0), 8-layer ansatz, angles seed 0: for each
                     cutoff threshold the kept term and X-group counts and the
                     energy (term by term); at threshold 0 and 1e-3 the full
                     adjoint gradient, with parameter shift on 2 seeded indices
                     at 1e-3 as a cross-check.
  hubbard2x7_v0.json 28-qubit 2x7 Hubbard (periodic long axis, t=1, U=8),
                     16 layers, angle batch seed 1, vector 0: the energy.
  hubbard2x6_grad.json, hubbard1d_13_grad.json
                     24-qubit 2x6 Hubbard (8 layers) and 26-qubit 13-site
                     chain (4 layers) at generic angles: the energy, the full
                     adjoint gradient and parameter shift on 2 seeded indices.

Usage: python tests/golden/make_golden.py [molecule_10|hubbard2x7_v0|hubbard2x6_grad|hubbard1d_13_grad]
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import expect, grad, hamiltonian as ham, slim, statevector as sv  # noqa: E402


def molecule_10():
    wl = synth.WORKLOADS["molecule_10"]
    n = wl.n_qubits
    t0 = time.time()
    h, g = synth.molecule_integrals(wl.n_orb, wl.integral_seed)
    H = ham.molecule(h, g)
    x, z, w = ham.to_masks(H)
    print(f"JW: {len(w)} terms in {time.time() - t0:.1f} s", flush=True)
    gates = sv.layered_ansatz(n, wl.layers)
    th = wl.thetas()[0]
    psi = sv.run(n, gates, th)
    out = {"workload": wl.name, "n_qubits": n, "layers": wl.layers, "n_terms_full": int(len(w)),
           "identity": float(w[(x == 0) & (z == 0)].sum()), "thresholds": {}}
    for th1 in wl.thresholds:
        keep, dropped = slim.threshold(x, z, w, th1)
        k = keep == 1
        E, norm = expect.energy_masks(psi, n, x[k], z[k], w[k])
        out["thresholds"][repr(th1)] = {"n_terms": int(k.sum()), "n_groups": int(len(set(x[k].tolist()))),
                                        "dropped_abs_sum": dropped, "energy": E}
        print(f"Th={th1}: {int(k.sum())} terms, E={E:.15f} ({time.time() - t0:.0f} s)", flush=True)
    for th1 in (0.0, 1e-3):
        keep, _ = slim.threshold(x, z, w, th1)
        k = keep == 1
        Hk = ham.from_masks(n, x[k], z[k], w[k])
        E, gr = grad.adjoint(n, gates, th, Hk)
        ps = {}
        if th1 > 0:
            idx = sorted(np.random.default_rng(99).choice(len(th), size=2, replace=False).tolist())
            ps = grad.param_shift(n, gates, th, Hk, indices=idx)
        out["thresholds"][repr(th1)]["adjoint_energy"] = E
        out["thresholds"][repr(th1)]["grad"] = gr.tolist()
        out["thresholds"][repr(th1)]["param_shift"] = {str(i): v for i, v in ps.items()}
        print(f"grad Th={th1} done ({time.time() - t0:.0f} s); max |adj-ps| "
              f"{max([abs(gr[i] - v) for i, v in ps.items()] + [0.0]):.2e}", flush=True)
    return out


def hubbard2x7_v0():
    wl = synth.WORKLOADS["hubbard2x7"]
    n = wl.n_qubits
    lat = wl.lattice
    t0 = time.time()
    H = ham.hubbard(lat.n_sites, list(lat.bonds), lat.t, lat.U)
    gates = sv.layered_ansatz(n, wl.layers)
    th = wl.thetas()[0]
    psi = sv.basis_state(n)
    for i, gt in enumerate(gates):
        sv.apply_gate(psi, n, gt, th)
        if i % 50 == 0:
            print(f"gate {i}/{len(gates)} ({time.time() - t0:.0f} s)", flush=True)
    E, norm = expect.energy(psi, n, H, route="masks")
    print(f"E={E:.15f} norm={norm:.15f} ({time.time() - t0:.0f} s)", flush=True)
    return {"workload": wl.name, "n_qubits": n, "layers": wl.layers, "theta_seed": wl.theta_seed,
            "vector": 0, "n_terms": len(H), "energy": E, "norm": norm}


def _lattice_grad(name):
    """Energy, full adjoint gradient and parameter shift on 2 seeded indices."""
    wl = synth.WORKLOADS[name]
    n = wl.n_qubits
    lat = wl.lattice
    t0 = time.time()
    H = ham.hubbard(lat.n_sites, list(lat.bonds), lat.t, lat.U)
    gates = sv.layered_ansatz(n, wl.layers)
    th = wl.thetas()[0]
    E, gr = grad.adjoint(n, gates, th, H)
    print(f"{name}: E={E:.15f}, adjoint done ({time.time() - t0:.0f} s)", flush=True)
    idx = sorted(np.random.default_rng(7).choice(len(th), size=2, replace=False).tolist())
    ps = grad.param_shift(n, gates, th, H, indices=idx)
    print(f"{name}: parameter shift on {idx} ({time.time() - t0:.0f} s); max |adj-ps| "
          f"{max(abs(gr[i] - v) for i, v in ps.items()):.2e}", flush=True)
    return {"workload": name, "n_qubits": n, "layers": wl.layers, "theta_seed": wl.theta_seed,
            "n_terms": len(H), "energy": E, "grad": gr.tolist(),
            "param_shift": {str(i): v for i, v in ps.items()}}


def hubbard2x6_grad():
    return _lattice_grad("hubbard2x6")


def hubbard1d_13_grad():
    return _lattice_grad("hubbard1d_13")


if __name__ == "__main__":
    which = sys.argv[1:] or ["molecule_10", "hubbard2x7_v0"]
    for name in which:
        res = globals()[name]()
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(res, f, indent=1)
        print(f"wrote {name}.json", flush=True)
