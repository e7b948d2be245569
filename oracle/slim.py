"""Hamiltonian cutoff ("slimming"), oracle side (Sec. II-D and III-D).

The paper sorts the Jordan-Wigner terms by |w| and drops those below a
threshold Th1; the justification is -|w| <= <psi|wP|psi> <= |w| for a
normalised state, so the energy error is at most the sum of the dropped |w|.

Readings used here:
  * threshold mode: keep a term iff |w| >= Th (only |w| < Th is dropped);
  * remove-percent mode: the "cutoff ratio" is the percentage of terms
    removed; sort the non-identity terms by (|w| descending, x ascending,
    z ascending) and drop the last floor(N * pct / 100);
  * budget mode: walk that order from its end, adding |w| into an FP64 running
    sum left to right; drop while the sum stays <= budget and stop at the first
    term that would exceed it.
  * keep-top mode (Algorithm 1's "top N x ratio terms"): keep the first K
    non-identity terms of that order, K = floor(N x ratio) given as a count.
In every mode the identity term (x = z = 0) is kept: it costs no sweep and is
a constant shift.  Each mode returns (keep mask, dropped sum of |w|), the
dropped sum being accumulated in the order the terms are dropped.
"""
from __future__ import annotations

import math

import numpy as np


def _order(x, z, w):
    """Indices of non-identity terms, most important first."""
    idx = [i for i in range(len(w)) if not (int(x[i]) == 0 and int(z[i]) == 0)]
    idx.sort(key=lambda i: (-abs(float(w[i])), int(x[i]), int(z[i])))
    return idx


def threshold(x, z, w, th):
    keep = np.ones(len(w), dtype=np.uint8)
    dropped = 0.0
    for i in range(len(w)):
        if int(x[i]) == 0 and int(z[i]) == 0:
            continue
        if abs(float(w[i])) < th:
            keep[i] = 0
    # dropped sum in the canonical drop order (smallest first)
    for i in reversed(_order(x, z, w)):
        if keep[i] == 0:
            dropped += abs(float(w[i]))
    return keep, dropped


def remove_percent(x, z, w, pct):
    order = _order(x, z, w)
    n_drop = (len(order) * int(pct)) // 100
    keep = np.ones(len(w), dtype=np.uint8)
    dropped = 0.0
    for i in reversed(order[len(order) - n_drop:]):
        keep[i] = 0
        dropped += abs(float(w[i]))
    return keep, dropped


def keep_top(x, z, w, count):
    order = _order(x, z, w)
    keep = np.ones(len(w), dtype=np.uint8)
    dropped = 0.0
    for i in reversed(order[int(count):]):
        keep[i] = 0
        dropped += abs(float(w[i]))
    return keep, dropped


def budget(x, z, w, limit):
    order = _order(x, z, w)
    keep = np.ones(len(w), dtype=np.uint8)
    s = 0.0
    for i in reversed(order):
        nxt = s + abs(float(w[i]))
        if nxt > limit:
            break
        s = nxt
        keep[i] = 0
    return keep, s


def dropped_bound_check(E_full, E_slim, dropped):
    """|E_full - E_slim| <= sum of dropped |w| (normalised state)."""
    return abs(E_full - E_slim) <= dropped * (1 + 1e-12) + 1e-15 * max(1.0, abs(E_full))


def fsum_abs(w):
    return math.fsum(abs(float(v)) for v in w)
