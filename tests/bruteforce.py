"""Exhaustive references on tiny decoding problems (test helpers).

These enumerate all 2^n error vectors; they implement the decoding problem's
definitions (Appendix A: He = s; Appendix B: wt(e) = sum_j e_j log((1-p_j)/p_j))
and never call BP.
"""
from __future__ import annotations

import numpy as np


def all_vectors(n: int) -> np.ndarray:
    idx = np.arange(1 << n, dtype=np.int64)
    return ((idx[:, None] >> np.arange(n)) & 1).astype(np.uint8)


def weights(p) -> np.ndarray:
    p = np.asarray(p, dtype=np.float64)
    return np.log((1.0 - p) / p)


def feasible(H, s, ev=None):
    H = np.asarray(H, dtype=np.int64)
    if ev is None:
        ev = all_vectors(H.shape[1])
    syn = (ev.astype(np.int64) @ H.T) & 1
    return ev[(syn == np.asarray(s, np.int64)[None, :]).all(1)]


def max_marginals(H, s, p, fixed=None):
    """min_{He=s, e_j=1} wt(e) - min_{He=s, e_j=0} wt(e) for every j.

    ``fixed`` maps columns to forced values.  Entries are +-inf where one side
    is infeasible and nan where both are.
    """
    H = np.asarray(H)
    n = H.shape[1]
    ev = feasible(H, s)
    if fixed:
        keep = np.ones(len(ev), bool)
        for j, v in fixed.items():
            keep &= ev[:, j] == v
        ev = ev[keep]
    w = ev.astype(np.float64) @ weights(p)
    out = np.empty(n)
    for j in range(n):
        one = w[ev[:, j] == 1]
        zero = w[ev[:, j] == 0]
        a = one.min() if one.size else np.inf
        b = zero.min() if zero.size else np.inf
        out[j] = np.nan if (np.isinf(a) and np.isinf(b)) else a - b
    return out


def min_weight_solution(H, s, p):
    """(weight, vector) of a minimum-weight e with He = s, or (inf, None)."""
    ev = feasible(H, s)
    if not len(ev):
        return np.inf, None
    w = ev.astype(np.float64) @ weights(p)
    k = int(np.argmin(w))
    return float(w[k]), ev[k]


def in_colspace(H, s) -> bool:
    return len(feasible(H, s)) > 0
