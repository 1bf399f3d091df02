"""Dense linear algebra over GF(2) for building codes and logical operators.

Matrices are numpy uint8 arrays holding 0/1.  These routines build inputs
(check matrices and logical bases); none of the decoder's arithmetic is here.
"""
from __future__ import annotations

import numpy as np


def _as_bits(a) -> np.ndarray:
    a = np.asarray(a, dtype=np.uint8) & 1
    if a.ndim != 2:
        raise ValueError("expected a 2-D 0/1 matrix")
    return a.copy()


def row_reduce(a):
    """Reduced row echelon form over GF(2).

    Returns (R, pivots) with R of the same shape as ``a``; the first
    ``len(pivots)`` rows of R are a basis of the row space.
    """
    r = _as_bits(a)
    rows, cols = r.shape
    pivots = []
    row = 0
    for col in range(cols):
        if row >= rows:
            break
        nz = np.nonzero(r[row:, col])[0]
        if nz.size == 0:
            continue
        p = row + nz[0]
        if p != row:
            r[[row, p]] = r[[p, row]]
        mask = r[:, col].astype(bool)
        mask[row] = False
        r[mask] ^= r[row]
        pivots.append(col)
        row += 1
    return r, pivots


def rank(a) -> int:
    return len(row_reduce(a)[1])


def nullspace(a) -> np.ndarray:
    """Basis (as rows) of {x : a x = 0} over GF(2)."""
    a = _as_bits(a)
    r, piv = row_reduce(a)
    n = a.shape[1]
    free = [c for c in range(n) if c not in set(piv)]
    basis = np.zeros((len(free), n), dtype=np.uint8)
    for k, f in enumerate(free):
        basis[k, f] = 1
        for i, pc in enumerate(piv):
            if r[i, f]:
                basis[k, pc] = 1
    return basis


def in_rowspace(a, v) -> bool:
    return rank(np.vstack([_as_bits(a), np.asarray(v, np.uint8)[None, :] & 1])) == rank(a)


def complement_basis(sub, sup) -> np.ndarray:
    """Rows of ``sup`` (greedily chosen) completing rowspace(sub) to rowspace(sup).

    The returned rows are independent modulo rowspace(sub).
    """
    sub = _as_bits(sub)
    sup = _as_bits(sup)
    basis, piv = row_reduce(sub)
    cur = basis[: len(piv)]
    r0 = len(piv)
    chosen = []
    for v in sup:
        trial = np.vstack([cur, v[None, :]])
        if rank(trial) > r0 + len(chosen):
            chosen.append(v.copy())
            cur = trial
    if not chosen:
        return np.zeros((0, sup.shape[1]), dtype=np.uint8)
    return np.array(chosen, dtype=np.uint8)
