"""Decoding problems (H, A, p) of the kind the decoder is evaluated on.

A decoding problem is a check matrix H (M detectors x N fault columns), a
logical matrix A (K x N) and per-column fault probabilities p (Appendix A of
the paper).  This module builds:

* bivariate bicycle (BB) codes from two polynomials in x = S_l (x) I_m and
  y = I_l (x) S_m, with H_X = [A | B], H_Z = [B^T | A^T] (the [[72,12,6]] and
  [[144,12,12]] codes used for code-capacity noise);
* the logical matrix for Z errors decoded with H_X: a basis of ker(H_Z)
  modulo rowspace(H_X) (X-type logical operators);
* a synthetic space-time detector graph of a BB code over several noisy
  syndrome rounds (data, measurement and hook fault columns) that stands in
  for the circuit-level detector error model, which is not available here.

Everything is seeded and deterministic; nothing here runs the decoder.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import gf2


@dataclass
class Problem:
    """A decoding problem in compressed sparse column form.

    colptr/rowidx: CSC of H (int32), rows ascending within a column.
    L: dense K x N uint8 logical matrix.  p: float64 priors, 0 < p_j < 1.
    """

    name: str
    m: int
    n: int
    colptr: np.ndarray
    rowidx: np.ndarray
    L: np.ndarray
    p: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def k(self) -> int:
        return int(self.L.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])

    def dense_H(self) -> np.ndarray:
        h = np.zeros((self.m, self.n), dtype=np.uint8)
        for j in range(self.n):
            h[self.rowidx[self.colptr[j]:self.colptr[j + 1]], j] = 1
        return h

    def L_csc(self):
        cols = [np.nonzero(self.L[:, j])[0] for j in range(self.n)]
        ptr = np.zeros(self.n + 1, dtype=np.int32)
        ptr[1:] = np.cumsum([len(c) for c in cols])
        idx = np.concatenate(cols).astype(np.int32) if ptr[-1] else np.zeros(0, np.int32)
        return ptr, idx

    def row_degrees(self) -> np.ndarray:
        return np.bincount(self.rowidx, minlength=self.m)

    def col_degrees(self) -> np.ndarray:
        return np.diff(self.colptr)


def csc_from_dense(h) -> tuple[np.ndarray, np.ndarray]:
    h = np.asarray(h, dtype=np.uint8)
    cols = [np.nonzero(h[:, j])[0] for j in range(h.shape[1])]
    ptr = np.zeros(h.shape[1] + 1, dtype=np.int32)
    ptr[1:] = np.cumsum([len(c) for c in cols])
    idx = np.concatenate(cols).astype(np.int32) if ptr[-1] else np.zeros(0, np.int32)
    return ptr, idx


def csc_from_columns(m: int, columns) -> tuple[np.ndarray, np.ndarray]:
    ptr = np.zeros(len(columns) + 1, dtype=np.int32)
    ptr[1:] = np.cumsum([len(c) for c in columns])
    idx = np.concatenate([np.sort(np.asarray(c, np.int64)) for c in columns]).astype(np.int32)
    if idx.size and (idx.min() < 0 or idx.max() >= m):
        raise ValueError("row index out of range")
    return ptr, idx


def problem_from_dense(name, h, L, p, meta=None) -> Problem:
    h = np.asarray(h, dtype=np.uint8) & 1
    ptr, idx = csc_from_dense(h)
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), (h.shape[1],)).copy()
    L = np.asarray(L, dtype=np.uint8).reshape(-1, h.shape[1]) & 1
    return Problem(name, h.shape[0], h.shape[1], ptr, idx, L, p, dict(meta or {}))


# --------------------------------------------------------------------------
# Bivariate bicycle codes
# --------------------------------------------------------------------------

def _shift(n: int) -> np.ndarray:
    return np.roll(np.eye(n, dtype=np.uint8), 1, axis=1)


def bb_matrices(l: int, m: int, a_terms=(("x", 3), ("y", 1), ("y", 2)),
                b_terms=(("y", 3), ("x", 1), ("x", 2))):
    """H_X = [A|B], H_Z = [B^T|A^T] for A, B sums of powers of x and y."""
    x = np.kron(_shift(l), np.eye(m, dtype=np.uint8)).astype(np.int64)
    y = np.kron(np.eye(l, dtype=np.uint8), _shift(m)).astype(np.int64)
    base = {"x": x, "y": y}

    def poly(terms):
        acc = np.zeros((l * m, l * m), dtype=np.int64)
        for var, power in terms:
            acc += np.linalg.matrix_power(base[var], power)
        return (acc % 2).astype(np.uint8)

    a = poly(a_terms)
    b = poly(b_terms)
    hx = np.hstack([a, b])
    hz = np.hstack([b.T, a.T])
    return hx, hz


def x_logicals(hx, hz) -> np.ndarray:
    """Basis of ker(H_Z) modulo rowspace(H_X): detects Z-type logical errors."""
    ker = gf2.nullspace(hz)
    return gf2.complement_basis(hx, ker)


def bb_code_capacity(l: int, m: int, p: float, name: str | None = None) -> Problem:
    """Z errors on the data qubits of a BB code, decoded with H_X."""
    hx, hz = bb_matrices(l, m)
    L = x_logicals(hx, hz)
    n = hx.shape[1]
    return problem_from_dense(name or f"bb{n}_cc", hx, L, np.full(n, p),
                              meta={"l": l, "m": m, "hz": hz})


def bb_xyz(l: int, m: int, p: float, name: str | None = None) -> Problem:
    """Depolarizing code-capacity problem of a BB code decoded over X, Y and Z
    faults together.

    Rows: the X checks (rows of H_X, which see Z and Y) then the Z checks (rows
    of H_Z, which see X and Y).  Columns in three blocks [X faults | Z faults |
    Y faults] of the data qubits; a Y column is the sum of the X and Z columns
    of its qubit, which puts length-4 cycles into the Tanner graph.  Each
    fault has probability p/3.  Logical rows: the Z-type logicals (they see the
    X part of an error) then the X-type logicals (they see the Z part).
    """
    hx, hz = bb_matrices(l, m)
    nq = hx.shape[1]
    mx, mz = hx.shape[0], hz.shape[0]
    zeros_x = np.zeros((mx, nq), np.uint8)
    zeros_z = np.zeros((mz, nq), np.uint8)
    h = np.vstack([np.hstack([zeros_x, hx, hx]),      # X checks: Z and Y faults
                   np.hstack([hz, zeros_z, hz])])     # Z checks: X and Y faults
    lz = x_logicals(hz, hx)   # ker(H_X) mod rowspace(H_Z): see X parts
    lx = x_logicals(hx, hz)   # ker(H_Z) mod rowspace(H_X): see Z parts
    L = np.vstack([np.hstack([lz, np.zeros_like(lz), lz]),
                   np.hstack([np.zeros_like(lx), lx, lx])])
    return problem_from_dense(name or f"bb{nq}_xyz", h, L, np.full(3 * nq, p / 3.0),
                              meta={"l": l, "m": m, "kind": "xyz", "hx": hx, "hz": hz,
                                    "qubits": nq})


# --------------------------------------------------------------------------
# Synthetic space-time graph of a BB code (stand-in for a circuit-level DEM)
# --------------------------------------------------------------------------

def bb_spacetime(l: int = 6, m: int = 12, rounds: int = 12, hooks: int = 6000,
                 p_lo: float = 1e-5, p_hi: float = 1e-3, seed: int = 0,
                 name: str | None = None) -> Problem:
    """Phenomenological space-time graph plus random hook columns.

    Detector layers 0..rounds (rounds noisy layers and a final perfect
    read-out layer) of the X checks.  Columns:
      data (r, q):         rows r*mx + c for the checks c of qubit q; logical column L[:, q]
      measurement (r, c):  rows r*mx + c and (r+1)*mx + c; no logical effect
      hook h:              w ~ U{4,5,6} distinct rows from layers r and r+1, at least one
                           in each, r ~ U{0..rounds-1}; logical column L[:, q_h], q_h ~ U
    Priors are log-uniform in [p_lo, p_hi].  Duplicate columns are resampled.
    """
    hx, hz = bb_matrices(l, m)
    L0 = x_logicals(hx, hz)
    mx, nq = hx.shape
    nlayers = rounds + 1
    M = mx * nlayers
    rng = np.random.Generator(np.random.PCG64(seed))

    cols: list[tuple[int, ...]] = []
    lcols: list[np.ndarray] = []
    kind: list[int] = []
    checks_of_q = [np.nonzero(hx[:, q])[0] for q in range(nq)]
    for r in range(rounds):
        for q in range(nq):
            cols.append(tuple(int(r * mx + c) for c in checks_of_q[q]))
            lcols.append(L0[:, q])
            kind.append(0)
    for r in range(rounds):
        for c in range(mx):
            cols.append((r * mx + c, (r + 1) * mx + c))
            lcols.append(np.zeros(L0.shape[0], np.uint8))
            kind.append(1)
    seen = set(cols)
    made = 0
    while made < hooks:
        r = int(rng.integers(0, rounds))
        w = int(rng.integers(4, 7))
        rows = rng.choice(2 * mx, size=w, replace=False)
        lo = rows < mx
        if lo.all() or (~lo).all():
            continue
        col = tuple(sorted(int(r * mx + x) for x in rows))
        if col in seen:
            continue
        q = int(rng.integers(0, nq))
        seen.add(col)
        cols.append(col)
        lcols.append(L0[:, q])
        kind.append(2)
        made += 1
    n = len(cols)
    ptr, idx = csc_from_columns(M, cols)
    L = np.stack(lcols, axis=1).astype(np.uint8)
    p = 10.0 ** rng.uniform(np.log10(p_lo), np.log10(p_hi), size=n)
    return Problem(name or f"bb{nq}_st{rounds}", M, n, ptr, idx, L, p,
                   meta={"l": l, "m": m, "rounds": rounds, "hooks": hooks, "seed": seed,
                         "kind": np.asarray(kind, np.int8)})


# --------------------------------------------------------------------------
# Small graphs for tests
# --------------------------------------------------------------------------

def random_tree_problem(n_checks: int, seed: int, max_leaf_vars: int = 2,
                        p_lo: float = 0.02, p_hi: float = 0.3) -> Problem:
    """A random cycle-free Tanner graph; every check has degree >= 2.

    Built by growing a bipartite tree: each new check attaches to one existing
    variable and brings 1..max_leaf_vars fresh variables.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    cols: list[list[int]] = [[]]
    for i in range(n_checks):
        anchor = int(rng.integers(0, len(cols)))
        cols[anchor].append(i)
        for _ in range(int(rng.integers(1, max_leaf_vars + 1))):
            cols.append([i])
    n = len(cols)
    if any(len(c) == 0 for c in cols):
        cols = [c for c in cols if c]
        n = len(cols)
    ptr, idx = csc_from_columns(n_checks, cols)
    p = rng.uniform(p_lo, p_hi, size=n)
    L = np.zeros((1, n), np.uint8)
    return Problem(f"tree{n_checks}_{seed}", n_checks, n, ptr, idx, L, p)


def random_ldpc_problem(m: int, n: int, col_weight: int, seed: int, p=0.05,
                        k_logicals: int = 2) -> Problem:
    """Random sparse H with fixed column weight; random logical rows (tests only)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cols = [sorted(rng.choice(m, size=col_weight, replace=False).tolist()) for _ in range(n)]
    ptr, idx = csc_from_columns(m, cols)
    L = rng.integers(0, 2, size=(k_logicals, n)).astype(np.uint8)
    pv = np.broadcast_to(np.asarray(p, dtype=np.float64), (n,)).copy()
    return Problem(f"ldpc{m}x{n}_{seed}", m, n, ptr, idx, L, pv)
