"""The seeded input generators: codes, the space-time graph and the sampler."""
from __future__ import annotations

import numpy as np
import pytest

from bsd_inputs import codes, gf2, sampler, workloads


@pytest.mark.parametrize("l,m,n,rank", [(6, 6, 72, 30), (6, 12, 144, 66)])
def test_bb_codes(l, m, n, rank):
    hx, hz = codes.bb_matrices(l, m)
    assert hx.shape == (n // 2, n) and hz.shape == (n // 2, n)
    assert ((hx.astype(int) @ hz.T.astype(int)) % 2 == 0).all()
    assert gf2.rank(hx) == rank and gf2.rank(hz) == rank
    assert (hx.sum(1) == 6).all() and (hx.sum(0) == 3).all()
    L = codes.x_logicals(hx, hz)
    assert L.shape == (n - 2 * rank, n) == (12, n)
    # logical rows commute with Z stabilizers and are independent of X stabilizers
    assert ((L.astype(int) @ hz.T.astype(int)) % 2 == 0).all()
    assert gf2.rank(np.vstack([hx, L])) == rank + 12


def test_spacetime_graph_structure():
    pr = workloads.problem("bb144_st12")
    kind = pr.meta["kind"]
    assert pr.m == 13 * 72 and pr.n == 1728 + 864 + 6000
    assert (kind == 0).sum() == 1728 and (kind == 1).sum() == 864 and (kind == 2).sum() == 6000
    deg = pr.col_degrees()
    assert (deg[kind == 0] == 3).all() and (deg[kind == 1] == 2).all()
    assert ((deg[kind == 2] >= 4) & (deg[kind == 2] <= 6)).all()
    cols = set()
    for j in range(pr.n):
        rows = pr.rowidx[pr.colptr[j]:pr.colptr[j + 1]]
        assert (np.diff(rows) > 0).all()
        layers = rows // 72
        if kind[j] == 2:
            assert layers.max() - layers.min() == 1
        cols.add(tuple(rows))
    assert len(cols) == pr.n
    assert (pr.p >= 1e-5).all() and (pr.p <= 1e-3).all()
    assert workloads.problem_digest(pr) == workloads.problem_digest(codes.bb_spacetime(6, 12, name="x"))


def test_sampler_rates_and_prefix():
    p = np.array([0.5, 0.1, 0.01, 0.3])
    shot, col = sampler.sample_faults(p, 20000, seed=3)
    counts = np.bincount(col, minlength=4) / 20000
    assert np.all(np.abs(counts - p) < 5 * np.sqrt(p * (1 - p) / 20000))
    s2, c2 = sampler.sample_faults(p, 5000, seed=3)
    keep = shot < 5000
    assert np.array_equal(shot[keep], s2) and np.array_equal(col[keep], c2)
    s3, c3 = sampler.sample_faults(p, 5000, seed=4)
    assert not (len(s3) == len(s2) and np.array_equal(s3, s2) and np.array_equal(c3, c2))
    # independence across columns: pairwise coincidence rate ~ p_a p_b
    e = sampler.dense_errors(type("P", (), {"n": 4})(), shot, col, 20000)
    both = (e[:, 0] & e[:, 3]).mean()
    assert abs(both - 0.15) < 0.02


def test_syndromes_are_He():
    pr = workloads.problem("bb72_cc_p0.03")
    d = sampler.sample(pr, 300, seed=1)
    e = sampler.dense_errors(pr, d["fault_shot"], d["fault_col"], 300)
    H = pr.dense_H()
    assert np.array_equal(d["syndromes"], (e.astype(int) @ H.T.astype(int)) % 2)
    assert np.array_equal(d["true_flips"], (e.astype(int) @ pr.L.T.astype(int)) % 2)


@pytest.mark.parametrize("l,m", [(6, 6), (6, 12)])
def test_xyz_problem_structure(l, m):
    """Depolarizing XYZ problem: a Y fault is an X and a Z fault on the same
    qubit; stabilizers are undetected and logically trivial; logical
    operators are undetected and flip a logical row."""
    pr = codes.bb_xyz(l, m, 0.06)
    hx, hz = codes.bb_matrices(l, m)
    nq = hx.shape[1]
    h = np.zeros((pr.m, pr.n), np.uint8)
    for j in range(pr.n):
        h[pr.rowidx[pr.colptr[j]:pr.colptr[j + 1]], j] = 1
    X, Z, Y = h[:, :nq], h[:, nq:2 * nq], h[:, 2 * nq:]
    assert ((X ^ Z) == Y).all()
    assert (X[:hx.shape[0]] == 0).all() and (Z[hx.shape[0]:] == 0).all()
    np.testing.assert_array_equal(Z[:hx.shape[0]], hx)
    np.testing.assert_array_equal(X[hx.shape[0]:], hz)
    Lx, Lz, Ly = pr.L[:, :nq], pr.L[:, nq:2 * nq], pr.L[:, 2 * nq:]
    assert ((Lx ^ Lz) == Ly).all() and pr.L.shape[0] == 24 == gf2.rank(pr.L)
    np.testing.assert_allclose(pr.p, 0.02)
    # stabilizer generators as errors: X-type (rows of H_X) in the X block,
    # Z-type (rows of H_Z) in the Z block
    for stab, block in ((hx, 0), (hz, 1)):
        for r in stab[:5]:
            e = np.zeros(pr.n, np.uint8)
            e[block * nq:(block + 1) * nq] = r
            assert not ((h.astype(int) @ e) % 2).any()
            assert not ((pr.L.astype(int) @ e) % 2).any()
    # logical operators as errors: undetected, nontrivial
    for lg, block in ((codes.x_logicals(hx, hz), 0), (codes.x_logicals(hz, hx), 1)):
        for r in lg:
            e = np.zeros(pr.n, np.uint8)
            e[block * nq:(block + 1) * nq] = r
            assert not ((h.astype(int) @ e) % 2).any()
            assert ((pr.L.astype(int) @ e) % 2).any()
