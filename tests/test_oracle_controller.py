"""Pins of the oracle's beam controller (Algorithm 3, Appendix B).

The per-run arithmetic is pinned elsewhere (tree max-marginals, punctured
graphs, warm starts, closed forms).  These tests pin the control flow around
it: the order in which paths are explored (descending score, Appendix B),
the bounded on-the-fly insertion into next_set (insert while there is room,
afterwards only with a strictly greater score, ejecting the smallest), the
return of the first converging child, and the output when nothing converges.

They compare the oracle with ``beam_reference.beam_decode``, a restatement of
the controller that keeps next_set as the text describes it (a list with
insertions and ejections, not a sort), on tiny codes whose beams prune, tie
and fail, and they check that every case the comparison relies on actually
occurs.
"""
from __future__ import annotations

import numpy as np
import pytest

from bsd_inputs import codes
import beam_reference as ref
import bruteforce as bf


def _syn(H, e):
    return ((np.asarray(H, np.int64) @ np.asarray(e, np.int64)) & 1).astype(np.uint8)


def _tiny(seed, m, n, uniform):
    rng = np.random.default_rng(seed)
    while True:
        H = (rng.random((m, n)) < 0.35).astype(np.uint8)
        if H.sum(0).min() >= 1 and H.sum(1).min() >= 2:
            break
    p = np.full(n, 0.1) if uniform else rng.uniform(0.03, 0.3, size=n)
    L = rng.integers(0, 2, size=(2, n)).astype(np.uint8)
    return H, p, L


def _syndromes(H, rng, count):
    """A mix of syndromes: random errors of weight 2-4 (mostly decodable, BP
    often fails at first) and random vectors (often outside the column space)."""
    m, n = H.shape
    out = []
    for q in range(count):
        if q % 3 == 2:
            out.append(rng.integers(0, 2, size=m).astype(np.uint8))
        else:
            e = np.zeros(n, np.uint8)
            e[rng.choice(n, size=int(rng.integers(2, 5)), replace=False)] = 1
            out.append(_syn(H, e))
    return np.array(out)


# (max_rounds, beam_width, initial_iters, iters_per_round, num_results)
PARAMS = [(3, 1, 1, 1, 1), (4, 2, 1, 1, 1), (5, 3, 2, 1, 1), (6, 1, 1, 2, 1),
          (4, 2, 1, 1, 3), (8, 2, 1, 1, 1)]


def _compare(op, syn, P, dtype, stats):
    max_rounds, bw, it0, itr, nres = P
    dec = op.decode(syn, max_rounds, bw, it0, itr, num_results=nres, dtype=dtype, threads=1)
    for q, s in enumerate(syn):
        trace = []
        e, conv, info = ref.beam_decode(op, s, max_rounds, bw, it0, itr, num_results=nres,
                                        dtype=dtype, trace=trace)
        ctx = (P, q)
        assert dec["converged"][q] == int(conv), ctx
        np.testing.assert_array_equal(dec["corrections"][q], e, err_msg=str(ctx))
        dg = dec["diag"][q]
        assert dg["runs"] == info["runs"], ctx
        if conv:
            assert (dg["winner_round"], dg["winner_gen"]) == (info["round"], info["gen"]), ctx
        # which situations the comparison covered
        for rd in trace:
            sc = [s for _, s in rd["children"]]
            if len(sc) > bw:
                stats["pruned"] += 1
                srt = sorted(sc, reverse=True)
                if srt[bw - 1] == srt[bw]:
                    stats["tie_at_cut"] += 1
            ex = [s for _, s in rd["explored"]]
            if len(set(ex)) > 1:
                stats["reordered"] += 1
            if len(set(ex)) < len(ex):
                stats["tie_explore"] = stats.get("tie_explore", 0) + 1
        if conv and info["round"] > 0:
            stats["won_in_round"] += 1
            if info["gen"] > 1:
                stats["won_late_gen"] += 1
        if not conv and max_rounds > 0 and len(trace) == max_rounds and trace[-1]["kept"]:
            stats["failed_with_set"] += 1


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_controller_matches_literal_appendix_b_on_tiny_codes(oracle_mod, dtype):
    """Algorithm 3 / Appendix B: the oracle's decode equals the literal
    restatement (descending-score exploration, v = 0 then 1, strict-'>'
    bounded insertion ejecting the smallest, first converging child
    returned, best remaining path on failure) on every shot, including the
    round and generation of the winner and the number of BP runs."""
    stats = dict(pruned=0, tie_at_cut=0, reordered=0, won_in_round=0, won_late_gen=0,
                 failed_with_set=0)
    for seed in range(6):
        rng = np.random.default_rng(1000 + seed)
        m, n = 6 + seed % 3, 10 + seed % 4
        H, p, L = _tiny(seed, m, n, uniform=(seed % 2 == 1))
        ptr, idx = codes.csc_from_dense(H)
        op = oracle_mod.OracleProblem(m, n, ptr, idx, p, L)
        syn = _syndromes(H, rng, 24)
        for P in PARAMS:
            _compare(op, syn, P, dtype, stats)
    # every behaviour the pin is about was exercised
    assert stats["pruned"] > 50, stats
    assert stats["reordered"] > 50, stats
    assert stats["won_in_round"] > 20, stats
    assert stats["won_late_gen"] > 5, stats
    assert stats["failed_with_set"] > 20, stats


def test_ties_on_a_symmetric_code(oracle_mod):
    """Appendix B with exact score ties.  Two identical disjoint copies of a
    code, uniform priors and a syndrome equal on both copies: a path fixing
    (a, 0), (b, 1) and its mirror image fixing (a, 1), (b, 0) get the same
    score bit for bit (each copy's |sum_LLR| fills one aligned half of the
    score's summation tree).  At the pruning cut a child whose score only
    equals the smallest kept one is not inserted (strict '>'), so the
    earlier generated stays; equal exploration scores go in generation
    order.  With iters_per_round = 0 every child scores 0 and the whole
    beam is decided by these two rules."""
    stats = dict(pruned=0, tie_at_cut=0, reordered=0, won_in_round=0, won_late_gen=0,
                 failed_with_set=0, tie_explore=0)
    for seed in range(4):
        rng = np.random.default_rng(300 + seed)
        while True:
            B = (rng.random((4, 8)) < 0.4).astype(np.uint8)
            if B.sum(0).min() >= 1 and B.sum(1).min() >= 2:
                break
        H = np.zeros((8, 16), np.uint8)
        H[:4, :8] = B
        H[4:, 8:] = B
        ptr, idx = codes.csc_from_dense(H)
        L = np.zeros((1, 16), np.uint8)
        L[0, ::3] = 1
        op = oracle_mod.OracleProblem(8, 16, ptr, idx, np.full(16, 0.1), L)
        syn = []
        for q in range(16):
            e = np.zeros(8, np.uint8)
            e[rng.choice(8, size=int(rng.integers(1, 4)), replace=False)] = 1
            s0 = _syn(B, e) if q % 4 else rng.integers(0, 2, size=4).astype(np.uint8)
            syn.append(np.concatenate([s0, s0]))
        syn = np.array(syn)
        for P in [(4, 1, 1, 1, 1), (4, 2, 1, 1, 1), (5, 3, 1, 2, 1), (4, 2, 1, 0, 1),
                  (6, 3, 1, 0, 1), (4, 2, 2, 1, 2)]:
            _compare(op, syn, P, np.float32, stats)
    assert stats["tie_at_cut"] > 20, stats
    assert stats["tie_explore"] > 20, stats


def test_beam_width_one_follows_the_best_child(oracle_mod):
    """Appendix B with beam_width = 1: after each round only the child with
    the highest score survives (the earlier one on a tie); the restatement's
    trace shows this directly, and the oracle's result is the one reached
    by following that child."""
    H, p, L = _tiny(31, 7, 12, uniform=False)
    ptr, idx = codes.csc_from_dense(H)
    op = oracle_mod.OracleProblem(7, 12, ptr, idx, p, L)
    rng = np.random.default_rng(5)
    syn = _syndromes(H, rng, 40)
    dec = op.decode(syn, 6, 1, 1, 1, dtype=np.float32, threads=1)
    checked = 0
    for q, s in enumerate(syn):
        trace = []
        e, conv, _ = ref.beam_decode(op, s, 6, 1, 1, 1, dtype=np.float32, trace=trace)
        for rd in trace:
            ch = rd["children"]
            best = max(sc for _, sc in ch)
            first_best = min(g for g, sc in ch if sc == best)
            assert rd["kept"] == [first_best]
            checked += 1
        assert dec["converged"][q] == int(conv)
        np.testing.assert_array_equal(dec["corrections"][q], e)
    assert checked > 30


def test_unpruned_search_returns_a_solution_of_the_first_successful_round(oracle_mod):
    """Algorithm 3 without pruning (beam_width >= 2^max_rounds): the returned
    child converges in the first round in which any child converges, and it
    satisfies He = s; among that round's converging children the oracle
    returns the first explored (descending parent score), which the
    restatement confirms."""
    H, p, L = _tiny(8, 6, 9, uniform=False)
    ptr, idx = codes.csc_from_dense(H)
    op = oracle_mod.OracleProblem(6, 9, ptr, idx, p, L)
    syn = bf.all_vectors(6)
    syn = syn[[bf.in_colspace(H, s) for s in syn]]
    dec = op.decode(syn, 9, 1 << 9, 1, 1, dtype=np.float64, threads=1)
    assert dec["converged"].all()
    for q, s in enumerate(syn):
        np.testing.assert_array_equal(_syn(H, dec["corrections"][q]), s)
        e, conv, info = ref.beam_decode(op, s, 9, 1 << 9, 1, 1, dtype=np.float64)
        assert conv
        np.testing.assert_array_equal(dec["corrections"][q], e)
        assert dec["diag"]["winner_round"][q] == info["round"]
