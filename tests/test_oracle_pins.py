"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test names the passage it pins.  None of them compares the oracle with
itself on the same input; the expected values come from brute force,
closed forms derived by hand, special cases or invariants.
"""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

from bsd_inputs import codes, gf2
from bsd_inputs.workloads import TABLE_I, DecoderParams
import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _oracle_for(oracle_mod, H, p, L=None):
    H = np.asarray(H, np.uint8)
    ptr, idx = codes.csc_from_dense(H)
    return oracle_mod.OracleProblem(H.shape[0], H.shape[1], ptr, idx, np.broadcast_to(p, (H.shape[1],)), L)


def _syn(H, e):
    return ((np.asarray(H, np.int64) @ np.asarray(e, np.int64)) & 1).astype(np.uint8)


# ---------------------------------------------------------------------------
# P1: eqs. (1)-(3) with alpha = 1 are exact max-marginals on cycle-free graphs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_tree_posteriors_are_exact_max_marginals(oracle_mod, seed):
    """Appendix A, eqs. (1)-(3): on a tree, min-sum posteriors converge to
    min_{He=s,e_j=1} wt(e) - min_{He=s,e_j=0} wt(e)."""
    pr = codes.random_tree_problem(n_checks=3 + seed % 5, seed=seed)
    assert pr.n <= 16
    H = pr.dense_H()
    rng = np.random.default_rng(100 + seed)
    op = oracle_mod.OracleProblem.from_problem(pr)
    for _ in range(3):
        e = (rng.random(pr.n) < 0.3).astype(np.uint8)
        s = _syn(H, e)
        ref = bf.max_marginals(H, s, pr.p)
        out = op.bp_run(s, max_iters=2 * pr.m + 4, alpha=1.0, stop=False)
        np.testing.assert_allclose(out["post"], ref, rtol=0, atol=1e-9)
        # eq. (4) from the exact marginals
        np.testing.assert_array_equal(out["ehat"], (ref <= 0).astype(np.uint8))


@pytest.mark.parametrize("seed", range(8))
def test_tree_masked_posteriors_are_conditional_max_marginals(oracle_mod, seed):
    """Algorithm 2: masking fixed nodes and flipping the syndrome for v = 1
    gives the max-marginals of the problem conditioned on those values."""
    pr = codes.random_tree_problem(n_checks=4 + seed % 4, seed=50 + seed, max_leaf_vars=3)
    H = pr.dense_H()
    rng = np.random.default_rng(7 + seed)
    op = oracle_mod.OracleProblem.from_problem(pr)
    checked = 0
    for _ in range(6):
        e = (rng.random(pr.n) < 0.3).astype(np.uint8)
        s = _syn(H, e)
        cols = rng.choice(pr.n, size=2, replace=False)
        pairs = [(int(c), int(rng.integers(0, 2))) for c in cols]
        ref = bf.max_marginals(H, s, pr.p, fixed=dict(pairs))
        if np.isnan(ref).all():
            continue
        out = op.bp_run(s, max_iters=2 * pr.m + 4, alpha=1.0, stop=False, pairs=pairs)
        for j in range(pr.n):
            if j in dict(pairs) or np.isnan(ref[j]):
                continue
            if np.isinf(ref[j]):
                assert np.sign(out["post"][j]) == np.sign(ref[j]) and abs(out["post"][j]) >= 1e29
            else:
                assert abs(out["post"][j] - ref[j]) <= 1e-9, (j, out["post"][j], ref[j])
            checked += 1
    assert checked > 0


# ---------------------------------------------------------------------------
# P2: closed forms with a scaling factor alpha
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("alpha", [1.0, 0.625, 0.8])
@pytest.mark.parametrize("s1,s2", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_two_check_path_closed_form(oracle_mod, alpha, s1, s2):
    """Eqs. (1)-(3) on the path a - (1) - b - (2) - c, worked by hand.

    t = 1: post_a = La + a*g1*Lb, post_b = Lb + a*g1*La + a*g2*Lc, post_c = Lc + a*g2*Lb
    t = 2: post_a = La + a*g1*(Lb + a*g2*Lc), post_c = Lc + a*g2*(Lb + a*g1*La),
           post_b unchanged; g_i = (-1)^{s_i}.
    """
    H = np.array([[1, 1, 0], [0, 1, 1]], np.uint8)
    p = np.array([0.1, 0.2, 0.05])
    La, Lb, Lc = np.log((1 - p) / p)
    g1, g2 = (-1) ** s1, (-1) ** s2
    op = _oracle_for(oracle_mod, H, p)
    s = np.array([s1, s2], np.uint8)
    one = op.bp_run(s, 1, alpha=alpha, stop=False)["post"]
    two = op.bp_run(s, 2, alpha=alpha, stop=False)["post"]
    a = alpha
    exp1 = [La + a * g1 * Lb, Lb + a * g1 * La + a * g2 * Lc, Lc + a * g2 * Lb]
    exp2 = [La + a * g1 * (Lb + a * g2 * Lc), Lb + a * g1 * La + a * g2 * Lc,
            Lc + a * g2 * (Lb + a * g1 * La)]
    np.testing.assert_allclose(one, exp1, rtol=1e-13)
    np.testing.assert_allclose(two, exp2, rtol=1e-13)
    one32 = op.bp_run(s, 1, alpha=alpha, stop=False, dtype=np.float32)["post"]
    np.testing.assert_allclose(one32, exp1, rtol=2e-6)


def test_single_check_signs_and_exclusive_min(oracle_mod):
    """Eq. (1) on one check of degree 4 from a warm start with mixed signs:
    D_j = alpha (-1)^s prod_{j' != j} sgn(E_j') min_{j' != j} |E_j'|."""
    H = np.ones((1, 4), np.uint8)
    p = np.full(4, 0.1)
    lam = np.log(0.9 / 0.1)
    op = _oracle_for(oracle_mod, H, p)
    e0 = np.array([2.0, -0.5, 3.0, -1.5])
    alpha = 0.75
    for s in (0, 1):
        out = op.bp_run(np.array([s], np.uint8), 1, alpha=alpha, e_start=e0, stop=False)
        g = (-1) ** s
        d = np.array([
            alpha * g * (-1) * (+1) * (-1) * 0.5,   # others: -0.5, 3, -1.5
            alpha * g * (+1) * (+1) * (-1) * 1.5,   # others: 2, 3, -1.5
            alpha * g * (+1) * (-1) * (-1) * 0.5,   # others: 2, -0.5, -1.5
            alpha * g * (+1) * (-1) * (+1) * 0.5,   # others: 2, -0.5, 3
        ])
        np.testing.assert_allclose(out["post"], lam + d, rtol=1e-14)
        # a single check per column: eq. (2) leaves E = Lambda
        np.testing.assert_allclose(out["e"], np.full(4, lam), rtol=0)


def test_hard_decision_zero_goes_to_one(oracle_mod):
    """Eq. (4): a posterior of exactly 0 decides e_j = 1."""
    H = np.array([[1, 1]], np.uint8)
    p = np.array([0.2, 0.2])
    op = _oracle_for(oracle_mod, H, p)
    out = op.bp_run(np.array([1], np.uint8), 1, alpha=1.0, stop=False)
    assert np.all(out["post"] == 0.0)
    np.testing.assert_array_equal(out["ehat"], [1, 1])


def test_empty_unmasked_neighbourhood_saturates(oracle_mod):
    """Algorithm 2 with every other neighbour of a check masked: the minimum
    over an empty set is llr_max, so the check pins the remaining node."""
    H = np.array([[1, 1, 1]], np.uint8)
    p = np.full(3, 0.1)
    op = _oracle_for(oracle_mod, H, p)
    for v0, v1, s in [(0, 0, 1), (1, 0, 1), (1, 1, 0), (0, 1, 0)]:
        out = op.bp_run(np.array([s], np.uint8), 1, alpha=0.625, pairs=[(0, v0), (1, v1)], stop=False)
        need = s ^ v0 ^ v1
        assert out["ehat"][2] == need
        assert abs(out["post"][2]) >= 0.6e30


# ---------------------------------------------------------------------------
# P3 / P4: masking equals puncturing; warm start semantics
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("seed", range(6))
def test_masked_bp_equals_punctured_graph(oracle_mod, dtype, seed):
    """Algorithm 2: masked BP on H equals plain BP on H with the masked
    columns deleted, the syndrome flipped by the columns fixed to 1, and the
    warm-start messages restricted to the remaining edges."""
    pr = codes.random_ldpc_problem(20, 40, 3, seed=seed, p=0.08)
    H = pr.dense_H()
    rng = np.random.default_rng(seed)
    e = (rng.random(pr.n) < 0.1).astype(np.uint8)
    s = _syn(H, e)
    op = oracle_mod.OracleProblem.from_problem(pr)
    warm = op.bp_run(s, 5, stop=False, dtype=dtype)["e"]
    cols = rng.choice(pr.n, size=4, replace=False)
    pairs = [(int(c), int(v)) for c, v in zip(cols, rng.integers(0, 2, size=4))]
    masked = op.bp_run(s, 7, e_start=warm, pairs=pairs, stop=False, dtype=dtype)

    keep = np.array([j for j in range(pr.n) if j not in dict(pairs)])
    Hp = H[:, keep]
    sp = s.copy()
    for c, v in pairs:
        if v:
            sp ^= H[:, c]
    ptr, idx = codes.csc_from_dense(Hp)
    op2 = oracle_mod.OracleProblem(pr.m, len(keep), ptr, idx, pr.p[keep])
    edge_keep = np.concatenate([np.arange(pr.colptr[j], pr.colptr[j + 1]) for j in keep])
    plain = op2.bp_run(sp, 7, e_start=warm[edge_keep], stop=False, dtype=dtype)
    np.testing.assert_array_equal(masked["e"][edge_keep], plain["e"])
    np.testing.assert_array_equal(masked["sum_llr"][keep], plain["sum_llr"])
    np.testing.assert_array_equal(masked["ehat"][keep], plain["ehat"])
    assert masked["converged"] == plain["converged"]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_warm_start_with_priors_is_standard_bp(oracle_mod, dtype):
    """Algorithm 2 with edge_msgs = Lambda and no pairs is the BP of Appendix A."""
    pr = codes.bb_code_capacity(6, 6, 0.05)
    H = pr.dense_H()
    op = oracle_mod.OracleProblem.from_problem(pr)
    rng = np.random.default_rng(3)
    lam = np.log((1 - pr.p) / pr.p).astype(dtype)
    e0 = np.repeat(lam, np.diff(pr.colptr))
    for _ in range(5):
        s = _syn(H, (rng.random(pr.n) < 0.06).astype(np.uint8))
        a = op.bp_run(s, 15, dtype=dtype)
        b = op.bp_run(s, 15, e_start=e0, dtype=dtype)
        for key in ("e", "sum_llr", "ehat", "post"):
            np.testing.assert_array_equal(a[key], b[key])
        assert a["iters"] == b["iters"] and a["converged"] == b["converged"]


def test_bp_state_is_the_edge_messages(oracle_mod):
    """Appendix A: D(t) depends on E(t-1) only, so T1 + T2 iterations equal
    T2 iterations warm-started from E(T1); and sum_LLR is the sum of the
    per-iteration posteriors (Algorithm 3, sum over all BP iterations)."""
    pr = codes.bb_code_capacity(6, 12, 0.05)
    H = pr.dense_H()
    op = oracle_mod.OracleProblem.from_problem(pr)
    rng = np.random.default_rng(11)
    s = _syn(H, (rng.random(pr.n) < 0.08).astype(np.uint8))
    full = op.bp_run(s, 9, stop=False)
    e = None
    acc = np.zeros(pr.n)
    for t in range(9):
        step = op.bp_run(s, 1, e_start=e, stop=False)
        acc += step["post"]
        e = step["e"]
    np.testing.assert_array_equal(e, full["e"])
    np.testing.assert_allclose(acc, full["sum_llr"], rtol=1e-12)


# ---------------------------------------------------------------------------
# Path score and branching node (Algorithm 3)
# ---------------------------------------------------------------------------

def test_next_pos_and_score_small_cases(oracle_mod):
    """next_pos = argmin_{j in U} |sum_LLR[j]| (lowest j on ties), and
    score = sum_{j in U} |sum_LLR[j]| / iters, on exactly representable values."""
    H = np.ones((1, 6), np.uint8)
    op = _oracle_for(oracle_mod, H, np.full(6, 0.1))
    sl = np.array([3.0, -1.0, 2.0, -0.5, 0.5, 8.0])
    for dt in (np.float64, np.float32):
        # the sums are exact in both precisions; the division is one rounding
        assert op.score(sl, [], 4, dtype=dt) == (3, dt(3 + 1 + 2 + 0.5 + 0.5 + 8) / dt(4))
        assert op.score(sl, [(3, 1)], 5, dtype=dt) == (4, dt(3 + 1 + 2 + 0.5 + 8) / dt(5))
        assert op.score(sl, [(3, 1), (4, 0)], 3, dtype=dt) == (1, dt(3 + 1 + 2 + 8) / dt(3))
        assert op.score(sl, [(j, 0) for j in range(6)], 3, dtype=dt) == (-1, 0.0)
        assert op.score(sl, [], 0, dtype=dt) == (3, 0.0)


def test_score_sum_order_is_aligned_pairwise_tree(oracle_mod):
    """The score's sum is an aligned pairwise tree over column index (the
    reading that fixes the rounding of the unordered sum): with values whose
    sum depends on association the tree result is the expected one."""
    n = 4
    H = np.ones((1, n), np.uint8)
    op = _oracle_for(oracle_mod, H, np.full(n, 0.1))
    big = np.float32(2.0 ** 24)
    # (1 + 1) + (1 + 2^24): the right pair rounds to 2^24 (ties to even), then + 2 is exact;
    # a left-to-right sum would give (3 + 2^24) rounded to 2^24 + 4.
    sl = np.array([1.0, 1.0, 1.0, big], np.float32)
    _, sc = op.score(sl, [], 1, dtype=np.float32)
    assert sc == np.float32(2.0 ** 24 + 2)
    assert np.float32(np.float32(np.float32(1 + 1) + 1) + big) == np.float32(2.0 ** 24 + 4)
    # a masked node enters the tree as a zero in its own position:
    # (1 + 1) + (0 + 2^24) = 2^24 + 2 exactly
    sl = np.array([1.0, 1.0, 5.0, big], np.float32)
    _, sc = op.score(sl, [(2, 0)], 1, dtype=np.float32)
    assert sc == np.float32(2.0 ** 24 + 2)


# ---------------------------------------------------------------------------
# P5 - P8: the controller against special cases and invariants
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_zero_rounds_is_plain_bp(oracle_mod, dtype):
    """Algorithm 3 with max_rounds = 0 returns the initial BP run's result."""
    pr = codes.bb_code_capacity(6, 6, 0.05)
    H = pr.dense_H()
    op = oracle_mod.OracleProblem.from_problem(pr)
    rng = np.random.default_rng(5)
    syn = np.array([_syn(H, (rng.random(pr.n) < 0.07).astype(np.uint8)) for _ in range(40)])
    dec = op.decode(syn, 0, 8, 25, 10, dtype=dtype)
    for q in range(len(syn)):
        r = op.bp_run(syn[q], 25, dtype=dtype)
        np.testing.assert_array_equal(dec["corrections"][q], r["ehat"])
        assert dec["converged"][q] == r["converged"]


@pytest.mark.parametrize("seed", range(5))
def test_unpruned_beam_is_complete(oracle_mod, seed):
    """With beam_width >= 2^max_rounds and max_rounds = n the branching tree is
    never pruned and its leaves fix every node, so a syndrome in the column
    space of H is always decoded (He = s), and one outside never is."""
    rng = np.random.default_rng(seed)
    m, n = 5, 7
    H = (rng.random((m, n)) < 0.45).astype(np.uint8)
    H[0, :] |= (np.arange(n) < 2).astype(np.uint8)
    p = rng.uniform(0.05, 0.3, size=n)
    op = _oracle_for(oracle_mod, H, p)
    syn = bf.all_vectors(m)
    dec = op.decode(syn, max_rounds=n, beam_width=1 << n, initial_iters=2, iters_per_round=2)
    for q, s in enumerate(syn):
        feasible = bf.in_colspace(H, s)
        assert dec["converged"][q] == (1 if feasible else 0)
        if feasible:
            np.testing.assert_array_equal(_syn(H, dec["corrections"][q]), s)


@pytest.mark.parametrize("seed", range(4))
def test_success_never_beats_minimum_weight(oracle_mod, seed):
    """Appendix B weight wt(e): a returned solution satisfies He = s and weighs
    at least the exhaustive minimum."""
    rng = np.random.default_rng(20 + seed)
    m, n = 8, 14
    H = (rng.random((m, n)) < 0.3).astype(np.uint8)
    p = rng.uniform(0.02, 0.2, size=n)
    op = _oracle_for(oracle_mod, H, p)
    syn = np.array([_syn(H, (rng.random(n) < 0.15).astype(np.uint8)) for _ in range(30)])
    dec = op.decode(syn, 4, 4, 6, 4)
    w = bf.weights(p)
    for q in range(len(syn)):
        if dec["converged"][q]:
            c = dec["corrections"][q]
            np.testing.assert_array_equal(_syn(H, c), syn[q])
            wmin, _ = bf.min_weight_solution(H, syn[q], p)
            assert float(c @ w) >= wmin - 1e-12


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_invariants_on_bb72(oracle_mod, dtype):
    """Converged => He = s and A ehat = the returned flips; zero syndrome =>
    one run of one iteration, ehat = 0; runs <= 1 + sum_r min(2^r, 2 bw);
    results do not depend on the number of host threads."""
    from bsd_inputs import workloads
    wl = workloads.WORKLOADS["W0"]
    pr = workloads.problem(wl.problem_key)
    H = pr.dense_H()
    op = oracle_mod.OracleProblem.from_problem(pr)
    d = workloads.shots_for(wl, shots=600, cache=False)
    syn = np.vstack([np.zeros((1, pr.m), np.uint8), d["syndromes"]])
    P = wl.params
    dec = op.decode_params(syn, P, dtype=dtype, threads=1)
    dec4 = op.decode_params(syn, P, dtype=dtype, threads=4)
    for key in ("corrections", "flips", "converged"):
        np.testing.assert_array_equal(dec[key], dec4[key])
    conv = dec["converged"].astype(bool)
    s_hat = (dec["corrections"].astype(np.int64) @ H.T.astype(np.int64)) & 1
    assert np.array_equal(s_hat[conv], syn[conv])
    f_hat = (dec["corrections"].astype(np.int64) @ pr.L.T.astype(np.int64)) & 1
    assert np.array_equal(f_hat, dec["flips"])
    dg = dec["diag"]
    assert conv[0] and dec["corrections"][0].sum() == 0
    assert dg["runs"][0] == 1 and dg["iterations"][0] == 1
    bound = 1 + sum(min(2 ** r, 2 * P.beam_width) for r in range(1, P.max_rounds + 1))
    assert dg["runs"].max() <= bound
    assert (dg["runs"] > 1).any(), "no shot exercised the beam search"


def test_syndrome_outside_column_space_never_converges(oracle_mod):
    """Appendix A: no ehat satisfies He = s when s is not in colspace(H); BB72's
    H_X has rank 30 < 36, so flipping one detector of a valid syndrome breaks
    a row dependency."""
    pr = codes.bb_code_capacity(6, 6, 0.03)
    H = pr.dense_H()
    assert gf2.rank(H) == 30
    op = oracle_mod.OracleProblem.from_problem(pr)
    rng = np.random.default_rng(9)
    syn = []
    for _ in range(12):
        s = _syn(H, (rng.random(pr.n) < 0.03).astype(np.uint8))
        s[int(rng.integers(0, pr.m))] ^= 1
        syn.append(s)
    dec = op.decode(np.array(syn), 3, 4, 10, 5)
    assert not dec["converged"].any()


def test_num_results_collects_distinct_solutions(oracle_mod):
    """Algorithm 3 with num_results > 1: the returned solution is valid and is
    no heavier than with num_results = 1 on the same syndrome."""
    from bsd_inputs import workloads
    pr = workloads.problem("bb144_cc_p0.05")
    H = pr.dense_H()
    op = oracle_mod.OracleProblem.from_problem(pr)
    d = workloads.shots_for(workloads.WORKLOADS["W1"], shots=200, cache=False)
    one = op.decode(d["syndromes"], 6, 16, 20, 8, num_results=1)
    many = op.decode(d["syndromes"], 6, 16, 20, 8, num_results=4)
    w = np.log((1 - pr.p) / pr.p)
    for q in range(200):
        if many["converged"][q]:
            np.testing.assert_array_equal(_syn(H, many["corrections"][q]), d["syndromes"][q])
        if one["converged"][q] and many["converged"][q]:
            assert many["corrections"][q] @ w <= one["corrections"][q] @ w + 1e-9
    assert (many["diag"]["n_results"] > 1).any()


# ---------------------------------------------------------------------------
# P9: Table I naming rule
# ---------------------------------------------------------------------------

def test_table_I_naming():
    """Table I: name = initial_iters + max_rounds * iters_per_round iterations."""
    with open(os.path.join(GOLDEN, "table1.json")) as f:
        rows = json.load(f)["rows"]
    for row in rows:
        p = TABLE_I[row["name"]]
        assert (p.max_rounds, p.beam_width, p.initial_iters, p.iters_per_round, p.num_results) == tuple(row["params"])
        assert p.total_iters == row["iters_in_name"]
