"""GPU decoder against the CPU oracle in configurations the workloads do not
reach on their own: eq. (1) as printed (alpha = 1) with the +-1e30
saturation acting, a check whose other neighbours are all masked
(Algorithm 2), priors above 1/2 (negative prior LLRs), the headline graph
against double precision, and the [[144,12,12]] code at the other beam
widths of Table I.

Bars as in test_gpu_parity: bit-exact against the single-precision oracle;
messages within |gpu - f64| <= 1e-4 (1 + |f64|) of the double-precision
oracle; corrections bit-exact on clean shots and the logical error rate
inside the double-precision oracle's Wilson 95% interval.
"""
from __future__ import annotations

import copy
import dataclasses

import numpy as np
import pytest

import gpu_common as gc
from bsd_inputs import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

LLR_MAX32 = np.float32(1e30)


@pytest.fixture(scope="module")
def bsd():
    import paper_2512_07057_amd as m
    m.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return m


_CODES = {}


def _code(bsd, key):
    if key not in _CODES:
        _CODES[key] = bsd.Code.from_problem(gc.problem(key))
    return _CODES[key]


def _oracle(oracle_mod, key):
    return oracle_mod.OracleProblem.from_problem(gc.problem(key))


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _decode(bsd, code, syn, P, mode=0, flags=0):
    prm = bsd.make_params(P.max_rounds, P.beam_width, P.initial_iters, P.iters_per_round,
                          P.num_results, P.alpha, mode, flags)
    out = code.decode(_dev(syn), prm)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}


def _same(got, ref, what):
    for k in ("corrections", "flips", "converged"):
        bad = np.nonzero((got[k] != ref[k]).reshape(len(got["converged"]), -1).any(1))[0]
        assert bad.size == 0, f"{what}: {k} differ on shots {bad[:10]}"


def _unmasked_edges(pr, pairs):
    keep = np.ones(pr.nnz, bool)
    for c, _ in pairs:
        keep[pr.colptr[c]:pr.colptr[c + 1]] = False
    return keep


def _run_both(code, op, pr, s, T, alpha, e_start=None, pairs=(), stop=False):
    ref = op.bp_run(s, T, alpha=alpha, e_start=e_start, pairs=pairs, stop=stop, dtype=np.float32)
    got = code.bp_run(_dev(s), T, alpha=alpha, e_start=None if e_start is None else _dev(e_start),
                      pairs=pairs, stop=stop)
    keep = _unmasked_edges(pr, pairs)
    np.testing.assert_array_equal(got["e"].cpu().numpy()[keep], ref["e"][keep])
    np.testing.assert_array_equal(got["sum_llr"].cpu().numpy(), ref["sum_llr"])
    np.testing.assert_array_equal(got["ehat"].cpu().numpy(), ref["ehat"])
    assert got["iters"] == ref["iters"] and got["converged"] == ref["converged"]
    npos, sc = op.score(ref["sum_llr"], pairs, ref["iters"], dtype=np.float32)
    assert got["next_pos"] == npos and np.float32(got["score"]) == np.float32(sc)
    return got, ref


# ---------------------------------------------------------------------------
# Eq. (1) as printed (alpha = 1), with the saturation acting
# ---------------------------------------------------------------------------

def test_alpha_one_saturated_runs_bitexact_and_near_double(bsd, oracle_mod):
    """Unscaled min-sum on the [[72,12,6]] code keeps growing once the hard
    decision is consistent; run on without stopping, every message reaches
    the +-1e30 saturation of both implementations (clamped D in the check
    phase and clamped E in the variable phase).  A masked run warm-started
    from those saturated messages follows."""
    key = "bb72_cc_p0.03"
    pr, code, op = gc.problem(key), _code(bsd, key), _oracle(oracle_mod, key)
    d = gc.samples("W0", 16, seed=3)
    rng = np.random.default_rng(2)
    saturated = 0
    for q in range(4):
        s = d["syndromes"][q]
        for T in (60, 120):
            gc.log("alpha 1 run, shot", q, "T", T)
            got, ref = _run_both(code, op, pr, s, T, 1.0)
            saturated += int((np.abs(ref["e"]) == LLR_MAX32).sum())
            r64 = op.bp_run(s, T, alpha=1.0, stop=False, dtype=np.float64)
            e = got["e"].cpu().numpy().astype(np.float64)
            assert np.max(np.abs(e - r64["e"]) / (1 + np.abs(r64["e"]))) <= 1e-4
        warm = op.bp_run(s, 120, alpha=1.0, stop=False, dtype=np.float32)["e"]
        cols = rng.choice(pr.n, size=3, replace=False)
        pairs = [(int(c), int(v)) for c, v in zip(cols, rng.integers(0, 2, size=3))]
        _run_both(code, op, pr, s, 20, 1.0, e_start=warm, pairs=pairs, stop=True)
        _run_both(code, op, pr, s, 20, 1.0, e_start=warm, pairs=pairs, stop=False)
    assert saturated > 0


@pytest.mark.parametrize("key,wl,hot,T", [("bb144_cc_p0.05", "W1", 0, 30),
                                          ("bb144_st12", "W2", 40, 6)])
def test_alpha_one_messages(bsd, oracle_mod, key, wl, hot, T):
    """Eq. (1) unscaled: bit-exact against single precision, within 1e-4 of
    double precision.  On the hot space-time graph unscaled min-sum amplifies
    single-precision rounding about twofold per iteration (the single-
    precision oracle drifts from the double one by 1.5e-5 at t = 4 and
    2.3e-3 at t = 12), so the double-precision bar is checked on short runs
    there; bit-exactness is checked at every length."""
    pr, code, op = gc.problem(key), _code(bsd, key), _oracle(oracle_mod, key)
    d = gc.samples(wl, 8, seed=5, hot=hot)
    worst = 0.0
    for q in range(4):
        s = d["syndromes"][q]
        _run_both(code, op, pr, s, 2 * T, 1.0)
        got, _ = _run_both(code, op, pr, s, T, 1.0)
        r64 = op.bp_run(s, T, alpha=1.0, stop=False, dtype=np.float64)
        for k in ("e", "sum_llr"):
            a = got[k].cpu().numpy().astype(np.float64)
            worst = max(worst, float(np.max(np.abs(a - r64[k]) / (1 + np.abs(r64[k])))))
    gc.log("alpha 1", key, "max relative error vs f64", worst)
    assert worst <= 1e-4


@pytest.mark.parametrize("wl,hot,shots", [("W0", 0, 3000), ("W1", 0, 1000), ("W2", 40, 6)])
def test_alpha_one_decode_bitexact(bsd, oracle_mod, wl, hot, shots):
    """Algorithm 3 with eq. (1) as printed, batched (and plain on a prefix)."""
    W = workloads.WORKLOADS[wl]
    P = dataclasses.replace(W.params, alpha=1.0)
    code, op = _code(bsd, W.problem_key), _oracle(oracle_mod, W.problem_key)
    d = gc.samples(wl, shots, seed=7, hot=hot)
    gc.log("alpha 1 decode", wl, hot, shots)
    got = _decode(bsd, code, d["syndromes"], P)
    ref = op.decode_params(d["syndromes"], P, dtype=np.float32, threads=16)
    _same(got, ref, f"{wl} alpha 1")
    n = min(shots, 60 if hot == 0 else 3)
    plain = _decode(bsd, code, d["syndromes"][:n], P, mode=1)
    _same(plain, {k: v[:n] for k, v in got.items() if k != "stats"}, f"{wl} alpha 1 plain")
    gc.log("  deep", got["stats"]["deep_shots"], "converged", got["converged"].mean())


# ---------------------------------------------------------------------------
# Algorithm 2: a check whose other neighbours are all masked
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("alpha", [0.625, 1.0])
def test_empty_unmasked_neighbourhood(bsd, oracle_mod, alpha):
    """A check with one unmasked neighbour: the minimum over the empty set of
    the others is the message bound, so the check sends alpha * 1e30 with
    the sign of its (flipped) syndrome bit and pins that node.  A check with
    no unmasked neighbour sends nothing and only enters the syndrome test."""
    key = "bb72_cc_p0.03"
    pr, code, op = gc.problem(key), _code(bsd, key), _oracle(oracle_mod, key)
    H = pr.dense_H()
    d = gc.samples("W0", 16, seed=8)
    rng = np.random.default_rng(4)
    for q in range(6):
        s = d["syndromes"][q]
        row = int(rng.integers(0, pr.m))
        cols = np.nonzero(H[row])[0]
        vals = rng.integers(0, 2, size=len(cols))
        for keep_one in (True, False):
            sel = cols[:-1] if keep_one else cols
            pairs = [(int(c), int(v)) for c, v in zip(sel, vals)]
            gc.log("masked row", row, "pairs", pairs)
            got, ref = _run_both(code, op, pr, s, 6, alpha, pairs=pairs, stop=False)
            if keep_one:
                # the lone unmasked node's posterior carries the bound
                assert abs(float(ref["sum_llr"][cols[-1]])) >= 0.5e30
            warm = op.bp_run(s, 3, alpha=alpha, stop=False, dtype=np.float32)["e"]
            _run_both(code, op, pr, s, 8, alpha, e_start=warm, pairs=pairs, stop=True)


# ---------------------------------------------------------------------------
# Priors above 1/2: negative prior LLRs
# ---------------------------------------------------------------------------

def _negative_prior_problem(key, cols, p_high):
    pr = copy.deepcopy(gc.problem(key))
    pr.p = pr.p.copy()
    pr.p[cols] = p_high
    pr.name = key + "_neg"
    return pr


@pytest.mark.parametrize("key,wl,shots,P", [
    ("bb72_cc_p0.03", "W0", 400, workloads.params_100iters(8)),
    ("bb144_cc_p0.05", "W1", 300, workloads.params_100iters(8)),
    ("bb144_st12", "W2", 48, workloads.DecoderParams(0, 32, 40, 30)),
])
def test_negative_priors(bsd, oracle_mod, key, wl, shots, P):
    """Columns with p_j > 1/2 have Lambda_j < 0.  Eq. (1) at iteration 1 then
    carries the parity of the other edges' negative priors; the table of
    iteration 1 stores it per row (and which edges are negative), and the
    result equals eq. (1) computed in full and the oracle."""
    base = gc.problem(key)
    rng = np.random.default_rng(12)
    cols = np.sort(rng.choice(base.n, size=max(3, base.n // 40), replace=False))
    pr = _negative_prior_problem(key, cols, rng.uniform(0.55, 0.8, size=len(cols)))
    code = bsd.Code.from_problem(pr)
    op = oracle_mod.OracleProblem.from_problem(pr)
    d = gc.samples(wl, shots, seed=6)
    syn = d["syndromes"]
    gc.log("negative priors", key, len(cols), "columns")
    table = _decode(bsd, code, syn, P)
    dense = _decode(bsd, code, syn, P, flags=bsd.FLAG_DENSE_FIRST)
    ref = op.decode_params(syn, P, dtype=np.float32, threads=16)
    _same(table, ref, "table")
    _same(dense, ref, "dense")
    plain = _decode(bsd, code, syn[:40], P, mode=1)
    _same(plain, {k: v[:40] for k, v in ref.items() if k != "diag"}, "plain")
    gc.log("  converged", table["converged"].mean(), "deep", table["stats"]["deep_shots"])


# ---------------------------------------------------------------------------
# Headline graph against double precision
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("hot,shots", [(0, 10_000), (32, 240)])
def test_w2_double_precision_clean_shots_and_ler(bsd, oracle_mod, hot, shots):
    """The BB144 12-round graph with beam32_340iters, at the nominal priors
    (1e4 shots) and with faults drawn at 32x the priors (240 shots, about a
    tenth of which go into beam rounds)."""
    W = workloads.WORKLOADS["W2"]
    code, op = _code(bsd, W.problem_key), _oracle(oracle_mod, W.problem_key)
    d = gc.samples("W2", shots, seed=0, hot=hot)
    got = _decode(bsd, code, d["syndromes"], W.params)
    ref = op.decode_params(d["syndromes"], W.params, dtype=np.float64, threads=16)
    clean = gc.clean_mask(ref["diag"])
    gc.log("W2 hot", hot, "clean", int(clean.sum()), "of", shots, "deep",
           got["stats"]["deep_shots"])
    assert clean.sum() > 0.5 * shots
    np.testing.assert_array_equal(got["corrections"][clean], ref["corrections"][clean])
    f_gpu = int(gc.failures(got, d["true_flips"]).sum())
    f_ref = int(gc.failures(ref, d["true_flips"]).sum())
    lo, hi = gc.wilson(f_ref, shots)
    gc.log("  LER gpu", f_gpu / shots, "oracle", f_ref / shots, "interval", (lo, hi))
    assert lo <= f_gpu / shots <= hi
    if hot:
        assert got["stats"]["deep_shots"] > 0


# ---------------------------------------------------------------------------
# Table I beam widths on the [[144,12,12]] code
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("bw", [8, 64])
def test_w1_other_beam_widths(bsd, oracle_mod, bw):
    """The code-capacity [[144,12,12]] workload at beam widths 8 and 64 (100
    iterations): batched and plain bit-exact against single precision."""
    P = workloads.params_100iters(bw)
    W = workloads.WORKLOADS["W1"]
    code, op = _code(bsd, W.problem_key), _oracle(oracle_mod, W.problem_key)
    d = gc.samples("W1", 2000, seed=14)
    got = _decode(bsd, code, d["syndromes"], P)
    ref = op.decode_params(d["syndromes"], P, dtype=np.float32, threads=16)
    _same(got, ref, f"W1 bw {bw}")
    plain = _decode(bsd, code, d["syndromes"][:80], P, mode=1)
    _same(plain, {k: v[:80] for k, v in ref.items() if k != "diag"}, f"W1 bw {bw} plain")
    gc.log("W1 bw", bw, "deep", got["stats"]["deep_shots"], "kernel ms", got["stats"]["kernel_ms"])
