"""GPU decoder against the CPU oracle (run on an MI355X).

Bars:
  * single precision oracle, same operation order: every output bit-exact
    (messages, sums, hard decisions, scores, corrections, flips, flags);
  * double precision oracle: BP messages within 1e-4 relative
    (|gpu - f64| <= 1e-4 (1 + |f64|)), corrections bit-exact on shots with
    no near-tie in any decision, logical error rate inside the oracle's
    Wilson 95% interval.
"""
from __future__ import annotations

import numpy as np
import pytest

import gpu_common as gc
from bsd_inputs import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bsd():
    import paper_2512_07057_amd as m
    m.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return m


@pytest.fixture(scope="module")
def codes(bsd):
    out = {}
    for key in ("bb72_cc_p0.03", "bb144_cc_p0.05", "bb144_st12"):
        out[key] = bsd.Code.from_problem(gc.problem(key))
        gc.log("code", key, out[key].info())
    return out


@pytest.fixture(scope="module")
def oracles(oracle_mod):
    return {key: oracle_mod.OracleProblem.from_problem(gc.problem(key))
            for key in ("bb72_cc_p0.03", "bb144_cc_p0.05", "bb144_st12")}


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


# ---------------------------------------------------------------------------
# One BP run (Algorithm 2)
# ---------------------------------------------------------------------------

RUN_CASES = [
    ("bb72_cc_p0.03", "W0", 0, [1, 4, 20]),
    ("bb144_cc_p0.05", "W1", 0, [1, 7, 30]),
    ("bb144_st12", "W2", 40, [1, 3, 12]),
]


@pytest.mark.parametrize("key,wl,hot,iters", RUN_CASES)
def test_bp_run_bitexact_vs_single_precision_oracle(codes, oracles, key, wl, hot, iters):
    code, op = codes[key], oracles[key]
    pr = gc.problem(key)
    d = gc.samples(wl, 24, seed=3, hot=hot)
    rng = np.random.default_rng(1)
    for q in range(6):
        s = d["syndromes"][q]
        for T in iters:
            # plain run from the priors, no early stop
            gc.log("bp_run", key, "shot", q, "T", T)
            ref = op.bp_run(s, T, alpha=0.625, stop=False, dtype=np.float32)
            got = code.bp_run(_dev(s), T, alpha=0.625, stop=False)
            np.testing.assert_array_equal(got["e"].cpu().numpy(), ref["e"])
            np.testing.assert_array_equal(got["sum_llr"].cpu().numpy(), ref["sum_llr"])
            np.testing.assert_array_equal(got["ehat"].cpu().numpy(), ref["ehat"])
            assert got["iters"] == ref["iters"] and got["converged"] == ref["converged"]
            npos, sc = op.score(ref["sum_llr"], [], ref["iters"], dtype=np.float32)
            assert got["next_pos"] == npos and np.float32(got["score"]) == np.float32(sc)
        # warm start and masks, with early stop
        cols = rng.choice(pr.n, size=3, replace=False)
        pairs = [(int(c), int(v)) for c, v in zip(cols, rng.integers(0, 2, size=3))]
        warm = op.bp_run(s, 5, alpha=0.625, stop=False, dtype=np.float32)["e"]
        ref = op.bp_run(s, iters[-1], alpha=0.625, e_start=warm, pairs=pairs, stop=True,
                        dtype=np.float32)
        got = code.bp_run(_dev(s), iters[-1], alpha=0.625, e_start=_dev(warm), pairs=pairs, stop=True)
        keep = np.ones(pr.nnz, bool)
        for c, _ in pairs:
            keep[pr.colptr[c]:pr.colptr[c + 1]] = False
        np.testing.assert_array_equal(got["e"].cpu().numpy()[keep], ref["e"][keep])
        np.testing.assert_array_equal(got["sum_llr"].cpu().numpy(), ref["sum_llr"])
        np.testing.assert_array_equal(got["ehat"].cpu().numpy(), ref["ehat"])
        assert got["iters"] == ref["iters"] and got["converged"] == ref["converged"]
        npos, sc = op.score(ref["sum_llr"], pairs, ref["iters"], dtype=np.float32)
        assert got["next_pos"] == npos and np.float32(got["score"]) == np.float32(sc)


@pytest.mark.parametrize("key,wl,hot,T", [("bb144_cc_p0.05", "W1", 0, 12),
                                          ("bb144_st12", "W2", 40, 10),
                                          ("bb72_cc_p0.03", "W0", 0, 12)])
def test_bp_messages_within_1e4_of_double_precision(codes, oracles, key, wl, hot, T):
    code, op = codes[key], oracles[key]
    d = gc.samples(wl, 24, seed=5, hot=hot)
    worst = 0.0
    for q in range(8):
        s = d["syndromes"][q]
        ref = op.bp_run(s, T, alpha=0.625, stop=False, dtype=np.float64)
        got = code.bp_run(_dev(s), T, alpha=0.625, stop=False)
        e = got["e"].cpu().numpy().astype(np.float64)
        err = np.abs(e - ref["e"]) / (1.0 + np.abs(ref["e"]))
        worst = max(worst, float(err.max()))
        sl = got["sum_llr"].cpu().numpy().astype(np.float64)
        errs = np.abs(sl - ref["sum_llr"]) / (1.0 + np.abs(ref["sum_llr"]))
        worst = max(worst, float(errs.max()))
    gc.log("max relative message error", key, worst)
    assert worst <= 1e-4


# ---------------------------------------------------------------------------
# Beam-search decoding (Algorithm 3)
# ---------------------------------------------------------------------------

DECODE_CASES = [
    ("W0", 0, 10_000),
    ("W1", 0, 3_000),
    ("W2", 0, 4_000),
    ("W2", 40, 16),
]


def _decode(bsd, code, syn, P, mode=0):
    out = code.decode(_dev(syn), gc.params_for(bsd, P, mode))
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}


@pytest.mark.parametrize("wl,hot,shots", DECODE_CASES)
def test_decode_bitexact_vs_single_precision_oracle(bsd, codes, oracles, wl, hot, shots):
    W = workloads.WORKLOADS[wl]
    key = W.problem_key
    d = gc.samples(wl, shots, seed=0, hot=hot)
    gc.log("decode", wl, "hot", hot, "shots", shots)
    got = _decode(bsd, codes[key], d["syndromes"], W.params)
    ref = oracles[key].decode_params(d["syndromes"], W.params, dtype=np.float32, threads=16)
    for k in ("corrections", "flips", "converged"):
        bad = np.nonzero((got[k] != ref[k]).reshape(len(d["syndromes"]), -1).any(1))[0]
        assert bad.size == 0, f"{k} differ on shots {bad[:10]}"
    st = got["stats"]
    # children of a round run concurrently on the GPU, so siblings after the
    # winner may have started before it converged: at least the oracle's runs
    assert st["runs"] >= int(ref["diag"]["runs"].sum())
    assert st["deep_shots"] == int((ref["diag"]["rounds"] > 0).sum())
    gc.log("  runs", st["runs"], "deep", st["deep_shots"], "kernel ms", st["kernel_ms"])


@pytest.mark.parametrize("wl,hot,shots", [("W0", 0, 400), ("W1", 0, 200), ("W2", 40, 6)])
def test_plain_form_equals_batched(bsd, codes, wl, hot, shots):
    W = workloads.WORKLOADS[wl]
    code = codes[W.problem_key]
    d = gc.samples(wl, shots, seed=2, hot=hot)
    gc.log("plain vs batched", wl, shots)
    a = _decode(bsd, code, d["syndromes"], W.params, mode=0)
    b = _decode(bsd, code, d["syndromes"], W.params, mode=1)
    for k in ("corrections", "flips", "converged"):
        np.testing.assert_array_equal(a[k], b[k])
    # the plain form runs children one at a time and stops at the winner
    assert a["stats"]["runs"] >= b["stats"]["runs"]
    assert a["stats"]["deep_shots"] == b["stats"]["deep_shots"]


@pytest.mark.parametrize("wl,shots", [("W0", 10_000), ("W1", 3_000)])
def test_decode_vs_double_precision_clean_shots_and_ler(bsd, codes, oracles, wl, shots):
    W = workloads.WORKLOADS[wl]
    key = W.problem_key
    d = gc.samples(wl, shots, seed=0)
    got = _decode(bsd, codes[key], d["syndromes"], W.params)
    ref = oracles[key].decode_params(d["syndromes"], W.params, dtype=np.float64, threads=16)
    clean = gc.clean_mask(ref["diag"])
    gc.log(wl, "clean shots", int(clean.sum()), "of", shots)
    assert clean.sum() > 0.5 * shots
    np.testing.assert_array_equal(got["corrections"][clean], ref["corrections"][clean])
    f_gpu = gc.failures(got, d["true_flips"]).sum()
    f_ref = gc.failures(ref, d["true_flips"]).sum()
    lo, hi = gc.wilson(int(f_ref), shots)
    gc.log(wl, "LER gpu", f_gpu / shots, "oracle", f_ref / shots, "interval", (lo, hi))
    assert lo <= f_gpu / shots <= hi


def test_full_size_w2_sampled_against_oracle_and_properties(bsd, codes, oracles):
    """All 1e5 W2 shots in one batched call (the benchmark's configuration):
    sampled shots against the oracle one by one; on every shot He = s when
    converged and the reported flips equal A e-hat."""
    W = workloads.WORKLOADS["W2"]
    pr = gc.problem(W.problem_key)
    d = workloads.shots_for(W)
    syn = d["syndromes"]
    out = codes[W.problem_key].decode(_dev(syn), gc.params_for(bsd, W.params))
    torch.cuda.synchronize()
    corr = out["corrections"]
    conv = out["converged"].cpu().numpy().astype(bool)
    nz = corr.nonzero().cpu().numpy()
    colptr, rowidx = pr.colptr, pr.rowidx
    deg = np.diff(colptr)[nz[:, 1]]
    rows = np.concatenate([rowidx[colptr[c]:colptr[c + 1]] for c in nz[:, 1]]) if len(nz) else np.zeros(0, int)
    cnt = np.zeros(syn.shape, np.int32)
    np.add.at(cnt, (np.repeat(nz[:, 0], deg), rows), 1)
    assert np.array_equal((cnt & 1)[conv], syn[conv])
    lf = np.zeros((syn.shape[0], pr.k), np.int32)
    np.add.at(lf, nz[:, 0], pr.L[:, nz[:, 1]].T.astype(np.int32))
    assert np.array_equal(lf & 1, out["flips"].cpu().numpy())
    rng = np.random.default_rng(0)
    pick = np.sort(rng.choice(syn.shape[0], size=300, replace=False))
    ref = oracles[W.problem_key].decode_params(syn[pick], W.params, dtype=np.float32, threads=16)
    np.testing.assert_array_equal(corr.cpu().numpy()[pick], ref["corrections"])
    np.testing.assert_array_equal(conv[pick], ref["converged"].astype(bool))
    f = gc.failures({"converged": conv, "flips": out["flips"].cpu().numpy()}, d["true_flips"])
    gc.log("W2 full: shots", syn.shape[0], "converged", conv.mean(), "LER", f.mean(),
           "stats", out["stats"])


# ---------------------------------------------------------------------------
# Edge cases
# ---------------------------------------------------------------------------

def test_edge_cases(bsd, codes, oracles):
    key = "bb72_cc_p0.03"
    code, op = codes[key], oracles[key]
    pr = gc.problem(key)
    W = workloads.WORKLOADS["W0"]
    d = gc.samples("W0", 200, seed=9)
    syn = d["syndromes"].copy()
    syn[0] = 0
    cases = [
        workloads.DecoderParams(0, 8, 20, 8),      # plain BP only
        workloads.DecoderParams(10, 8, 0, 8),      # no initial iterations
        workloads.DecoderParams(5, 8, 20, 0),      # no masked iterations
        workloads.DecoderParams(10, 1, 20, 8),     # beam width 1
        workloads.DecoderParams(6, 64, 10, 4),     # widest beam
        workloads.DecoderParams(3, 4, 1, 1),
    ]
    for P in cases:
        gc.log("edge case", P)
        got = _decode(bsd, code, syn, P)
        ref = op.decode_params(syn, P, dtype=np.float32, threads=16)
        for k in ("corrections", "flips", "converged"):
            np.testing.assert_array_equal(got[k], ref[k])
        assert got["converged"][0] == 1 and got["corrections"][0].sum() == 0
    # one shot
    got = _decode(bsd, code, syn[:1], W.params)
    assert got["converged"][0] == 1
    # syndromes outside the column space never converge
    bad = syn[:32].copy()
    bad[:, 0] ^= 1
    H = pr.dense_H()
    from bsd_inputs import gf2
    assert gf2.rank(H) < pr.m
    got = _decode(bsd, code, bad, W.params)
    ref = op.decode_params(bad, W.params, dtype=np.float32, threads=16)
    np.testing.assert_array_equal(got["converged"], ref["converged"])
    np.testing.assert_array_equal(got["corrections"], ref["corrections"])
    # zero shots
    out = code.decode(torch.zeros((0, pr.m), dtype=torch.uint8, device="cuda"), gc.params_for(bsd, W.params))
    assert out["corrections"].shape == (0, pr.n)
    # bytes outside {0,1} are rejected
    wrong = syn[:4].copy()
    wrong[2, 3] = 2
    with pytest.raises(bsd.BsdError) as ei:
        code.decode(_dev(wrong), gc.params_for(bsd, W.params))
    assert ei.value.status == bsd.BSD_EINVAL
    with pytest.raises(bsd.BsdError):
        code.decode(_dev(syn[:4]), bsd.make_params(10, 0, 20, 8))


def test_deterministic_and_repeatable(bsd, codes):
    W = workloads.WORKLOADS["W1"]
    code = codes[W.problem_key]
    d = gc.samples("W1", 2000, seed=4)
    a = _decode(bsd, code, d["syndromes"], W.params)
    b = _decode(bsd, code, d["syndromes"], W.params)
    for k in ("corrections", "flips", "converged"):
        np.testing.assert_array_equal(a[k], b[k])
