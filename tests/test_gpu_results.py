"""num_results > 1 on the GPU (Algorithm 3 with the results set of Appendix B):
converged children keep branching, distinct solutions are collected in
exploration order and the lightest by wt(e) = sum_j e_j log((1-p_j)/p_j) is
returned.  Bar: every output bit-exact against the single-precision oracle,
and the plain form identical to the batched one."""
from __future__ import annotations

import numpy as np
import pytest

import gpu_common as gc
from bsd_inputs import workloads
from bsd_inputs.workloads import DecoderParams, TABLE_I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = [
    # workload, hot multiplier, shots, decoder
    ("W0", 3, 600, DecoderParams(6, 8, 20, 8, 4)),
    ("W0", 3, 300, DecoderParams(8, 16, 10, 6, 24)),
    ("W1", 2, 300, DecoderParams(10, 8, 20, 8, 3)),
    ("W1", 0, 2000, DecoderParams(10, 8, 20, 8, 2)),
    ("W2", 40, 8, DecoderParams(4, 8, 40, 30, 3)),
    ("W2", 40, 6, TABLE_I["beam64_32res_640iters"]),
]


@pytest.fixture(scope="module")
def bsd():
    import paper_2512_07057_amd as m
    m.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return m


def _run(bsd, code, syn, P, mode):
    prm = bsd.make_params(P.max_rounds, P.beam_width, P.initial_iters, P.iters_per_round,
                          P.num_results, P.alpha, mode)
    out = code.decode(torch.from_numpy(np.ascontiguousarray(syn)).cuda(), prm)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}


@pytest.mark.parametrize("wl,hot,shots,P", CASES)
def test_results_set_bitexact_vs_single_precision_oracle(bsd, oracle_mod, wl, hot, shots, P):
    W = workloads.WORKLOADS[wl]
    pr = gc.problem(W.problem_key)
    d = gc.samples(wl, shots, seed=5, hot=hot)
    gc.log("results", wl, "hot", hot, "shots", shots, P)
    code = bsd.Code.from_problem(pr)
    got = _run(bsd, code, d["syndromes"], P, bsd.MODE_BATCHED)
    ref = oracle_mod.OracleProblem.from_problem(pr).decode_params(d["syndromes"], P,
                                                                 dtype=np.float32, threads=16)
    for k in ("corrections", "flips", "converged"):
        bad = np.nonzero((got[k] != ref[k]).reshape(shots, -1).any(1))[0]
        assert bad.size == 0, f"{k} differ on shots {bad[:10]}"
    nres = ref["diag"]["n_results"]
    gc.log("  shots with >1 result", int((nres > 1).sum()), "reached num_results",
           int((nres >= P.num_results).sum()), "runs", got["stats"]["runs"],
           "oracle runs", int(ref["diag"]["runs"].sum()))
    # with a results set no child is cancelled: the GPU runs what the oracle runs
    # up to the child that completes the set
    assert got["stats"]["runs"] >= int(ref["diag"]["runs"].sum())
    assert (nres > 1).any(), "the case should exercise several results"


@pytest.mark.parametrize("wl,hot,shots,P", [CASES[0], CASES[2], CASES[4]])
def test_results_set_plain_equals_batched(bsd, wl, hot, shots, P):
    W = workloads.WORKLOADS[wl]
    code = bsd.Code.from_problem(gc.problem(W.problem_key))
    n = min(shots, 120)
    d = gc.samples(wl, shots, seed=5, hot=hot)
    syn = d["syndromes"][:n]
    a = _run(bsd, code, syn, P, bsd.MODE_BATCHED)
    b = _run(bsd, code, syn, P, bsd.MODE_PLAIN)
    for k in ("corrections", "flips", "converged"):
        np.testing.assert_array_equal(a[k], b[k])
    assert a["stats"]["deep_shots"] == b["stats"]["deep_shots"]
