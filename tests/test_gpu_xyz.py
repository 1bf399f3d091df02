"""XYZ decoding on the GPU: the [[144,12,12]] code under depolarizing noise,
decoded over X, Y and Z faults together (a Tanner graph with length-4
cycles from the Y columns).  Same bars as the other workloads: bit-exact
against the single-precision oracle, clean shots against the double
precision oracle, logical error rate inside its Wilson interval, plain form
identical to batched."""
from __future__ import annotations

import numpy as np
import pytest

import gpu_common as gc
from bsd_inputs import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

W = workloads.WORKLOADS["W3"]


@pytest.fixture(scope="module")
def bsd():
    import paper_2512_07057_amd as m
    m.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return m


@pytest.fixture(scope="module")
def code(bsd):
    return bsd.Code.from_problem(gc.problem(W.problem_key))


@pytest.fixture(scope="module")
def oracle(oracle_mod):
    return oracle_mod.OracleProblem.from_problem(gc.problem(W.problem_key))


def _decode(bsd, code, syn, P, mode=0):
    out = code.decode(torch.from_numpy(np.ascontiguousarray(syn)).cuda(), gc.params_for(bsd, P, mode))
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}


@pytest.mark.parametrize("shots,bw", [(4000, 8), (1000, 32)])
def test_xyz_bitexact_vs_single_precision_oracle(bsd, code, oracle, shots, bw):
    P = workloads.params_100iters(bw)
    d = gc.samples("W3", shots, seed=1)
    got = _decode(bsd, code, d["syndromes"], P)
    ref = oracle.decode_params(d["syndromes"], P, dtype=np.float32, threads=16)
    for k in ("corrections", "flips", "converged"):
        bad = np.nonzero((got[k] != ref[k]).reshape(shots, -1).any(1))[0]
        assert bad.size == 0, f"{k} differ on shots {bad[:10]}"
    assert got["stats"]["deep_shots"] == int((ref["diag"]["rounds"] > 0).sum())
    gc.log("xyz bw", bw, "deep", got["stats"]["deep_shots"], "runs", got["stats"]["runs"])


def test_xyz_clean_shots_and_ler_vs_double_precision(bsd, code, oracle):
    shots = W.shots
    d = gc.samples("W3", shots, seed=0)
    got = _decode(bsd, code, d["syndromes"], W.params)
    ref = oracle.decode_params(d["syndromes"], W.params, dtype=np.float64, threads=16)
    clean = gc.clean_mask(ref["diag"])
    gc.log("xyz clean shots", int(clean.sum()), "of", shots)
    assert clean.sum() > 0.5 * shots
    np.testing.assert_array_equal(got["corrections"][clean], ref["corrections"][clean])
    f_gpu = gc.failures(got, d["true_flips"]).sum()
    f_ref = gc.failures(ref, d["true_flips"]).sum()
    lo, hi = gc.wilson(int(f_ref), shots)
    gc.log("xyz LER gpu", f_gpu / shots, "oracle", f_ref / shots, "interval", (lo, hi))
    assert lo <= f_gpu / shots <= hi


def test_xyz_plain_equals_batched(bsd, code):
    d = gc.samples("W3", 300, seed=3)
    a = _decode(bsd, code, d["syndromes"], W.params, mode=0)
    b = _decode(bsd, code, d["syndromes"], W.params, mode=1)
    for k in ("corrections", "flips", "converged"):
        np.testing.assert_array_equal(a[k], b[k])
