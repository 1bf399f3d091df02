"""Batched runtime on the GPU: HIP-graph replay and the launch-geometry
autotuner leave every output unchanged."""
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


def _np(out):
    return {k: out[k].cpu().numpy() for k in ("corrections", "flips", "converged")}


def test_graph_replay_matches_eager(bsd):
    W = workloads.WORKLOADS["W1"]
    code = bsd.Code.from_problem(gc.problem(W.problem_key))
    a = torch.from_numpy(gc.samples("W1", 1500, seed=11)["syndromes"]).cuda()
    b = torch.from_numpy(gc.samples("W1", 1500, seed=12)["syndromes"]).cuda()
    P = W.params
    eager = gc.params_for(bsd, P)
    graph = bsd.make_params(P.max_rounds, P.beam_width, P.initial_iters, P.iters_per_round,
                            1, P.alpha, bsd.MODE_BATCHED, bsd.FLAG_GRAPH)
    ref_a = _np(code.decode(a, eager))
    ref_b = _np(code.decode(b, eager))
    out = {"corrections": torch.empty((1500, code.n), dtype=torch.uint8, device="cuda"),
           "flips": torch.empty((1500, code.k), dtype=torch.uint8, device="cuda"),
           "converged": torch.empty((1500,), dtype=torch.uint8, device="cuda")}
    for rep in range(4):
        gc.log("graph replay", rep)
        out["corrections"].fill_(7)
        got = _np(code.decode(a, graph, out=out))
        for k in ref_a:
            np.testing.assert_array_equal(got[k], ref_a[k])
        # eager work on other data between replays
        got_b = _np(code.decode(b, eager))
        for k in ref_b:
            np.testing.assert_array_equal(got_b[k], ref_b[k])
        torch.cuda.synchronize()


@pytest.mark.parametrize("key,wl,shots", [("bb72_cc_p0.03", "W0", 3000),
                                          ("bb144_cc_p0.05", "W1", 2000),
                                          ("bb144_st12", "W2", 20000)])
def test_autotune_keeps_results(bsd, key, wl, shots):
    W = workloads.WORKLOADS[wl]
    code = bsd.Code.from_problem(gc.problem(key))
    syn = torch.from_numpy(gc.samples(wl, shots, seed=13)["syndromes"]).cuda()
    prm = gc.params_for(bsd, W.params)
    before = _np(code.decode(syn, prm))
    info0 = code.info()
    tuned = code.autotune(syn, prm)
    gc.log("autotune", wl, "default", info0, "chosen", tuned)
    assert tuned["block"] in (64, 128, 256, 512, 1024) and tuned["grid"] > 0
    after = _np(code.decode(syn, prm))
    for k in before:
        np.testing.assert_array_equal(after[k], before[k])


@pytest.mark.parametrize("wl,hot,shots", [("W2", 0, 20000), ("W2", 40, 12), ("W1", 0, 2000),
                                          ("W0", 0, 2000)])
def test_first_iteration_table_equals_dense(bsd, wl, hot, shots):
    """Iteration 1 of the initial runs taken from the per-(code, alpha) table
    (default) gives the same outputs and work counts as eq. (1) computed in
    full."""
    W = workloads.WORKLOADS[wl]
    code = bsd.Code.from_problem(gc.problem(W.problem_key))
    syn = torch.from_numpy(gc.samples(wl, shots, seed=21, hot=hot)["syndromes"]).cuda()
    P = W.params
    dense = bsd.make_params(P.max_rounds, P.beam_width, P.initial_iters, P.iters_per_round, 1,
                            P.alpha, bsd.MODE_BATCHED, bsd.FLAG_DENSE_FIRST)
    a = code.decode(syn, dense)
    b = code.decode(syn, gc.params_for(bsd, P))
    for k in ("corrections", "flips", "converged"):
        np.testing.assert_array_equal(a[k].cpu().numpy(), b[k].cpu().numpy())
    assert a["stats"]["deep_shots"] == b["stats"]["deep_shots"]
    gc.log(wl, hot, "dense ms", a["stats"]["kernel_ms"], "table ms", b["stats"]["kernel_ms"])


def test_host_buffers_equal_device_buffers(bsd):
    """bsd_decode with host memory (staged by the library) gives the outputs
    of the same call on device memory, batched and plain."""
    W = workloads.WORKLOADS["W1"]
    code = bsd.Code.from_problem(gc.problem(W.problem_key))
    syn = gc.samples("W1", 700, seed=31)["syndromes"]
    for mode in (bsd.MODE_BATCHED, bsd.MODE_PLAIN):
        prm = gc.params_for(bsd, W.params, mode)
        n = 700 if mode == bsd.MODE_BATCHED else 60
        dev = _np(code.decode(torch.from_numpy(syn[:n]).cuda(), prm))
        host = code.decode_host(syn[:n], prm)
        for k in dev:
            np.testing.assert_array_equal(host[k], dev[k])
