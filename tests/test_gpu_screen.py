"""The sparse screen of iterations 1 and 2 in front of the batched decoder.

At t = 1 from the priors (all positive), only columns of flipped detectors
can decide 1 (eq. (4)); the screen sums their posteriors in the dense
variable phase's order and finishes the shots whose decision satisfies the
syndrome.  At t = 2 only rows that flipped or receive a negative E(1) send
negative messages; the screen forms those exactly, bounds the others from
below, and forms exact messages where the bound does not decide.  Bars:
every output, the per-call work counters (runs, iterations, deep shots) and
the errors equal those of the same call with iteration 1 only, without the
screen, and with iteration 1 computed by eq. (1) in full, on the headline
batch and on shots that overflow the screen's lists.
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


_CODES = {}


def _code(bsd, key):
    if key not in _CODES:
        _CODES[key] = bsd.Code.from_problem(gc.problem(key))
    return _CODES[key]


def _params(bsd, P, flags=0):
    return bsd.make_params(P.max_rounds, P.beam_width, P.initial_iters, P.iters_per_round,
                           P.num_results, P.alpha, bsd.MODE_BATCHED, flags)


def _np(out):
    return {k: out[k].cpu().numpy() for k in ("corrections", "flips", "converged")}


def _check_same(a, b, what):
    for k in ("corrections", "flips", "converged"):
        bad = np.nonzero((a[k] != b[k]).reshape(len(a["converged"]), -1).any(1))[0]
        assert bad.size == 0, f"{what}: {k} differ on shots {bad[:10]}"


@pytest.mark.parametrize("wl,hot,shots", [("W2", 0, 100_000), ("W2", 40, 24), ("W2", 20, 400),
                                          ("W0", 0, 10_000), ("W1", 0, 20_000), ("W3", 0, 4_000)])
def test_screen_equals_dense_first_iteration(bsd, wl, hot, shots):
    W = workloads.WORKLOADS[wl]
    code = _code(bsd, W.problem_key)
    if hot:
        syn = gc.samples(wl, shots, seed=21, hot=hot)["syndromes"]
    else:
        syn = workloads.shots_for(W, shots=shots)["syndromes"]
    syn = torch.from_numpy(np.ascontiguousarray(syn)).cuda()
    gc.log("screen", wl, hot, shots)
    outs = {}
    # ("beside" right after "screen": the decoder beside the screen runs
    # while the stream's last call handed on few shots)
    for name, flags in (("screen", 0), ("beside", bsd.FLAG_BESIDE),
                        ("screen1", bsd.FLAG_NO_SCREEN2),
                        ("no_screen", bsd.FLAG_NO_SCREEN), ("dense", bsd.FLAG_DENSE_FIRST)):
        r = code.decode(syn, _params(bsd, W.params, flags), latency=True)
        torch.cuda.synchronize()
        outs[name] = (_np(r), r["stats"], r["latency_ticks"].cpu().numpy())
        gc.log("  ", name, r["stats"])
    for name in ("beside", "screen1", "no_screen", "dense"):
        _check_same(outs["screen"][0], outs[name][0], name)
        assert outs["screen"][1]["deep_shots"] == outs[name][1]["deep_shots"], name
        if outs["screen"][1]["deep_shots"] == 0:
            # (with beam rounds, siblings of a winner stop at points that vary
            # from call to call, and so do the run and iteration counts)
            for k in ("runs", "iterations", "edge_updates"):
                assert outs["screen"][1][k] == outs[name][1][k], (name, k)
    lat = outs["screen"][2]
    assert (lat > 0).all()
    st, st1 = outs["screen"][1], outs["screen1"][1]
    assert st1["screened2_shots"] == 0 and st["screened2_shots"] <= st["screened_shots"]
    assert st["screened_shots"] - st["screened2_shots"] == st1["screened_shots"]
    if wl == "W2" and not hot:
        # iteration 2 finishes most shots that iteration 1 leaves
        assert st["screened2_shots"] > 0.8 * (shots - st1["screened_shots"])


@pytest.mark.parametrize("alpha", [1.0, 1.3])
def test_screen_alpha_beyond_the_single_detector_flag(bsd, alpha):
    """Iteration 1's first pass trusts a per-column flag proved for alpha <= 1:
    at alpha = 1 (the bound's edge) it is used, above 1 the full pass runs.
    Both equal the call without the screen, on W2 at 4x and 20x the priors
    (many flipped rows, full queues) and on W1."""
    screened = 0
    for wl, hot, shots in (("W2", 4, 4000), ("W2", 20, 1000), ("W1", 0, 5000)):
        W = workloads.WORKLOADS[wl]
        code = _code(bsd, W.problem_key)
        if hot:
            syn = gc.samples(wl, shots, seed=23, hot=hot)["syndromes"]
        else:
            syn = workloads.shots_for(W, shots=shots)["syndromes"]
        syn = torch.from_numpy(np.ascontiguousarray(syn)).cuda()
        P = W.params
        outs = {}
        for name, flags in (("screen", bsd.FLAG_BESIDE), ("no_screen", bsd.FLAG_NO_SCREEN)):
            prm = bsd.make_params(P.max_rounds, P.beam_width, P.initial_iters, P.iters_per_round,
                                  P.num_results, alpha, bsd.MODE_BATCHED, flags)
            r = code.decode(syn, prm)
            torch.cuda.synchronize()
            outs[name] = (_np(r), r["stats"])
            gc.log("  alpha", alpha, wl, name, r["stats"])
        _check_same(outs["screen"][0], outs["no_screen"][0], f"{wl} alpha {alpha}")
        screened += outs["screen"][1]["screened_shots"]
    assert screened > 0


def test_screen_tiny_batches(bsd):
    """Batches smaller than a workgroup's waves or than the dense decoder's
    grid, some shots handed on (W2 at 40x the priors): the screen, the
    decoder launched beside it (when the stream's last call handed on few
    shots) and the one after it end cleanly and agree with the call without
    the screen."""
    W = workloads.WORKLOADS["W2"]
    code = _code(bsd, W.problem_key)
    for shots in (1, 7, 63, 300):
        syn = gc.samples("W2", shots, seed=31 + shots, hot=40 if shots < 300 else 0)["syndromes"]
        syn = torch.from_numpy(np.ascontiguousarray(syn)).cuda()
        outs = {}
        for name, flags in (("screen", bsd.FLAG_BESIDE), ("no_screen", bsd.FLAG_NO_SCREEN)):
            r = code.decode(syn, _params(bsd, W.params, flags))
            torch.cuda.synchronize()
            outs[name] = _np(r)
        gc.log("  tiny", shots)
        _check_same(outs["screen"], outs["no_screen"], f"{shots} shots")


def test_screen_iteration2_with_schedule(bsd):
    """Iteration 2 scaled by the schedule's second entry (iteration 1 by the
    first): equal to the call without the screen."""
    W = workloads.WORKLOADS["W2"]
    pr = gc.problem(W.problem_key)
    code = bsd.Code.from_problem(pr)
    code.set_alpha_schedule([0.7, 0.55, 0.625])
    syn = torch.from_numpy(workloads.shots_for(W, shots=20_000)["syndromes"]).cuda()
    outs = {}
    for name, flags in (("screen", 0), ("no_screen", bsd.FLAG_NO_SCREEN)):
        r = code.decode(syn, _params(bsd, W.params, bsd.FLAG_ALPHA_SCHEDULE | flags))
        torch.cuda.synchronize()
        outs[name] = (_np(r), r["stats"])
        gc.log("  schedule", name, r["stats"])
    _check_same(outs["screen"][0], outs["no_screen"][0], "schedule")
    assert outs["screen"][1]["screened2_shots"] > 0
    if outs["screen"][1]["deep_shots"] == 0:
        for k in ("runs", "iterations"):
            assert outs["screen"][1][k] == outs["no_screen"][1][k], k


def test_screen_with_unaligned_buffers(bsd):
    """Syndromes and corrections at odd addresses: byte loads and stores."""
    W = workloads.WORKLOADS["W2"]
    pr = gc.problem(W.problem_key)
    code = _code(bsd, W.problem_key)
    syn_h = workloads.shots_for(W, shots=3000)["syndromes"]
    n = len(syn_h)
    ref = _np(code.decode(torch.from_numpy(syn_h).cuda(), _params(bsd, W.params)))
    big = torch.zeros(n * pr.m + 1, dtype=torch.uint8, device="cuda")
    syn = big[1:].view(n, pr.m)
    syn.copy_(torch.from_numpy(syn_h))
    cbig = torch.full((n * pr.n + 3,), 9, dtype=torch.uint8, device="cuda")
    out = {"corrections": cbig[3:].view(n, pr.n),
           "flips": torch.empty((n, pr.k), dtype=torch.uint8, device="cuda"),
           "converged": torch.empty((n,), dtype=torch.uint8, device="cuda")}
    got = _np(code.decode(syn, _params(bsd, W.params), out=out))
    _check_same(got, ref, "unaligned")
    assert int(cbig[:3].sum()) == 27  # nothing written before the buffer


def test_screen_in_graph_replay_and_errors(bsd):
    W = workloads.WORKLOADS["W2"]
    pr = gc.problem(W.problem_key)
    code = _code(bsd, W.problem_key)
    syn = torch.from_numpy(workloads.shots_for(W, shots=5000)["syndromes"]).cuda()
    ref = _np(code.decode(syn, _params(bsd, W.params)))
    graph = _params(bsd, W.params, bsd.FLAG_GRAPH)
    out = {"corrections": torch.empty((5000, pr.n), dtype=torch.uint8, device="cuda"),
           "flips": torch.empty((5000, pr.k), dtype=torch.uint8, device="cuda"),
           "converged": torch.empty((5000,), dtype=torch.uint8, device="cuda")}
    for rep in range(3):
        out["corrections"].fill_(7)
        _check_same(_np(code.decode(syn, graph, out=out)), ref, f"replay {rep}")
        code.decode(syn[:100].contiguous(), _params(bsd, W.params))  # eager work between replays
        torch.cuda.synchronize()
    # a byte outside {0, 1} in a shot the screen finishes, and in one it passes on
    for q in (0, 1):
        bad = syn[:64].clone()
        bad[q, 5] = 3
        with pytest.raises(bsd.BsdError) as ei:
            code.decode(bad, _params(bsd, W.params))
        assert ei.value.status == bsd.BSD_EINVAL
    # all-zero syndromes: every shot finished by the screen, nothing listed
    z = torch.zeros((1000, pr.m), dtype=torch.uint8, device="cuda")
    r = code.decode(z, _params(bsd, W.params))
    assert int(r["converged"].sum()) == 1000 and int(r["corrections"].sum()) == 0
    assert r["stats"]["iterations"] == 1000 and r["stats"]["runs"] == 1000
