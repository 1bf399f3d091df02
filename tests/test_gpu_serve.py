"""Serving loop on the GPU: persistent decoders for W0, W1 and W2 resident
together, fed continuously through their request rings.  Every request's
outputs must equal those of the same syndrome decoded alone in a batch call
(identical alone and in the mix); admission must hold requests back when a
ring is full and lose none."""
from __future__ import annotations

import numpy as np
import pytest

import gpu_common as gc
from bsd_inputs import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MIX = [("W0", 0.60), ("W1", 0.25), ("W2", 0.15)]


@pytest.fixture(scope="module")
def bsd():
    import paper_2512_07057_amd as m
    m.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return m


@pytest.fixture(scope="module")
def setup(bsd):
    codes, params, syns = [], [], []
    for wl, _ in MIX:
        W = workloads.WORKLOADS[wl]
        codes.append(bsd.Code.from_problem(gc.problem(W.problem_key)))
        params.append(gc.params_for(bsd, W.params))
        syns.append(gc.samples(wl, {"W0": 3000, "W1": 1500, "W2": 1000}[wl], seed=9)["syndromes"])
    return codes, params, syns


def _alone(code, prm, syn):
    out = code.decode(torch.from_numpy(np.ascontiguousarray(syn)).cuda(), prm)
    torch.cuda.synchronize()
    return {k: out[k].cpu().numpy() for k in ("corrections", "flips", "converged")}


def test_serving_mix_identical_to_alone(bsd, setup):
    codes, params, syns = setup
    requests = 4000
    import os
    gc.log("GPU_MAX_HW_QUEUES", os.environ.get("GPU_MAX_HW_QUEUES"))
    with bsd.Server(codes, params) as srv:
        gc.log("serving", requests, "requests at 20k/s", [w for w, _ in MIX])
        outs, lat, code_of, rep = srv.serve_poisson(20_000.0, [f for _, f in MIX], requests, syns, seed=3)
    gc.log("report", {k: v for k, v in rep.items() if k != "per_code"})
    gc.log("per code", rep["per_code"])
    assert rep["requests"] == requests and (lat > 0).all()
    counts = np.bincount(code_of, minlength=3)
    assert abs(counts[0] / requests - 0.60) < 0.05 and abs(counts[2] / requests - 0.15) < 0.05
    for i, (wl, _) in enumerate(MIX):
        used = min(int(counts[i]), len(syns[i]))
        ref = _alone(codes[i], params[i], syns[i][:used])
        for k in ("corrections", "flips", "converged"):
            np.testing.assert_array_equal(outs[i][k][:used], ref[k], err_msg=f"{wl} {k}")


def test_admission_holds_requests_when_ring_full(bsd, setup):
    codes, params, syns = setup
    with bsd.Server(codes[:1], params[:1], ring_bytes=1) as srv:  # smallest ring: 64 rows
        tickets = []
        while True:
            t = srv.submit(0, syns[0][len(tickets)])
            if t is None:
                break
            tickets.append(t)
        gc.log("ring rows admitted", len(tickets))
        assert len(tickets) == 64
        got = {}
        import time
        t0 = time.time()
        while len(got) < len(tickets) and time.time() - t0 < 20:
            for t in tickets:
                if t not in got:
                    r = srv.poll(0, t)
                    if r is not None:
                        got[t] = r
        assert len(got) == len(tickets)
        # a freed row admits the next request
        t = srv.submit(0, syns[0][64])
        assert t == 64
        while (r := srv.poll(0, t)) is None:
            pass
        got[t] = r
    ref = _alone(codes[0], params[0], syns[0][:65])
    for t, r in got.items():
        np.testing.assert_array_equal(r["corrections"], ref["corrections"][t])
        np.testing.assert_array_equal(r["flips"], ref["flips"][t])
        assert r["converged"] == ref["converged"][t]


def test_decoders_restart_after_idle(bsd, setup):
    """Decoders that end after their idle limit (100 ms here) are started
    again by the next request, six times over; every answer equals the
    syndrome decoded alone.  A workgroup that ends returns its spare
    context, so no relaunch loses any (without that the [[144,12,12]]
    decoder, 32 workgroups over 96 contexts, would stall by the fourth)."""
    import time
    codes, params, syns = setup
    refs = [_alone(codes[i], params[i], syns[i][:60]) for i in range(2)]
    with bsd.Server(codes[:2], params[:2], idle_ms=100) as srv:
        base = None
        for cycle in range(6):
            tickets = [[srv.submit(i, syns[i][q]) for q in range(60)] for i in range(2)]
            got = [dict() for _ in range(2)]
            t0 = time.time()
            while any(len(got[i]) < 60 for i in range(2)):
                assert time.time() - t0 < 20, f"cycle {cycle}: requests not answered"
                for i in range(2):
                    for q, t in enumerate(tickets[i]):
                        if q not in got[i]:
                            r = srv.poll(i, t)
                            if r is not None:
                                got[i][q] = r
            for i in range(2):
                for q, r in got[i].items():
                    np.testing.assert_array_equal(r["corrections"], refs[i]["corrections"][q])
                    assert r["converged"] == refs[i]["converged"][q]
            time.sleep(0.6)
            info = [srv.info(i) for i in range(2)]
            gc.log("cycle", cycle, info)
            assert not any(x["running"] for x in info), info
            # one launch per cycle after the first (a decoder may also have
            # idled out before the first requests, while the server started
            # the other)
            if base is None:
                base = [x["launches"] for x in info]
                assert all(b >= 1 for b in base), info
            assert all(x["launches"] == b + cycle for x, b in zip(info, base)), (base, info)
