#!/usr/bin/env python3
"""Benchmark of the batched GPU beam-search decoder on one MI355X.

Workload: the [[144,12,12]] bivariate bicycle code's 12-round space-time
detector graph (936 detectors x 8592 fault columns, 37303 edges, priors
log-uniform in [1e-5, 1e-3]); 1e5 seeded synthetic syndromes; decoder
beam32_340iters (max_rounds 10, beam_width 32, initial_iters 40,
iters_per_round 30) with scaling 0.625 and fp32 messages.

A step decodes the whole batch (syndromes already in device memory) with
one call of the batched decoder: the iteration-1 screen, then the
persistent decoder for the shots the screen hands on.  Printed as one JSON
line: shots/s, per-shot device decode latency percentiles, the plain
one-launch-per-BP-run form's shots/s on a prefix of the same syndromes, the
call's position against the HBM floor of its mandatory input and output,
legs for beams of uneven depth (faults drawn at 40x the priors) and for the
[[144,12,12]] code-capacity workload, the serving loop, and the CPU oracle's
rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "shots/sec + p99.9 decode latency, BB144 12-round, beam 32; batched vs plain"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_w2_decode.json")
LEGS = ("host", "plain", "hot", "w1", "serving", "cpu")


def kernel_source_digest() -> str:
    """Digest of every HIP source and header of the library."""
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2512_07057_amd", "csrc")
    for f in sorted(os.listdir(src)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(src, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per call from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_digest") != kernel_source_digest():
        return None
    return t


def pct(x, q):
    return float(np.percentile(x, q)) if len(x) else None


def host_cpu():
    info = {"threads": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
            else os.cpu_count()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Core(s) per socket", "Socket(s)"):
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def cpu_baseline(pr, params, syn_all, target_s=8.0):
    """The oracle on the host cores: single precision in the GPU's operation
    order (the value) and double precision, both built -O3 -march=native
    without FMA contraction; one shot per thread over every host thread."""
    import oracle
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    op = oracle.OracleProblem.from_problem(pr, flavour="native")
    res = {}
    for name, dt in (("f32", np.float32), ("f64", np.float64)):
        probe = min(2000, len(syn_all))
        t0 = time.perf_counter()
        op.decode_params(syn_all[:probe], params, dtype=dt, threads=cores)
        dt_probe = time.perf_counter() - t0
        n = int(min(len(syn_all), max(probe, probe * target_s / max(dt_probe, 1e-6))))
        t0 = time.perf_counter()
        op.decode_params(syn_all[:n], params, dtype=dt, threads=cores)
        wall = time.perf_counter() - t0
        res[name] = {"shots_per_s": n / wall, "shots": n, "wall_s": wall}
    # single-thread time per shot (the kind of figure the paper reports for its CPU decoder)
    nl = min(1000, len(syn_all))
    per = np.empty(nl)
    for i in range(nl):
        t1 = time.perf_counter()
        op.decode_params(syn_all[i:i + 1], params, dtype=np.float32, threads=1)
        per[i] = (time.perf_counter() - t1) * 1e6
    f32 = res["f32"]
    return {"value": f32["shots_per_s"], "unit": "shots/s", "cores": cores, "kind": "oracle",
            "sample": f"first {f32['shots']} of the benchmark's syndromes, single-precision "
                      f"oracle in the GPU's operation order (-O3 -march=native, no FMA "
                      f"contraction), one shot per thread over {cores} host threads, "
                      f"{f32['wall_s']:.1f} s wall",
            "f64": res["f64"], "host": host_cpu(),
            "single_thread_latency_us": {"p50": pct(per, 50), "p99": pct(per, 99),
                                         "p999": pct(per, 99.9), "shots": nl}}


def serving(bsd, torch, w2_code, w2_syn, w2_corr, seconds=2.0, rate=20_000.0):
    """The serving loop: W0, W1 and W2 resident together, Poisson arrivals at
    `rate` per second mixing them 60/25/15 %, decoded continuously by one
    persistent decoder per code; latency from arrival to result on the host."""
    from bsd_inputs import workloads
    mix = [("W0", 0.60), ("W1", 0.25), ("W2", 0.15)]
    codes, params, syns = [], [], []
    for wl, _ in mix:
        W = workloads.WORKLOADS[wl]
        P = W.params
        params.append(bsd.make_params(P.max_rounds, P.beam_width, P.initial_iters,
                                      P.iters_per_round, P.num_results, P.alpha, bsd.MODE_BATCHED))
        if wl == "W2":
            codes.append(w2_code)
            syns.append(w2_syn)
        else:
            codes.append(bsd.Code.from_problem(workloads.problem(W.problem_key)))
            syns.append(np.ascontiguousarray(workloads.shots_for(W, shots=20_000)["syndromes"]))
    requests = int(seconds * rate)
    with bsd.Server(codes, params) as srv:
        outs, lat, code_of, rep = srv.serve_poisson(rate, [f for _, f in mix], requests, syns, seed=0)
    # identical alone and in the mix: W2 against the batched benchmark's own
    # outputs, W0 and W1 against a batched call on the syndromes they used
    counts = np.bincount(code_of, minlength=3)
    same = True
    for i, (wl, _) in enumerate(mix):
        used = int(min(counts[i], len(syns[i])))
        if wl == "W2":
            ref = w2_corr[:used]
        else:
            r = codes[i].decode(torch.from_numpy(syns[i][:used]).cuda(), params[i])
            ref = r["corrections"].cpu().numpy()
        same = same and bool((outs[i]["corrections"][:used] == ref).all())
    return {"offered_req_per_s": rep["offered_per_s"], "served_req_per_s": rep["served_per_s"],
            "requests": rep["requests"], "p50_us": rep["p50_us"], "p99_us": rep["p99_us"],
            "p999_us": rep["p999_us"], "max_us": rep["max_us"],
            "admission_waits": rep["admission_waits"],
            "per_code": {wl: pc for (wl, _), pc in zip(mix, rep["per_code"])},
            "identical_to_alone": same,
            "what": "Poisson arrivals mixing W0/W1/W2 60/25/15 %, one persistent decoder per "
                    "code fed through rings in pinned host memory; latency from arrival to "
                    "result on the host clock"}


def timed_calls(code, syn, prm, steps, torch):
    """`steps` decode calls after one warm-up; per-call stats and wall time."""
    code.decode(syn, prm)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        stats.append(code.decode(syn, prm)["stats"])
    torch.cuda.synchronize()
    return stats, time.perf_counter() - t0


def hot_leg(bsd, torch, code, pr, P, shots=2000, mult=40.0, steps=3):
    """Beams of uneven depth on the headline graph: faults drawn at `mult` x
    the priors (the decoder keeps the true priors), so most shots enter
    beam rounds.  Work rate and the slot traffic of the child runs: each
    child reads its parent's messages and writes its own (nnz_pad fp32 each)."""
    from bsd_inputs import sampler
    hot = type("Hot", (), {"p": np.minimum(pr.p * mult, 0.4), "colptr": pr.colptr,
                           "rowidx": pr.rowidx, "m": pr.m, "k": pr.k, "L": pr.L})()
    d = sampler.sample(hot, shots, 0)
    syn = torch.from_numpy(np.ascontiguousarray(d["syndromes"])).cuda()
    prm = bsd.make_params(P.max_rounds, P.beam_width, P.initial_iters, P.iters_per_round,
                          P.num_results, P.alpha, bsd.MODE_BATCHED)
    stats, wall = timed_calls(code, syn, prm, steps, torch)
    r = code.decode(syn, prm, latency=True)
    torch.cuda.synchronize()
    lat = r["latency_ticks"].cpu().numpy().astype(np.float64) / 100.0
    conv = r["converged"].cpu().numpy().astype(bool)
    fails = (~conv) | (r["flips"].cpu().numpy() != d["true_flips"]).any(1)
    kms = float(np.mean([s["kernel_ms"] for s in stats]))
    runs = float(np.mean([s["runs"] for s in stats]))
    iters = float(np.mean([s["iterations"] for s in stats]))
    child_runs = runs - shots
    slot_bytes = 2 * 4 * ((pr.nnz + 3) // 4 * 4)
    return {"workload": f"W2-hot: the W2 graph and decoder, faults at {mult:g}x the priors "
                        f"(about {pr.p.sum() * mult:.0f} per shot), {shots} seeded shots",
            "shots_per_s": shots / (wall / steps), "kernel_ms": kms,
            "deep_shots": int(stats[-1]["deep_shots"]), "runs": runs, "bp_iterations": iters,
            "edge_updates_per_s": iters * pr.nnz / (kms * 1e-3),
            "child_runs": child_runs,
            "slot_bytes_per_child_run": slot_bytes,
            "slot_traffic_GBs": child_runs * slot_bytes / (kms * 1e-3) / 1e9,
            "latency_us": {"p50": pct(lat, 50), "p99": pct(lat, 99), "p999": pct(lat, 99.9),
                           "max": float(lat.max())},
            "ler": float(fails.mean()), "converged_frac": float(conv.mean())}


def w1_leg(bsd, torch, steps=3):
    """The [[144,12,12]] code-capacity workload (p = 0.05, 1e5 shots, beam width
    32, 100 iterations split 20 + 10 x 8)."""
    from bsd_inputs import workloads
    W = workloads.WORKLOADS["W1"]
    P = W.params
    pr = workloads.problem(W.problem_key)
    code = bsd.Code.from_problem(pr)
    d = workloads.shots_for(W)
    syn = torch.from_numpy(np.ascontiguousarray(d["syndromes"])).cuda()
    prm = bsd.make_params(P.max_rounds, P.beam_width, P.initial_iters, P.iters_per_round,
                          P.num_results, P.alpha, bsd.MODE_BATCHED)
    stats, wall = timed_calls(code, syn, prm, steps, torch)
    info = code.info()
    kms = float(np.mean([s["kernel_ms"] for s in stats]))
    iters = float(np.mean([s["iterations"] for s in stats]))
    return {"workload": "W1: [[144,12,12]] BB code capacity, 72 x 144, 432 edges, p = 0.05, "
                        "1e5 seeded shots, beam width 32, 100 iterations",
            "shots_per_s": len(syn) / (wall / steps), "kernel_ms": kms,
            "screened_shots": int(stats[-1]["screened_shots"]),
            "deep_shots": int(stats[-1]["deep_shots"]),
            "runs": float(np.mean([s["runs"] for s in stats])), "bp_iterations": iters,
            "edge_updates_per_s": iters * pr.nnz / (kms * 1e-3),
            "block_threads": info["block"], "grid_blocks": info["grid"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--shots", type=int, default=100_000)
    ap.add_argument("--streams", type=int, default=4,
                    help="streams the timed calls are spread over (each a workspace of its own)")
    ap.add_argument("--plain-shots", type=int, default=10_000)
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated extra legs to run after the headline: " + ",".join(LEGS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-host-buffers", action="store_true",
                    help="skip the host-buffer (bus-inclusive) leg, e.g. under a profiler")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving-loop measurement (Poisson arrivals over W0/W1/W2)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a kernel of "
                         "known traffic for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this decoder runs on one GPU; --gpus {args.gpus} is not supported "
              f"(shots shard across GPUs with no exchange, see the design notes)", file=sys.stderr)
        sys.exit(2)
    legs = {x for x in args.legs.split(",") if x}
    if args.no_cpu_baseline:
        legs.discard("cpu")
    if args.no_host_buffers:
        legs.discard("host")
    if args.no_serving:
        legs.discard("serving")

    # The serving measurement keeps three persistent decoders on streams of
    # their own: enough hardware queues that none waits behind another kernel.
    if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < 8:
        os.environ["GPU_MAX_HW_QUEUES"] = "8"
    import torch
    import paper_2512_07057_amd as bsd
    from bsd_inputs import workloads

    wl = workloads.WORKLOADS["W2"]
    P = wl.params
    pr = workloads.problem(wl.problem_key)
    data = workloads.shots_for(wl, shots=args.shots)
    syn_h = np.ascontiguousarray(data["syndromes"])
    dev = torch.device("cuda:0")
    code = bsd.Code.from_problem(pr)
    info = code.info()
    syn = torch.from_numpy(syn_h).to(dev)
    shots = syn.shape[0]
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    out = {
        "corrections": torch.empty((shots, pr.n), dtype=torch.uint8, device=dev),
        "flips": torch.empty((shots, pr.k), dtype=torch.uint8, device=dev),
        "converged": torch.empty((shots,), dtype=torch.uint8, device=dev),
    }
    prm = bsd.make_params(P.max_rounds, P.beam_width, P.initial_iters, P.iters_per_round,
                          P.num_results, P.alpha, bsd.MODE_BATCHED)
    # Calls enqueued back to back (asynchronous, as a pipeline of batches
    # makes them) on `nstreams` streams in turn, each stream with its own
    # workspace in the library and its own output buffers; one error check
    # per stream at the end.  HIP events on the timing stream, which waits
    # for every call, give the device time.
    # The streams are made once; the synchronous calls below run on the
    # first (a stream's workspace, its helper stream included, is reused).
    # Each stream decodes a copy of the batch of its own, its shots rotated
    # by a quarter of the batch per stream, so that no two streams read the
    # same syndrome memory.
    pool = [torch.cuda.Stream() for _ in range(max(args.streams, 1))]
    extra_outs = [{k: torch.empty_like(v) for k, v in out.items()}
                  for _ in range(len(pool) - 1)]
    shift = [(i * shots) // max(len(pool), 1) for i in range(len(pool))]
    syns = [syn] + [torch.roll(syn, -shift[i], dims=0).contiguous() for i in range(1, len(pool))]

    def timed_async(nstreams):
        streams = pool[:nstreams]
        outs = ([out] + extra_outs)[:nstreams]
        for st, o, x in zip(streams, outs, syns):
            for _ in range(max(args.warmup, 1)):
                code.decode(x, prm, out=o, stream=st)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for st in streams:
            st.wait_stream(torch.cuda.current_stream())
        for i in range(args.steps):
            code.decode(syns[i % nstreams], prm, out=outs[i % nstreams],
                        stream=streams[i % nstreams], sync=False)
        for st in streams:
            torch.cuda.current_stream().wait_stream(st)
        e1.record()
        for st in streams:
            code.sync(st)
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - t0) / args.steps * 1e3
        same = all(bool((o["corrections"] == torch.roll(out["corrections"], -shift[i], dims=0))
                        .all().item()) for i, o in enumerate(outs) if i > 0)
        return wall_ms, e0.elapsed_time(e1) / args.steps, same

    ms_per_step, dev_ms, same_out = timed_async(args.streams)
    assert same_out, "outputs differ between streams"
    value = shots / (ms_per_step / 1e3)
    one_stream = timed_async(1) if args.streams != 1 else None
    # The same number of synchronous calls, each reporting its kernel times
    # and counts (and waiting for its results before the next is enqueued).
    stats = []
    ts = time.perf_counter()
    for _ in range(args.steps):
        stats.append(code.decode(syn, prm, out=out, stream=pool[0])["stats"])
    torch.cuda.synchronize()
    sync_ms = (time.perf_counter() - ts) / args.steps * 1e3
    kms = float(np.mean([s["kernel_ms"] for s in stats]))
    sms = float(np.mean([s["screen_ms"] for s in stats]))
    iters = float(np.mean([s["iterations"] for s in stats]))

    # Per-shot device latency and the logical error rate, from one more call.
    r = code.decode(syn, prm, out=out, latency=True, stream=pool[0])
    torch.cuda.synchronize()
    lat_us = r["latency_ticks"].cpu().numpy().astype(np.float64) / 100.0  # 100 MHz clock
    conv = out["converged"].cpu().numpy().astype(bool)
    fails = (~conv) | (out["flips"].cpu().numpy() != data["true_flips"]).any(1)

    # Roofline: the HBM floor of the call's mandatory traffic, syndromes in
    # (m bytes per shot) and corrections, logical flips and the converged
    # flag out (n + k + 1 bytes per shot), over the device time per call in
    # the timed region (HIP events on the calls' stream, the gaps between
    # calls included).  The messages of every BP run live in LDS and never
    # reach HBM.
    io_bytes_per_shot = pr.m + pr.n + pr.k + 1
    io_bytes = float(io_bytes_per_shot * shots)
    achieved = io_bytes / (dev_ms * 1e-3) / 1e9
    tr = measured_traffic()
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": tr["hbm_bytes_per_call"] if tr else None}
    assert roofline["frac"] <= 1.0, roofline

    res = {
        "metric": METRIC, "value": value, "unit": "shots/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "W2: [[144,12,12]] BB code 12-round space-time graph "
                               "(936 detectors x 8592 columns, 37303 edges), priors log-uniform "
                               "[1e-5,1e-3], 1e5 seeded syndromes, beam32_340iters, alpha 0.625",
                   "shots": shots, "beam_width": P.beam_width, "max_rounds": P.max_rounds,
                   "initial_iters": P.initial_iters, "iters_per_round": P.iters_per_round,
                   "block_threads": info["block"], "grid_blocks": info["grid"],
                   "lds_bytes": info["lds_bytes"]},
        "latency_us": {"p50": pct(lat_us, 50), "p99": pct(lat_us, 99), "p999": pct(lat_us, 99.9),
                       "max": float(lat_us.max()),
                       "what": "per shot, device clock: its processing time in the screen "
                               "(iteration 1, and iteration 2 if it needs it) plus, for a shot "
                               "the screen hands on, the persistent decoder's time from its "
                               "initial BP run to its result write"},
        "device_ms_per_step": dev_ms,
        "streams": args.streams,
        "one_stream": ({"ms_per_step": one_stream[0], "device_ms_per_step": one_stream[1],
                        "shots_per_s": shots / (one_stream[0] * 1e-3)} if one_stream else None),
        "sync_calls": {"ms_per_call": sync_ms, "shots_per_s": shots / (sync_ms * 1e-3),
                       "kernel_ms": kms,
                       "what": "the same calls made synchronously (each returns its stats "
                               "after its results are written); kernel_ms is the call's HIP-event "
                               "time on its stream"},
        "kernel_ms": kms,
        "kernels": {"screen_ms": sms, "dense_ms": kms - sms,
                    "screened_shots": int(stats[-1]["screened_shots"]),
                    "screened_at_t2": int(stats[-1]["screened2_shots"]),
                    "dense_shots": int(shots - stats[-1]["screened_shots"]),
                    "what": "synchronous calls on one stream: screen_ms from the call's "
                            "start to the end of k_screen12 (iterations 1 and 2 of the "
                            "initial run, one wave per shot); dense_ms the rest of the call, "
                            "k_batched (the persistent decoder) on the shots the screen lists"},
        "work_rate": {"edge_updates_per_s": iters * pr.nnz / (kms * 1e-3),
                      "bp_iterations_per_step": iters,
                      "what": "BP iterations x Tanner edges per second of kernel time; a work "
                              "rate, not a roofline position"},
        "io_floor": {"bytes_per_shot": io_bytes_per_shot,
                     "shots_per_s_at_peak": HBM_PEAK_GBS * 1e9 / io_bytes_per_shot},
        "ler": float(fails.mean()),
        "converged_frac": float(conv.mean()),
        "roofline": roofline,
    }
    if tr:
        res["traffic_detail"] = {k: tr[k] for k in ("hbm_bytes_per_call", "per_kernel") if k in tr}

    # The same decode from host buffers (syndromes in and results out over
    # the bus, staged by the library): the bus-inclusive rate.
    if "host" in legs:
        code.decode_host(syn_h[:1000], prm)
        th = time.perf_counter()
        code.decode_host(syn_h, prm)
        res["host_buffers_shots_per_s"] = shots / (time.perf_counter() - th)

    # Plain form: one kernel launch per BP run, beam bookkeeping on the host.
    if "plain" in legs:
        nplain = min(args.plain_shots, shots)
        prm_plain = bsd.make_params(P.max_rounds, P.beam_width, P.initial_iters,
                                    P.iters_per_round, P.num_results, P.alpha, bsd.MODE_PLAIN)
        code.decode(syn[:64].contiguous(), prm_plain)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        rp = code.decode(syn[:nplain].contiguous(), prm_plain)
        torch.cuda.synchronize()
        plain_rate = nplain / (time.perf_counter() - tp)
        # per-shot host latency (a separate call: it synchronises every shot)
        nlat = min(nplain, 2000)
        rl = code.decode(syn[:nlat].contiguous(), prm_plain, latency=True)
        plat = rl["latency_ticks"].cpu().numpy().astype(np.float64) / 100.0
        same = bool((rp["corrections"] == out["corrections"][:nplain]).all().item())
        res["plain"] = {"shots_per_s": plain_rate, "shots": nplain, "identical_to_batched": same,
                        "latency_us": {"p50": pct(plat, 50), "p99": pct(plat, 99),
                                       "p999": pct(plat, 99.9), "shots": nlat,
                                       "what": "host time per shot (its launches and "
                                               "transfers), first shots of the batch"}}
        res["batched_over_plain"] = value / plain_rate

    if "hot" in legs:
        res["hot"] = hot_leg(bsd, torch, code, pr, P)
    if "w1" in legs:
        res["w1"] = w1_leg(bsd, torch)
    if "serving" in legs:
        res["serving"] = serving(bsd, torch, code, syn_h, out["corrections"].cpu().numpy())
    if "cpu" in legs:
        res["cpu_baseline"] = cpu_baseline(pr, P, syn_h)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
