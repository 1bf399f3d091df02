"""Learn per-iteration scalings alpha_t and prior LLRs with the differentiable
unrolled min-sum decoder, then evaluate them by the beam decoder's logical
error rate.

Training: T flooding iterations (default 25) on batches of freshly sampled
shots (default 4096), loss = mean binary cross-entropy of the final marginals
against the sampled error, Adam on (alpha, Lambda); forward and adjoint are
the library's kernels (bsd_unroll_*), checkpoints every K iterations.

Evaluation: the beam-search decoder at beam width 8 (100 iterations: 20
initial + 10 rounds x 8) on held-out shots, once with the defaults (alpha =
0.625, the true priors) and once with the learned factors (the schedule
alpha_t for iteration t of every run, the priors p_j = 1 / (1 + e^Lambda_j)),
and the same two with BP alone (the initial run of 20 iterations, no beam).
Prints one JSON line.

    python -m paper_2512_07057_amd.train --steps 300
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np


def wilson(k: int, n: int, z: float = 1.96):
    if n == 0:
        return (0.0, 1.0)
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return (max(0.0, c - h), min(1.0, c + h))


def errors_of(d, n):
    e = np.zeros((len(d["syndromes"]), n), np.uint8)
    np.bitwise_xor.at(e, (d["fault_shot"], d["fault_col"]), 1)
    return e


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--problem", default="bb144_cc_p0.05")
    ap.add_argument("--T", type=int, default=25)
    ap.add_argument("--K", type=int, default=5)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--lr", type=float, default=0.01)
    ap.add_argument("--eval-shots", type=int, default=100_000)
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--train", choices=["both", "alpha", "lambda"], default="both",
                    help="which factors to learn (the others keep their defaults)")
    args = ap.parse_args(argv)

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import torch
    import paper_2512_07057_amd as bsd
    from bsd_inputs import sampler, workloads

    pr = workloads.problem(args.problem)
    code = bsd.Code.from_problem(pr)
    lam0 = np.log((1 - pr.p) / pr.p)
    lam = torch.tensor(lam0, dtype=torch.float32, device="cuda", requires_grad=True)
    alpha = torch.full((args.T,), 0.625, dtype=torch.float32, device="cuda", requires_grad=True)
    learn = {"both": [lam, alpha], "alpha": [alpha], "lambda": [lam]}[args.train]
    for t in (lam, alpha):
        t.requires_grad_(any(t is x for x in learn))
    opt = torch.optim.Adam(learn, lr=args.lr)
    losses = []
    t0 = time.perf_counter()
    for step in range(args.steps):
        d = sampler.sample(pr, args.batch, args.seed + step)  # fresh shots every step
        syn = torch.from_numpy(d["syndromes"]).cuda()
        err = torch.from_numpy(errors_of(d, pr.n)).float().cuda()
        opt.zero_grad()
        post = bsd.unrolled_minsum(code, lam, alpha, syn, K=args.K)
        loss = torch.nn.functional.binary_cross_entropy_with_logits(-post, err, reduction="mean")
        loss.backward()
        opt.step()
        with torch.no_grad():
            alpha.clamp_(min=1e-3)
        losses.append(float(loss.detach()))
        if step % 50 == 0 or step == args.steps - 1:
            print(f"step {step} loss {losses[-1]:.6f}", file=sys.stderr, flush=True)
    train_s = time.perf_counter() - t0

    # Evaluate with the beam decoder at beam width 8.
    ev = sampler.sample(pr, args.eval_shots, 0)
    syn = torch.from_numpy(ev["syndromes"]).cuda()
    P = workloads.params_100iters(8)

    def ler(c, flags, rounds=None):
        prm = bsd.make_params(P.max_rounds if rounds is None else rounds, P.beam_width,
                              P.initial_iters, P.iters_per_round, 1, P.alpha, bsd.MODE_BATCHED, flags)
        out = c.decode(syn, prm)
        fail = (out["converged"].cpu().numpy() == 0) | \
               (out["flips"].cpu().numpy() != ev["true_flips"]).any(1)
        return int(fail.sum())

    base = ler(code, 0)
    lam_l = lam.detach().double().cpu().numpy()
    learned = bsd.Code(pr.m, pr.n, pr.colptr, pr.rowidx, 1.0 / (1.0 + np.exp(lam_l)), pr.L)
    learned.set_alpha_schedule(alpha.detach().cpu().numpy())
    lrn = ler(learned, bsd.FLAG_ALPHA_SCHEDULE)
    # The same factors in plain BP (the initial run only, no beam).
    base_bp = ler(code, 0, rounds=0)
    lrn_bp = ler(learned, bsd.FLAG_ALPHA_SCHEDULE, rounds=0)
    n = args.eval_shots
    res = {
        "problem": args.problem, "train": args.train, "T": args.T, "K": args.K, "batch": args.batch,
        "steps": args.steps,
        "lr": args.lr, "train_seconds": train_s, "loss_first": losses[0], "loss_last": losses[-1],
        "alpha_learned": [round(float(a), 4) for a in alpha.detach().cpu().numpy()],
        "lambda_change_rms": float(np.sqrt(np.mean((lam_l - lam0) ** 2))),
        "eval_shots": n, "decoder": "beam 8, 20 + 10 x 8 iterations",
        "ler_default": base / n, "ler_default_interval": wilson(base, n),
        "ler_learned": lrn / n, "ler_learned_interval": wilson(lrn, n),
        "bp_only_iters": P.initial_iters,
        "ler_bp_only_default": base_bp / n, "ler_bp_only_learned": lrn_bp / n,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
