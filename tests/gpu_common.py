"""Shared helpers of the GPU tests (inputs, oracle runs, checks)."""
from __future__ import annotations

import functools
import math
import sys

import numpy as np

from bsd_inputs import sampler, workloads


def log(*a):
    print(*a, flush=True, file=sys.stderr)


@functools.lru_cache(maxsize=None)
def problem(key):
    return workloads.problem(key)


def hot_problem(pr, mult):
    """Same graph and decoder priors, faults drawn at mult x the priors."""
    return type("Hot", (), {"p": np.minimum(pr.p * mult, 0.4), "colptr": pr.colptr,
                            "rowidx": pr.rowidx, "m": pr.m, "k": pr.k, "L": pr.L})()


@functools.lru_cache(maxsize=None)
def samples(name, shots, seed=0, hot=0):
    wl = workloads.WORKLOADS[name]
    pr = problem(wl.problem_key)
    if hot:
        return sampler.sample(hot_problem(pr, hot), shots, seed)
    return workloads.shots_for(wl, shots=shots, seed=seed, cache=False)


def wilson(k, n, z=1.959963984540054):
    if n == 0:
        return (0.0, 1.0)
    ph = k / n
    den = 1 + z * z / n
    c = (ph + z * z / (2 * n)) / den
    h = z * math.sqrt(ph * (1 - ph) / n + z * z / (4 * n * n)) / den
    return (max(0.0, c - h), min(1.0, c + h))


def failures(out, true_flips):
    conv = np.asarray(out["converged"]).astype(bool)
    fl = np.asarray(out["flips"])
    return (~conv) | (fl != true_flips).any(axis=1)


def clean_mask(diag, post_eps=1e-3, gap_eps=1e-3, score_rel=1e-5):
    """Shots whose double-precision trajectory has no near-tie in a decision."""
    return ((diag["min_abs_post"] >= post_eps) & (diag["min_nextpos_gap"] >= gap_eps)
            & (diag["min_score_gap_rel"] >= score_rel))


def params_for(bsd, P, mode=0):
    return bsd.make_params(P.max_rounds, P.beam_width, P.initial_iters, P.iters_per_round,
                           P.num_results, P.alpha, mode)
