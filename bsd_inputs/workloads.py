"""The named workloads and decoder settings used by the tests and the bench.

W0  [[72,12,6]] BB code (l = m = 6), code-capacity Z noise p = 0.03, 1e4 shots,
    beam width 8, 100 min-sum iterations, scaling 0.625.
W1  [[144,12,12]] BB code (l = 6, m = 12), code-capacity Z noise p = 0.05,
    1e5 shots, beam widths 8/32/64, 100 iterations.
W2  [[144,12,12]] space-time graph over 12 noisy rounds plus a perfect
    read-out layer (936 detectors, 1728 data + 864 measurement + 6000 hook
    columns), log-uniform priors in [1e-5, 1e-3], 1e5 shots, beam32_340iters.

Decoder parameters follow the five parameters of Algorithm 3 and Table I
(max_rounds, beam_width, initial_iters, iters_per_round, num_results); a
configuration named "N iterations" spends initial_iters + max_rounds *
iters_per_round = N iterations.  "100 iterations" is split as 20 + 10 * 8.
"""
from __future__ import annotations

import hashlib
import os
from dataclasses import dataclass, asdict

import numpy as np

from . import codes, sampler


@dataclass(frozen=True)
class DecoderParams:
    max_rounds: int
    beam_width: int
    initial_iters: int
    iters_per_round: int
    num_results: int = 1
    alpha: float = 0.625

    @property
    def total_iters(self) -> int:
        return self.initial_iters + self.max_rounds * self.iters_per_round

    def as_dict(self):
        return asdict(self)


# Table I of the paper.
TABLE_I = {
    "beam8_230iters": DecoderParams(10, 8, 30, 20, 1),
    "beam32_340iters": DecoderParams(10, 32, 40, 30, 1),
    "beam64_640iters": DecoderParams(20, 64, 40, 30, 1),
    "beam64_32res_640iters": DecoderParams(20, 64, 40, 30, 32),
}


def params_100iters(beam_width: int) -> DecoderParams:
    return DecoderParams(10, beam_width, 20, 8, 1, 0.625)


@dataclass(frozen=True)
class Workload:
    name: str
    problem_key: str
    shots: int
    seed: int
    params: DecoderParams


WORKLOADS = {
    "W0": Workload("W0", "bb72_cc_p0.03", 10_000, 0, params_100iters(8)),
    "W1": Workload("W1", "bb144_cc_p0.05", 100_000, 0, params_100iters(32)),
    "W2": Workload("W2", "bb144_st12", 100_000, 0, TABLE_I["beam32_340iters"]),
    # XYZ decoding of the [[144,12,12]] code under depolarizing noise
    "W3": Workload("W3", "bb144_xyz_p0.06", 10_000, 0, params_100iters(8)),
}

_PROBLEM_CACHE: dict = {}


def problem(key: str) -> codes.Problem:
    if key in _PROBLEM_CACHE:
        return _PROBLEM_CACHE[key]
    if key == "bb72_cc_p0.03":
        pr = codes.bb_code_capacity(6, 6, 0.03, name=key)
    elif key == "bb144_cc_p0.05":
        pr = codes.bb_code_capacity(6, 12, 0.05, name=key)
    elif key == "bb144_xyz_p0.06":
        pr = codes.bb_xyz(6, 12, 0.06, name=key)
    elif key == "bb72_xyz_p0.06":
        pr = codes.bb_xyz(6, 6, 0.06, name=key)
    elif key == "bb144_st12":
        pr = codes.bb_spacetime(6, 12, rounds=12, hooks=6000, seed=0, name=key)
    else:
        raise KeyError(key)
    _PROBLEM_CACHE[key] = pr
    return pr


def problem_digest(pr: codes.Problem) -> str:
    h = hashlib.sha256()
    for a in (pr.colptr, pr.rowidx, pr.L, pr.p):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def _cache_dir() -> str:
    d = os.environ.get("BSD_INPUT_CACHE")
    if not d:
        import tempfile
        d = os.path.join(tempfile.gettempdir(), "bsd_input_cache")
    return d


def shots_for(wl: Workload, shots: int | None = None, seed: int | None = None, cache: bool = True):
    """Syndromes and true logical flips for ``shots`` shots of a workload."""
    pr = problem(wl.problem_key)
    shots = wl.shots if shots is None else shots
    seed = wl.seed if seed is None else seed
    path = os.path.join(_cache_dir(), f"{wl.problem_key}_{problem_digest(pr)[:12]}_s{seed}_n{shots}.npz")
    if cache and os.path.exists(path):
        z = np.load(path)
        return {"syndromes": z["syndromes"], "true_flips": z["true_flips"],
                "fault_shot": z["fault_shot"], "fault_col": z["fault_col"]}
    out = sampler.sample(pr, shots, seed)
    if cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            np.savez(path + ".tmp.npz", **out)
            os.replace(path + ".tmp.npz", path)
        except OSError:
            pass
    return out
