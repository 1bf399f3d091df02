"""Pins of the unrolled min-sum oracle (oracle/unrolled.py), on the CPU.

* Its forward pass is the BP of the main oracle: T iterations without early
  stop give the same posteriors, with one scaling or with a per-iteration
  schedule (chaining one-iteration warm-started runs).
* A hand-derived one-check case fixes the values and the derivatives.
* Its gradients equal central finite differences of the loss (double
  precision) at points away from ties of the minimum.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

from bsd_inputs import codes, workloads
from oracle import unrolled as U


def errors_of(d, n):
    """The sampled error of each shot as a dense 0/1 matrix."""
    e = np.zeros((len(d["syndromes"]), n), np.uint8)
    np.bitwise_xor.at(e, (d["fault_shot"], d["fault_col"]), 1)
    return e


@pytest.fixture(scope="module")
def w0():
    pr = workloads.problem("bb72_cc_p0.03")
    d = workloads.shots_for(workloads.WORKLOADS["W0"], shots=64, seed=4, cache=False)
    return pr, U.Graph.from_problem(pr), d


def test_forward_equals_bp_of_the_main_oracle(oracle_mod, w0):
    pr, g, d = w0
    op = oracle_mod.OracleProblem.from_problem(pr)
    lam = np.log((1 - pr.p) / pr.p)
    T = 7
    syn = d["syndromes"][:6]
    post = U.unrolled_minsum(g, torch.tensor(lam), torch.full((T,), 0.625, dtype=torch.float64), syn)
    for b in range(len(syn)):
        ref = op.bp_run(syn[b], T, alpha=0.625, stop=False)
        assert ref["iters"] == T
        np.testing.assert_allclose(post[b].numpy(), ref["post"], rtol=1e-13, atol=1e-12)


def test_schedule_equals_chained_warm_started_iterations(oracle_mod, w0):
    pr, g, d = w0
    op = oracle_mod.OracleProblem.from_problem(pr)
    rng = np.random.default_rng(2)
    lam = np.log((1 - pr.p) / pr.p) * rng.uniform(0.7, 1.3, pr.n)
    alpha = rng.uniform(0.4, 1.0, 5)
    syn = d["syndromes"][:4]
    post = U.unrolled_minsum(g, torch.tensor(lam), torch.tensor(alpha), syn)
    # the main oracle takes priors p; Lambda = log((1-p)/p) -> p = 1/(1+e^Lambda)
    op2 = oracle_mod.OracleProblem.from_problem(
        type("P", (), {"m": pr.m, "n": pr.n, "colptr": pr.colptr, "rowidx": pr.rowidx,
                       "p": 1.0 / (1.0 + np.exp(lam)), "L": pr.L, "k": pr.k})())
    for b in range(len(syn)):
        e = None
        for t, a in enumerate(alpha):
            r = op2.bp_run(syn[b], 1, alpha=float(a), e_start=e, stop=False)
            e = r["e"]
        np.testing.assert_allclose(post[b].numpy(), r["post"], rtol=1e-12, atol=1e-11)


def test_one_check_closed_form():
    # one check over three degree-1 columns, Lambda = (1, 2, 3), s = 1, one iteration:
    # post_0 = 1 - a*min(2,3), post_1 = 2 - a*min(1,3), post_2 = 3 - a*min(1,2)
    g = U.Graph(1, 3, [0, 1, 2, 3], [0, 0, 0])
    lam = torch.tensor([1.0, 2.0, 3.0], dtype=torch.float64, requires_grad=True)
    a = torch.tensor([0.5], dtype=torch.float64, requires_grad=True)
    post = U.unrolled_minsum(g, lam, a, np.array([[1]], np.uint8))
    np.testing.assert_allclose(post.detach().numpy(), [[0.0, 1.5, 2.5]])
    post[0, 0].backward()
    np.testing.assert_allclose(lam.grad.numpy(), [1.0, -0.5, 0.0])
    np.testing.assert_allclose(a.grad.numpy(), [-2.0])


@pytest.mark.parametrize("T", [1, 4, 9])
def test_gradients_equal_central_differences(w0, T):
    pr, g, d = w0
    rng = np.random.default_rng(T)
    lam = np.log((1 - pr.p) / pr.p) * rng.uniform(0.6, 1.4, pr.n)
    alpha = rng.uniform(0.4, 1.0, T)
    syn = d["syndromes"][:3]
    err = errors_of(d, pr.n)[:3]
    gap = U.min_tie_gap(g, lam, alpha, syn)
    assert gap > 1e-5, "test point too close to a tie"
    loss, _, gl, ga = U.loss_and_grads(g, lam, alpha, syn, err)
    h = 1e-6

    def f(l, a):
        with torch.no_grad():
            return float(U.bce_loss(U.unrolled_minsum(g, torch.tensor(l), torch.tensor(a), syn), err))

    for j in rng.choice(pr.n, 12, replace=False):
        lp, lm = lam.copy(), lam.copy()
        lp[j] += h
        lm[j] -= h
        fd = (f(lp, alpha) - f(lm, alpha)) / (2 * h)
        assert abs(fd - gl[j]) <= 1e-6 * (1 + abs(fd)), (j, fd, gl[j])
    for t in range(T):
        ap, am = alpha.copy(), alpha.copy()
        ap[t] += h
        am[t] -= h
        fd = (f(lam, ap) - f(lam, am)) / (2 * h)
        assert abs(fd - ga[t]) <= 1e-6 * (1 + abs(fd)), (t, fd, ga[t])


def test_constant_schedule_equals_single_alpha(oracle_mod, w0):
    pr, g, d = w0
    op = oracle_mod.OracleProblem.from_problem(pr)
    syn = d["syndromes"][:64]
    a = op.decode(syn, 6, 8, 20, 8, alpha=0.625, dtype=np.float32)
    b = op.decode(syn, 6, 8, 20, 8, alpha=0.9, dtype=np.float32, alpha_sched=[0.625] * 5)
    for k in ("corrections", "flips", "converged"):
        np.testing.assert_array_equal(a[k], b[k])


def test_schedule_initial_run_is_unrolled_minsum_stopped_at_a_solution(oracle_mod, w0):
    """max_rounds = 0 with a schedule: the decision is that of the first
    iteration whose hard decision satisfies He = s (eq. (4) on the unrolled
    posteriors), else of the last iteration."""
    pr, g, d = w0
    op = oracle_mod.OracleProblem.from_problem(pr)
    rng = np.random.default_rng(11)
    alpha = rng.uniform(0.4, 1.0, 6)
    T = 9  # beyond the schedule: the last entry repeats
    sched_full = np.concatenate([alpha, np.full(T - len(alpha), alpha[-1])])
    syn = d["syndromes"][:12]
    lam = torch.tensor(np.log((1 - pr.p) / pr.p))
    H = np.zeros((pr.m, pr.n), np.int64)
    for j in range(pr.n):
        H[pr.rowidx[pr.colptr[j]:pr.colptr[j + 1]], j] = 1
    got = op.decode(syn, 0, 8, T, 8, dtype=np.float64, alpha_sched=alpha)
    for b in range(len(syn)):
        want = None
        for t in range(1, T + 1):
            post = U.unrolled_minsum(g, lam, torch.tensor(sched_full[:t]), syn[b:b + 1])[0].numpy()
            eh = (post <= 0).astype(np.int64)
            if ((H @ eh) % 2 == syn[b]).all():
                want = (eh, 1)
                break
        if want is None:
            want = (eh, 0)
        np.testing.assert_array_equal(got["corrections"][b], want[0])
        assert got["converged"][b] == want[1]
