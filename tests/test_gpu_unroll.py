"""Differentiable unrolled min-sum on the GPU (forward kernel and its
hand-written adjoint, through the autograd binding), on the [[144,12,12]]
code-capacity graph with T = 25 iterations and checkpoints every 5.

Bars:
  * double precision: post(T) and the gradients with respect to Lambda and
    alpha equal the oracle's (autograd of the plain definition) to 1e-10
    relative; the gradient equals central finite differences of the GPU's
    own loss on 8 shots away from ties of the minimum;
  * the checkpoint spacing K does not change any gradient bit;
  * single precision: within 1e-4 (post) and 1e-3 (gradients) of the oracle.
"""
from __future__ import annotations

import numpy as np
import pytest

import gpu_common as gc
from bsd_inputs import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KEY = "bb144_cc_p0.05"
T = 25


@pytest.fixture(scope="module")
def bsd():
    import paper_2512_07057_amd as m
    m.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return m


@pytest.fixture(scope="module")
def setup(bsd):
    pr = gc.problem(KEY)
    code = bsd.Code.from_problem(pr)
    d = gc.samples("W1", 4096, seed=17)
    err = np.zeros((len(d["syndromes"]), pr.n), np.uint8)
    np.bitwise_xor.at(err, (d["fault_shot"], d["fault_col"]), 1)
    rng = np.random.default_rng(5)
    # distinct priors (factors 0.8 .. 1.2 at least 0.4/n apart): no tie at t = 1
    lam = np.log((1 - pr.p) / pr.p) * (0.8 + 0.4 * rng.permutation(pr.n) / pr.n)
    alpha = rng.uniform(0.5, 0.9, T)
    return pr, code, d["syndromes"], err, lam, alpha


def _gpu(bsd, code, lam, alpha, syn, err, dtype, K=5):
    lt = torch.tensor(lam, dtype=dtype, device="cuda", requires_grad=True)
    at = torch.tensor(alpha, dtype=dtype, device="cuda", requires_grad=True)
    post = bsd.unrolled_minsum(code, lt, at, torch.from_numpy(np.ascontiguousarray(syn)).cuda(), K=K)
    loss = torch.nn.functional.binary_cross_entropy_with_logits(
        -post, torch.from_numpy(err).to(post), reduction="mean")
    loss.backward()
    return (float(loss.detach()), post.detach().cpu().numpy(), lt.grad.cpu().numpy(),
            at.grad.cpu().numpy())


def _rel(a, b):
    return float(np.max(np.abs(a - b) / (1.0 + np.abs(b))))


def test_double_precision_equals_oracle_autograd(bsd, setup):
    from oracle import unrolled as U
    pr, code, syn, err, lam, alpha = setup
    g = U.Graph.from_problem(pr)
    s, e = syn[:8], err[:8]
    loss_o, post_o, gl_o, ga_o = U.loss_and_grads(g, lam, alpha, s, e)
    loss, post, gl, ga = _gpu(bsd, code, lam, alpha, s, e, torch.float64)
    gc.log("f64 rel post", _rel(post, post_o), "lam", _rel(gl, gl_o), "alpha", _rel(ga, ga_o))
    assert abs(loss - loss_o) <= 1e-12 * (1 + abs(loss_o))
    assert _rel(post, post_o) <= 1e-12
    assert _rel(gl, gl_o) <= 1e-10 and _rel(ga, ga_o) <= 1e-10


def test_double_precision_gradient_equals_finite_differences(bsd, setup):
    from oracle import unrolled as U
    pr, code, syn, err, lam, alpha = setup
    g = U.Graph.from_problem(pr)
    # the 8 of the first 24 shots farthest from a tie of the minimum
    gaps = np.array([U.min_tie_gap(g, lam, alpha, syn[b:b + 1]) for b in range(24)])
    pick = np.sort(np.argsort(-gaps)[:8])
    s, e = syn[pick], err[pick]
    gc.log("tie gaps of the chosen shots", gaps[pick].min())
    assert gaps[pick].min() > 1e-4, "no 8 shots far enough from a tie"
    _, _, gl, ga = _gpu(bsd, code, lam, alpha, s, e, torch.float64)
    h = 1e-6

    def f(l, a):
        lt = torch.tensor(l, dtype=torch.float64, device="cuda")
        at = torch.tensor(a, dtype=torch.float64, device="cuda")
        with torch.no_grad():
            post = bsd.unrolled_minsum(code, lt, at, torch.from_numpy(np.ascontiguousarray(s)).cuda())
            return float(torch.nn.functional.binary_cross_entropy_with_logits(
                -post, torch.from_numpy(e).to(post), reduction="mean"))

    rng = np.random.default_rng(1)
    for j in rng.choice(pr.n, 16, replace=False):
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


@pytest.mark.parametrize("K", [1, 3, 25])
def test_checkpoint_spacing_changes_nothing(bsd, setup, K):
    pr, code, syn, err, lam, alpha = setup
    s, e = syn[:64], err[:64]
    ref = _gpu(bsd, code, lam, alpha, s, e, torch.float64, K=5)
    got = _gpu(bsd, code, lam, alpha, s, e, torch.float64, K=K)
    for a, b in zip(got[1:], ref[1:]):
        np.testing.assert_array_equal(a, b)


def test_single_precision_close_to_oracle(bsd, setup):
    from oracle import unrolled as U
    pr, code, syn, err, lam, alpha = setup
    s, e = syn[:8], err[:8]
    _, post_o, gl_o, ga_o = U.loss_and_grads(U.Graph.from_problem(pr), lam, alpha, s, e)
    _, post, gl, ga = _gpu(bsd, code, lam, alpha, s, e, torch.float32)
    gc.log("f32 rel post", _rel(post, post_o), "lam", _rel(gl, gl_o), "alpha", _rel(ga, ga_o))
    assert _rel(post, post_o) <= 1e-4
    assert _rel(gl, gl_o) <= 1e-3 and _rel(ga, ga_o) <= 1e-3


def test_batch_of_4096_trains(bsd, setup):
    """One batch of 4096 shots in single precision: a few Adam steps on
    (alpha_t, Lambda) lower the loss."""
    pr, code, syn, err, lam, alpha = setup
    lt = torch.tensor(np.log((1 - pr.p) / pr.p), dtype=torch.float32, device="cuda", requires_grad=True)
    at = torch.full((T,), 0.625, dtype=torch.float32, device="cuda", requires_grad=True)
    st = torch.from_numpy(np.ascontiguousarray(syn)).cuda()
    et = torch.from_numpy(err).float().cuda()
    opt = torch.optim.Adam([lt, at], lr=0.02)
    losses = []
    for _ in range(8):
        opt.zero_grad()
        post = bsd.unrolled_minsum(code, lt, at, st)
        loss = torch.nn.functional.binary_cross_entropy_with_logits(-post, et, reduction="mean")
        loss.backward()
        opt.step()
        losses.append(float(loss))
    gc.log("losses", [round(x, 5) for x in losses])
    assert np.isfinite(losses).all() and losses[-1] < losses[0]


@pytest.mark.parametrize("mode", [0, 1])
def test_decoder_alpha_schedule_bitexact_vs_oracle(bsd, oracle_mod, mode):
    """The beam decoder with a per-iteration scaling schedule (the factors the
    unrolled decoder learns) equals the single-precision oracle with the
    same schedule, batched and plain."""
    pr = gc.problem(KEY)
    code = bsd.Code.from_problem(pr)
    rng = np.random.default_rng(8)
    sched = rng.uniform(0.45, 0.95, T).astype(np.float32)
    code.set_alpha_schedule(sched)
    P = workloads.params_100iters(8)
    shots = 2000 if mode == 0 else 150
    d = gc.samples("W1", shots, seed=23, hot=2)
    prm = bsd.make_params(P.max_rounds, P.beam_width, P.initial_iters, P.iters_per_round, 1,
                          P.alpha, mode, bsd.FLAG_ALPHA_SCHEDULE)
    out = code.decode(torch.from_numpy(d["syndromes"]).cuda(), prm)
    ref = oracle_mod.OracleProblem.from_problem(pr).decode_params(
        d["syndromes"], P, dtype=np.float32, threads=16, alpha_sched=sched.astype(np.float64))
    for k in ("corrections", "flips", "converged"):
        got = out[k].cpu().numpy()
        bad = np.nonzero((got != ref[k]).reshape(shots, -1).any(1))[0]
        assert bad.size == 0, f"{k} differ on shots {bad[:10]}"
    gc.log("schedule mode", mode, "deep", out["stats"]["deep_shots"])


def test_zero_iterations_gradient_is_grad_post(bsd, setup):
    """With T = 0 the output is post(0) = Lambda, so dL/dLambda is dL/dpost
    summed over shots (the oracle's autograd of the same definition)."""
    from oracle import unrolled as U
    pr, code, syn, err, lam, alpha = setup
    g = U.Graph.from_problem(pr)
    s, e = syn[:8], err[:8]
    loss_o, post_o, gl_o, ga_o = U.loss_and_grads(g, lam, alpha[:0], s, e)
    loss, post, gl, ga = _gpu(bsd, code, lam, alpha[:0], s, e, torch.float64)
    assert ga.shape == (0,) and ga_o.shape == (0,)
    np.testing.assert_array_equal(post, np.broadcast_to(lam, post.shape))
    assert _rel(gl, gl_o) <= 1e-12
    assert np.abs(gl).max() > 0
