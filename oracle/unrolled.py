"""Oracle of the differentiable unrolled min-sum decoder -- test
infrastructure only (tests, smoke check and bench CPU baseline may use it).

Plain PyTorch CPU operations in double precision, written from Appendix A:
T flooding iterations of min-sum from E(0) = Lambda (no early stop), the
detector-to-error messages of eq. (1) scaled by alpha_t at iteration t, the
posteriors of eq. (3) and the error-to-detector messages of eq. (2).  Every
message is saturated to +-llr_max, as in the decoder (a guard that never
acts on these inputs).  The output is the final posterior LLR post_j(T); the
final marginal is P(e_j = 1) = 1 / (1 + exp(post_j(T))).

Gradients with respect to alpha and Lambda are those of this definition,
computed by torch.autograd.  They are exact wherever no check has a tie
between the two smallest |E| of its neighbourhood and no E is exactly 0
(there the min-sum map is not differentiable).
"""
from __future__ import annotations

import numpy as np
import torch

LLR_MAX = 1e30


class Graph:
    """Neighbourhoods of a check matrix given in CSC form."""

    def __init__(self, m, n, colptr, rowidx):
        self.m, self.n = int(m), int(n)
        self.colptr = np.asarray(colptr, dtype=np.int64)
        self.rowidx = np.asarray(rowidx, dtype=np.int64)
        self.nnz = int(self.colptr[-1])
        self.edge_col = np.repeat(np.arange(self.n), np.diff(self.colptr))
        # edges of each row in ascending column order
        self.row_edges = [np.nonzero(self.rowidx == i)[0] for i in range(self.m)]
        self.col_edges = [np.arange(self.colptr[j], self.colptr[j + 1]) for j in range(self.n)]

    @classmethod
    def from_problem(cls, pr):
        return cls(pr.m, pr.n, pr.colptr, pr.rowidx)


def sgn(x):
    """sgn(x) = -1 iff x < 0 (a constant: no gradient)."""
    return torch.where(x < 0, -torch.ones_like(x), torch.ones_like(x))


def check_phase(g: Graph, E, syn, alpha_t, llr_max=LLR_MAX):
    """Eq. (1) times alpha_t for every edge.  E: [B, nnz]; syn: [B, m] in {0,1}."""
    D = torch.zeros_like(E)
    cols = []
    for i in range(g.m):
        ed = g.row_edges[i]
        s_fac = 1.0 - 2.0 * syn[:, i].to(E.dtype)  # (-1)^{s_i}
        for a, e in enumerate(ed):
            others = [int(x) for k, x in enumerate(ed) if k != a]
            if others:
                ev = E[:, others]
                sign = torch.prod(sgn(ev), dim=1)
                mag = torch.min(torch.abs(ev), dim=1).values
            else:  # min over an empty set
                sign = torch.ones_like(E[:, 0])
                mag = torch.full_like(E[:, 0], llr_max)
            d = alpha_t * s_fac * sign * mag
            cols.append((int(e), torch.clamp(d, -llr_max, llr_max)))
    D = torch.stack([c for _, c in sorted(cols)], dim=1) if cols else D
    return D


def variable_phase(g: Graph, D, lam, llr_max=LLR_MAX):
    """Eqs. (3) and (2): posteriors [B, n] and new messages E [B, nnz]."""
    B = D.shape[0]
    post_cols, e_cols = [], [None] * g.nnz
    for j in range(g.n):
        ed = g.col_edges[j]
        post = lam[j].expand(B)
        for e in ed:
            post = post + D[:, int(e)]
        post_cols.append(post)
        for a, e in enumerate(ed):
            x = lam[j].expand(B)
            for k, f in enumerate(ed):
                if k != a:
                    x = x + D[:, int(f)]
            e_cols[int(e)] = torch.clamp(x, -llr_max, llr_max)
    E = torch.stack(e_cols, dim=1) if g.nnz else torch.zeros((B, 0), dtype=D.dtype)
    return torch.stack(post_cols, dim=1), E


def unrolled_minsum(g: Graph, lam, alpha, syn, llr_max=LLR_MAX):
    """post(T) [B, n] for priors lam [n], scalings alpha [T], syndromes syn [B, m]."""
    syn = torch.as_tensor(np.asarray(syn), dtype=torch.int64)
    B = syn.shape[0]
    E = lam[torch.as_tensor(g.edge_col)].expand(B, g.nnz)  # E(0) = Lambda on every edge
    post = None
    for t in range(alpha.shape[0]):
        D = check_phase(g, E, syn, alpha[t], llr_max)
        post, E = variable_phase(g, D, lam, llr_max)
    if post is None:
        post = lam.expand(B, g.n)
    return post


def bce_loss(post, err):
    """Mean binary cross-entropy of the final marginals P(e_j = 1) =
    sigmoid(-post_j) against the sampled error `err` [B, n]."""
    err = torch.as_tensor(np.asarray(err), dtype=post.dtype)
    return torch.nn.functional.binary_cross_entropy_with_logits(-post, err, reduction="mean")


def loss_and_grads(g: Graph, lam0, alpha0, syn, err, grad_post=None):
    """Loss (or <grad_post, post> when grad_post is given) and its gradients
    with respect to Lambda and alpha, in double precision."""
    lam = torch.tensor(np.asarray(lam0, dtype=np.float64), requires_grad=True)
    alpha = torch.tensor(np.asarray(alpha0, dtype=np.float64), requires_grad=True)
    post = unrolled_minsum(g, lam, alpha, syn)
    if grad_post is not None:
        obj = (post * torch.as_tensor(np.asarray(grad_post), dtype=torch.float64)).sum()
    else:
        obj = bce_loss(post, err)
    obj.backward()
    # a parameter the output does not depend on (alpha when T = 0) has no .grad
    grad = lambda x: np.zeros(x.shape) if x.grad is None else x.grad.numpy().copy()
    return float(obj.detach()), post.detach().numpy(), grad(lam), grad(alpha)


def min_tie_gap(g: Graph, lam0, alpha0, syn):
    """Smallest, over iterations, checks and shots, of the gap between the two
    smallest |E| of a check's neighbourhood, and of |E| itself: how far the
    point is from the places where the map is not differentiable."""
    with torch.no_grad():
        lam = torch.tensor(np.asarray(lam0, dtype=np.float64))
        alpha = torch.tensor(np.asarray(alpha0, dtype=np.float64))
        syn_t = torch.as_tensor(np.asarray(syn), dtype=torch.int64)
        B = syn_t.shape[0]
        E = lam[torch.as_tensor(g.edge_col)].expand(B, g.nnz)
        gap = float("inf")
        for t in range(alpha.shape[0]):
            a = torch.abs(E)
            gap = min(gap, float(a.min()))
            for i in range(g.m):
                ed = g.row_edges[i]
                if len(ed) >= 2:
                    v = torch.sort(a[:, torch.as_tensor(ed)], dim=1).values
                    gap = min(gap, float((v[:, 1] - v[:, 0]).min()))
            D = check_phase(g, E, syn_t, alpha[t])
            _, E = variable_phase(g, D, lam)
    return gap
