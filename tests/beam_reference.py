"""A second, independent statement of the beam controller (test helper).

Algorithm 3 with the ordering and pruning of Appendix B, written directly
from the text: paths are explored in descending order of their reliability
score, each explored path is branched on its least reliable node with the
value 0 and then 1, and the children of a round go into a bounded
``next_set`` on the fly -- a child is inserted while the set has fewer than
``beam_width`` paths, and afterwards only if its score is strictly greater
than the smallest score in the set, which is then ejected.  The first child
whose hard decision satisfies the syndrome is returned (num_results = 1);
with num_results > 1 distinct solutions are collected and the lightest
returned.

The per-run arithmetic (one masked BP run, Algorithm 2; the score and least
reliable node of a finished run) comes from the oracle's ``bp_run`` and
``score``, which the tree max-marginal, punctured-graph, warm-start and
closed-form tests pin on their own.  Only the control flow is restated
here; it shares no code with the oracle's controller.

Readings where the text is silent (the same ones the decoder documents):
equal exploration scores go in generation order, the child of the k-th
explored parent with value v having generation 2k + v; among equal minima
the latest generated is ejected; a path with no unmasked node has no
children; on failure the output is the last hard decision (fixed values
filled in) of the best path of the final set, or of the initial run when
that set is empty or there were no rounds.
"""
from __future__ import annotations

import numpy as np


def _solution(ehat, pairs):
    e = np.array(ehat, dtype=np.uint8, copy=True)
    for c, v in pairs:
        e[c] = v
    return e


def beam_decode(op, s, max_rounds, beam_width, initial_iters, iters_per_round,
                num_results=1, alpha=0.625, dtype=np.float32, trace=None):
    """Decode one syndrome; returns (ehat, converged, info).

    ``info`` holds the round and generation of the returned child (0, 0 for
    the initial run; -1 if none converged) and the number of BP runs.
    ``trace`` (a list, optional) receives one entry per round: the explored
    parents' (generation, score) in exploration order, every child's
    (generation, score) in the order generated, and the survivors'
    generations.
    """
    runs = 1
    results, weights, origins = [], [], []
    wt = np.log((1 - op.p) / op.p)

    def offer(e, rnd, gen):
        for r in results:
            if np.array_equal(r, e):
                return False
        results.append(e)
        weights.append(float(np.sum(wt[e.astype(bool)])))
        origins.append((rnd, gen))
        return len(results) >= num_results

    def lightest():
        best = 0
        for q in range(1, len(results)):
            if weights[q] < weights[best]:
                best = q
        return results[best], True, {"round": origins[best][0], "gen": origins[best][1],
                                     "runs": runs}

    r0 = op.bp_run(s, initial_iters, alpha=alpha, stop=True, dtype=dtype)
    if r0["converged"] and offer(_solution(r0["ehat"], []), 0, 0):
        return lightest()
    npos, _ = op.score(r0["sum_llr"], [], r0["iters"], dtype=dtype)
    current = [{"e": r0["e"], "pairs": [], "next_pos": npos, "score": 0.0, "gen": 0,
                "ehat": _solution(r0["ehat"], [])}]

    for rnd in range(1, max_rounds + 1):
        if not current:
            break
        # descending score; ties in generation order
        explore = sorted(current, key=lambda p: p["gen"])
        explore = sorted(explore, key=lambda p: p["score"], reverse=True)
        nxt, children = [], []
        for k, par in enumerate(explore):
            if par["next_pos"] < 0:
                continue
            for v in (0, 1):
                pairs = par["pairs"] + [(par["next_pos"], v)]
                rr = op.bp_run(s, iters_per_round, alpha=alpha, e_start=par["e"], pairs=pairs,
                               stop=True, dtype=dtype)
                runs += 1
                e_hat = _solution(rr["ehat"], pairs)
                if rr["converged"] and offer(e_hat, rnd, 2 * k + v):
                    return lightest()
                npos, sc = op.score(rr["sum_llr"], pairs, rr["iters"], dtype=dtype)
                child = {"e": rr["e"], "pairs": pairs, "next_pos": npos, "score": float(sc),
                         "gen": 2 * k + v, "ehat": e_hat}
                children.append((child["gen"], child["score"]))
                if len(nxt) < beam_width:
                    nxt.append(child)
                    continue
                low = min(c["score"] for c in nxt)
                if child["score"] > low:
                    victim = max((q for q in range(len(nxt)) if nxt[q]["score"] == low),
                                 key=lambda q: nxt[q]["gen"])
                    del nxt[victim]
                    nxt.append(child)
        if trace is not None:
            trace.append({"explored": [(p["gen"], p["score"]) for p in explore],
                          "children": children, "kept": sorted(c["gen"] for c in nxt)})
        current = nxt

    if results:
        return lightest()
    info = {"round": -1, "gen": -1, "runs": runs}
    if current and max_rounds > 0:
        best = sorted(current, key=lambda p: p["gen"])
        best = sorted(best, key=lambda p: p["score"], reverse=True)[0]
        return best["ehat"], False, info
    return _solution(r0["ehat"], []), False, info
