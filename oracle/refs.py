"""Independent reference computations used to pin the oracle.  TEST
INFRASTRUCTURE ONLY.

None of these reuse the oracle's PROBE or walk code; each computes SimRank or
a first-meeting probability by a different route, so that a mistake in the
oracle (a dropped term, a wrong exclusion index, a wrong scale) shows up as a
disagreement.

  power_method          Eq. (related-simrank): S <- (c P^T S P) v I from S = I
  exact_simrank         direct linear solve of the SimRank equations (Eq. 1)
  first_meeting_bruteforce  Definition of the first-meeting probability,
                        by enumerating every in-walk of v of the right length
  expected_estimate     exact expectation of the truncated estimator: the sum
                        over t = 2..L of Pr[two sqrt(c)-walks first meet at
                        step t] (Eq. single-simrank-meet), by dynamic
                        programming over node pairs
  pair_monte_carlo      Section 2.2 pairwise Monte Carlo estimate
"""

from __future__ import annotations

import itertools
import math

import numpy as np


def in_lists(n, src, dst):
    ins = [[] for _ in range(n)]
    for a, b in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()):
        ins[b].append(a)
    return [sorted(x) for x in ins]


def out_lists(n, src, dst):
    outs = [[] for _ in range(n)]
    for a, b in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()):
        outs[a].append(b)
    return [sorted(x) for x in outs]


def transition(n, src, dst) -> np.ndarray:
    """P[x, v] = 1/|I(v)| when x is an in-neighbour of v (column-stochastic
    over in-neighbours; columns of nodes with no in-neighbour are zero)."""
    P = np.zeros((n, n))
    ins = in_lists(n, src, dst)
    for v in range(n):
        for x in ins[v]:
            P[x, v] = 1.0 / len(ins[v])
    return P


def power_method(n, src, dst, c, iters=None, tol=1e-12) -> np.ndarray:
    """All-pairs SimRank by S <- max(c P^T S P, I) starting from S = I
    (Eq. related-simrank).  With iters=None it runs ceil(ln tol / ln c)
    iterations, which bounds the error by tol since the error after t
    iterations is at most c^(t+1)."""
    if iters is None:
        iters = int(math.ceil(math.log(tol) / math.log(c)))
    P = transition(n, src, dst)
    S = np.eye(n)
    for _ in range(iters):
        S = np.maximum(c * (P.T @ S @ P), np.eye(n))
    return S


def exact_simrank(n, src, dst, c) -> np.ndarray:
    """Solves the SimRank equations s(a,a) = 1,
    s(a,b) = c/(|I(a)||I(b)|) sum_{x in I(a), y in I(b)} s(x,y) for a != b
    (zero when either in-set is empty) as one n^2 x n^2 linear system."""
    ins = in_lists(n, src, dst)
    N = n * n
    A = np.eye(N)
    rhs = np.zeros(N)
    for a in range(n):
        for b in range(n):
            r = a * n + b
            if a == b:
                rhs[r] = 1.0
                continue
            if not ins[a] or not ins[b]:
                continue
            f = c / (len(ins[a]) * len(ins[b]))
            for x in ins[a]:
                for y in ins[b]:
                    A[r, x * n + y] -= f
    return np.linalg.solve(A, rhs).reshape(n, n)


def first_meeting_bruteforce(n, src, dst, path, c) -> np.ndarray:
    """P(v, (u_1..u_i)) for every v != u_1 (Definition of first-meeting
    probability): the probability that a sqrt(c)-walk W(v) = (v_1, v_2, ...)
    has v_i = u_i and v_t != u_t for t = 1..i-1.  Enumerates every sequence
    of in-neighbour choices of length i-1; each step survives with
    probability sqrt(c) and picks one of |I(.)| in-neighbours."""
    ins = in_lists(n, src, dst)
    i = len(path)
    sc = math.sqrt(c)
    out = np.zeros(n)
    for v in range(n):
        if v == path[0]:
            continue
        total = 0.0

        def rec(node, t, prob):
            # node = v_t (1-based t); it already differs from u_t for t < i
            nonlocal total
            if t == i:
                if node == path[i - 1]:
                    total += prob
                return
            if node == path[t - 1]:
                return
            for x in ins[node]:
                rec(x, t + 1, prob * sc / len(ins[node]))

        rec(v, 1, 1.0)
        out[v] = total
    return out


def expected_estimate(n, src, dst, u, c, L) -> np.ndarray:
    """E[s^(u, v)] of the unpruned estimator whose u-walks are cut at L
    nodes: sum over t = 2..L of Pr[W(u), W(v) first meet at step t]
    (Eq. single-simrank-meet).  Both walks move together; a pair of distinct
    nodes (x, y) moves to (x', y') with probability c/(|I(x)||I(y)|) for each
    in-neighbour pair and is absorbed when x' = y'."""
    ins = in_lists(n, src, dst)
    out = np.zeros(n)
    for v in range(n):
        if v == u:
            continue
        dist = {(u, v): 1.0}
        met = 0.0
        for _t in range(2, L + 1):
            nxt = {}
            for (x, y), p in dist.items():
                if not ins[x] or not ins[y]:
                    continue
                f = p * c / (len(ins[x]) * len(ins[y]))
                for a in ins[x]:
                    for b in ins[y]:
                        if a == b:
                            met += f
                        else:
                            nxt[(a, b)] = nxt.get((a, b), 0.0) + f
            dist = nxt
        out[v] = met
    return out


def pair_monte_carlo(n, src, dst, u, v, c, r, seed=0) -> float:
    """Section 2.2: fraction of r pairs of independent sqrt(c)-walks from u
    and v that meet (their t-th nodes coincide for some t)."""
    ins = in_lists(n, src, dst)
    rng = np.random.default_rng(seed)
    sc = math.sqrt(c)
    hits = 0
    for _ in range(r):
        a, b = u, v
        while True:
            if a == b:
                hits += 1
                break
            if rng.random() <= 1 - sc or rng.random() <= 1 - sc or not ins[a] or not ins[b]:
                break
            a = ins[a][rng.integers(len(ins[a]))]
            b = ins[b][rng.integers(len(ins[b]))]
    return hits / r


def random_graph(n, p, seed):
    """Small seeded digraph for brute-force checks (edges i->j, i != j, kept
    with probability p)."""
    rng = np.random.default_rng(seed)
    src, dst = [], []
    for a, b in itertools.permutations(range(n), 2):
        if rng.random() < p:
            src.append(a)
            dst.append(b)
    return np.array(src, np.int32), np.array(dst, np.int32)
