"""Top-k accuracy measures of the paper's experiments (Section 6, top-k
queries), for evaluating results against ground-truth SimRank values.
TEST INFRASTRUCTURE.

Readings: the normaliser Z_k is the same discounted gain sum taken over the
ground-truth list, (2^s - 1) / log(i + 1) with the natural log (the base
cancels in the ratio); the Kendall difference compares every pair of returned
nodes, concordant when their returned order agrees with the order of their
true values, discordant when it contradicts it, and neither on a tie.
"""

import math

import numpy as np


def true_topk(s_row: np.ndarray, u: int, k: int) -> np.ndarray:
    """The k nodes v != u with the largest true values (ties by smaller id)."""
    v = np.array([x for x in np.lexsort((np.arange(s_row.size), -s_row)) if x != u][:k])
    return v


def precision_at_k(got, truth) -> float:
    """|V_k intersect V'_k| / k."""
    return len(set(int(x) for x in got) & set(int(x) for x in truth)) / len(truth)


def ndcg_at_k(got, truth, s_row: np.ndarray) -> float:
    """sum (2^s(u,v_i) - 1) / log(i+1) over the returned list, divided by the
    same sum over the ground-truth list (i from 1)."""
    def dcg(lst):
        return sum((2.0 ** float(s_row[v]) - 1.0) / math.log(i + 2) for i, v in enumerate(lst))
    z = dcg(truth)
    return dcg(got) / z if z > 0 else 1.0


def kendall_tau_k(got, s_row: np.ndarray) -> float:
    """(concordant - discordant) / (k(k-1)/2) over the pairs of the returned
    list, ranked as returned, against their true values."""
    k = len(got)
    if k < 2:
        return 1.0
    conc = disc = 0
    for i in range(k):
        for j in range(i + 1, k):
            a, b = float(s_row[got[i]]), float(s_row[got[j]])
            if a > b:
                conc += 1
            elif a < b:
                disc += 1
    return (conc - disc) / (k * (k - 1) / 2)
