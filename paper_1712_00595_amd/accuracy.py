"""Accuracy of an approximate score vector against an exact one.

The experiments' accuracy section measures an approximate RWR vector by its
L1 distance to the exact vector and its ranking by Spearman's rank
correlation.  This module computes both on the host with numpy, plus the
overlap of the top-k node sets (the nodes a recommender would return).

Ties: Spearman uses average ranks (the textbook definition: the Pearson
correlation of the two rank vectors); top-k breaks ties by the smaller node
id, so the set is unique.
"""

from __future__ import annotations

import numpy as np


def l1(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).sum())


def average_ranks(x) -> np.ndarray:
    """Ranks 1..n of x in ascending order; equal values share the mean of the
    ranks they span."""
    x = np.asarray(x, np.float64)
    n = x.shape[0]
    order = np.argsort(x, kind="stable")
    xs = x[order]
    ranks = np.empty(n, np.float64)
    # runs of equal values in sorted order
    starts = np.flatnonzero(np.r_[True, xs[1:] != xs[:-1]])
    ends = np.r_[starts[1:], n]
    mean_rank = (starts + ends - 1) / 2.0 + 1.0
    run_of = np.repeat(np.arange(starts.shape[0]), ends - starts)
    ranks[order] = mean_rank[run_of]
    return ranks


def spearman(a, b) -> float:
    """Spearman's rank correlation of a and b (1 = same order, -1 = reversed).
    nan when either vector is constant."""
    ra = average_ranks(a)
    rb = average_ranks(b)
    ra -= ra.mean()
    rb -= rb.mean()
    den = np.sqrt((ra * ra).sum() * (rb * rb).sum())
    if den == 0.0:
        return float("nan")
    return float((ra * rb).sum() / den)


def top_k(x, k: int) -> np.ndarray:
    """Ids of the k largest entries (ties: smaller id first), best first."""
    x = np.asarray(x, np.float64)
    k = min(int(k), x.shape[0])
    # lexicographic: descending value, then ascending id
    order = np.lexsort((np.arange(x.shape[0]), -x))
    return order[:k]


def topk_overlap(a, b, k: int) -> float:
    """|top_k(a) ∩ top_k(b)| / k."""
    k = min(int(k), np.asarray(a).shape[0])
    if k <= 0:
        return float("nan")
    return len(np.intersect1d(top_k(a, k), top_k(b, k), assume_unique=True)) / float(k)


def compare(scores, reference, ks=(10, 100, 1000)) -> dict:
    """L1, Spearman and top-k overlaps of `scores` against `reference`."""
    out = {"l1": l1(scores, reference), "spearman": spearman(scores, reference)}
    for k in ks:
        out[f"top{k}_overlap"] = topk_overlap(scores, reference, k)
    return out
