"""Rank-accuracy metrics (L1, Spearman with average ranks, top-k overlap)
against scipy's independent implementation and hand-worked cases."""

import numpy as np
import pytest
from scipy import stats

from paper_1712_00595_amd import accuracy


def test_average_ranks_match_scipy_with_ties():
    rng = np.random.default_rng(1)
    for _ in range(20):
        x = rng.integers(0, 6, size=50).astype(np.float64)  # many ties
        assert np.array_equal(accuracy.average_ranks(x), stats.rankdata(x, method="average"))


def test_spearman_matches_scipy():
    rng = np.random.default_rng(2)
    for n in (5, 37, 1000):
        a = rng.random(n)
        b = a + 0.3 * rng.random(n)
        assert accuracy.spearman(a, b) == pytest.approx(stats.spearmanr(a, b).statistic, abs=1e-12)
        # ties on both sides
        at = np.round(a * 4)
        bt = np.round(b * 4)
        assert accuracy.spearman(at, bt) == pytest.approx(stats.spearmanr(at, bt).statistic, abs=1e-12)


def test_spearman_special_cases():
    x = np.array([0.1, 0.5, 0.2, 0.9])
    assert accuracy.spearman(x, x) == pytest.approx(1.0)
    assert accuracy.spearman(x, -x) == pytest.approx(-1.0)
    # a monotone map keeps the ranks
    assert accuracy.spearman(x, np.exp(5 * x)) == pytest.approx(1.0)
    assert np.isnan(accuracy.spearman(np.ones(4), x))
    # hand-worked: ranks (1,2,3,4) vs (2,1,4,3): d^2 = 4, rho = 1 - 6*4/(4*15)
    assert accuracy.spearman([1, 2, 3, 4], [2, 1, 4, 3]) == pytest.approx(1 - 24 / 60)


def test_top_k_and_overlap():
    a = np.array([0.3, 0.9, 0.3, 0.1, 0.9])
    # descending value, ties by smaller id
    assert accuracy.top_k(a, 3).tolist() == [1, 4, 0]
    b = np.array([0.9, 0.8, 0.7, 0.6, 0.5])
    assert accuracy.top_k(b, 2).tolist() == [0, 1]
    assert accuracy.topk_overlap(a, b, 2) == pytest.approx(0.5)  # {1,4} vs {0,1}
    assert accuracy.topk_overlap(a, a, 5) == 1.0
    assert accuracy.topk_overlap(b, -b, 2) == 0.0
    assert accuracy.topk_overlap(a, b, 99) == 1.0  # k capped at n


def test_compare_fields():
    rng = np.random.default_rng(3)
    ref = rng.random(2000)
    ref /= ref.sum()
    approx = ref + 1e-9 * rng.standard_normal(2000)
    out = accuracy.compare(approx, ref, ks=(10, 100))
    assert out["l1"] == pytest.approx(np.abs(approx - ref).sum())
    assert out["spearman"] > 0.99
    assert set(out) == {"l1", "spearman", "top10_overlap", "top100_overlap"}
