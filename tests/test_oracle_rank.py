"""Pins of the oracle's ranking output (Section 6, "Vertex Ranking"): the
vertex ranking by score and Kendall's tau-b between two score vectors.

tau-b is pinned to scipy's independent implementation (Knight's O(n log n)
algorithm) on inputs with many ties, to hand-counted examples and closed
forms, and to the invariances that any correct rank correlation has.  The
ranking is pinned by the properties that define it uniquely: a permutation,
scores non-decreasing along it, equal scores in id order.
"""
import math

import numpy as np
import pytest
import scipy.stats

import oracle


def _tie_heavy(n, levels, seed):
    rng = np.random.default_rng(seed)
    a = rng.integers(0, levels, n).astype(np.float64)
    b = a + rng.integers(0, max(2, levels // 4), n)  # correlated, with ties in both
    return a, b


@pytest.mark.parametrize("n,levels,seed", [(2, 2, 0), (17, 3, 1), (300, 20, 2), (1000, 1000, 3),
                                           (1500, 7, 4), (800, 100000, 5)])
def test_tau_b_matches_scipy(n, levels, seed):
    a, b = _tie_heavy(n, levels, seed)
    ref = scipy.stats.kendalltau(a, b, variant="b").statistic
    got = oracle.kendall_tau_b(a, b)
    if math.isnan(ref):
        assert math.isnan(got)
    else:
        assert abs(got - ref) <= 1e-13, (got, ref)


def test_tau_b_hand_counted():
    # one discordant pair (the middle swap) out of six
    assert oracle.kendall_counts([1, 2, 3, 4], [1, 3, 2, 4]) == (5, 1, 0, 0, 0)
    assert oracle.kendall_tau_b([1, 2, 3, 4], [1, 3, 2, 4]) == 4 / 6
    # (0,1) tied in a, (0,2) concordant, (1,2) tied in b: 1 / sqrt(2 * 2)
    assert oracle.kendall_counts([1, 1, 2], [1, 2, 2]) == (1, 0, 1, 1, 0)
    assert oracle.kendall_tau_b([1, 1, 2], [1, 2, 2]) == 0.5
    # a pair tied in both counts in both tie totals and in neither n_c nor n_d
    assert oracle.kendall_counts([5, 5, 1], [2, 2, 0]) == (2, 0, 1, 1, 1)


def test_tau_b_closed_forms():
    x = np.random.default_rng(7).permutation(500).astype(np.float64)
    assert oracle.kendall_tau_b(x, x) == 1.0
    assert oracle.kendall_tau_b(x, -x) == -1.0
    assert math.isnan(oracle.kendall_tau_b(np.ones(10), x[:10]))
    assert math.isnan(oracle.kendall_tau_b([3.0], [1.0]))  # no pairs
    # a single transposition of adjacent ranks: n_d = 1 of n(n-1)/2 pairs
    n = 40
    y = np.arange(n, dtype=np.float64)
    y[[10, 11]] = y[[11, 10]]
    p = n * (n - 1) // 2
    assert oracle.kendall_tau_b(np.arange(n, dtype=np.float64), y) == (p - 2) / p


def test_tau_b_invariances():
    a, b = _tie_heavy(400, 30, 9)
    t = oracle.kendall_tau_b(a, b)
    assert oracle.kendall_tau_b(b, a) == t
    assert oracle.kendall_tau_b(a, -b) == -t
    assert oracle.kendall_tau_b(np.exp(a / 10.0), b) == t      # strictly increasing map
    perm = np.random.default_rng(3).permutation(a.size)
    assert oracle.kendall_tau_b(a[perm], b[perm]) == t          # relabelling the vertices
    nc, nd, ta, tb, tab = oracle.kendall_counts(a, b)
    assert nc + nd + ta + tb - tab == a.size * (a.size - 1) // 2


def _check_ranking(score, descending):
    s = np.asarray(score, np.float64)
    order, rank = oracle.ranking(s, descending)
    n = s.size
    assert sorted(order.tolist()) == list(range(n))
    assert np.array_equal(rank[order], np.arange(n))
    key = -s[order] if descending else s[order]
    for i in range(n - 1):
        assert key[i] <= key[i + 1]
        if key[i] == key[i + 1]:
            assert order[i] < order[i + 1]


@pytest.mark.parametrize("descending", [False, True])
def test_ranking_properties(descending):
    rng = np.random.default_rng(11)
    for n, levels in ((0, 1), (1, 1), (9, 3), (1000, 50), (1000, 10**9)):
        _check_ranking(rng.integers(0, levels, n) / 7.0, descending)
    _check_ranking([0.0, -0.0, np.inf, -np.inf, 1e-300, -1e-300, 0.0, np.inf], descending)


def test_ranking_examples():
    s = [3.0, -0.0, 0.0, 1.0, 3.0]
    order, rank = oracle.ranking(s)
    assert order.tolist() == [1, 2, 3, 0, 4] and rank.tolist() == [3, 0, 1, 2, 4]
    order, _ = oracle.ranking(s, descending=True)
    assert order.tolist() == [0, 4, 3, 1, 2]
    with pytest.raises(ValueError):
        oracle.ranking([1.0, float("nan")])
