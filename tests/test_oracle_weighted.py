"""Pins for the oracle on weighted graphs (Section 2 allows non-negative edge
weights; G's edges then weigh alpha w in G*, the edges to u* weigh 1).

What fixes the weighted sampler, independently of its own code:
  * With every weight 1 the weighted rule is the unweighted one, tree for tree
    (the running weight sums are exact integers).
  * A uniform spanning tree of the weighted G* has P(T) proportional to the
    product of its edge weights; checked by chi-square against brute-force
    enumeration of all spanning trees.
  * Kirchhoff: P[{u*, v} in T] = Omega_vv for Omega = (alpha L_w + I)^{-1};
    exact rationals vs the enumerated tree weights vs the sampled frequency.
  * The closed form of a single weighted edge, zero-weight edges never taken,
    and the (eps, delta) guarantee against the dense forest matrix.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle
import inputs


def test_unit_weights_are_the_unweighted_sampler():
    g = inputs.erdos_renyi(90, 0.06, 4)
    gw = inputs.CSRGraph(g.n, g.row_ptr, g.col_idx, "unit", np.ones(g.col_idx.size))
    a = oracle.sample(g, 0.7, 123, 5, 60, stream=3, per_tree=True)
    b = oracle.sample(gw, 0.7, 123, 5, 60, stream=3, per_tree=True)
    assert np.array_equal(a.parents, b.parents)
    assert np.array_equal(a.tree_visits, b.tree_visits)
    assert np.array_equal(a.R, b.R)
    assert np.array_equal(a.digests, b.digests)
    for d in (0, 1, 2, 7, 1000):
        assert oracle.root_threshold_w(0.7, float(d)) == oracle.root_threshold(0.7, d)


@pytest.mark.parametrize("name,n,edges,alpha", [
    ("triangle", 3, [(0, 1, 0.5), (1, 2, 2.0), (0, 2, 3.25)], 1.5),
    ("path_isolated", 4, [(0, 1, 0.25), (1, 2, 4.0)], 1.0),
    ("star", 4, [(0, 1, 1.0), (0, 2, 0.125), (0, 3, 6.0)], 0.5),
    ("cycle4", 4, [(0, 1, 3.0), (1, 2, 0.5), (2, 3, 1.0), (3, 0, 2.0)], 2.0),
])
def test_weighted_tree_distribution(name, n, edges, alpha):
    g = inputs.from_weighted_edge_list(n, edges, name)
    trees = oracle.spanning_trees(g)
    a = Fraction(alpha)
    w = np.array([float(a ** k * wp) for _, k, wp in trees])
    probs = w / w.sum()
    index = {t: i for i, (t, _, _) in enumerate(trees)}
    n_trees = 60000
    res = oracle.sample(g, alpha, 17, 0, n_trees, per_tree=True)
    counts = np.zeros(len(trees), np.int64)
    for row in res.parents:
        counts[index[tuple(int(x) for x in row)]] += 1
    _, p = stats.chisquare(counts, n_trees * probs)
    assert p > 1e-3, (name, counts, n_trees * probs)


def test_weighted_root_frequency_equals_exact_omega():
    g = inputs.from_weighted_edge_list(5, [(0, 1, 0.5), (1, 2, 1.75), (2, 3, 3.0), (3, 0, 0.25),
                                           (0, 2, 2.5), (3, 4, 1.0)])
    alpha = Fraction(3, 4)
    exact = oracle.exact_omega_diag(g, alpha)
    trees = oracle.spanning_trees(g)
    W = sum(alpha ** k * wp for _, k, wp in trees)
    for v in range(g.n):
        frac = sum(alpha ** k * wp for t, k, wp in trees if t[v] == g.n) / W
        assert frac == exact[v]
    n_trees = 200000
    res = oracle.sample(g, float(alpha), 9, 0, n_trees)
    for v in range(g.n):
        p = float(exact[v])
        sd = math.sqrt(p * (1 - p) / n_trees)
        assert abs(res.R[v] / n_trees - p) < 5 * sd


@pytest.mark.parametrize("alpha,w", [(1.0, 0.5), (2.0, 3.0), (0.3, 10.0)])
def test_single_weighted_edge_closed_form(alpha, w):
    g = inputs.from_weighted_edge_list(2, [(0, 1, w)])
    Om = oracle.forest_matrix(g, alpha)
    assert np.allclose(np.diag(Om), (1 + alpha * w) / (1 + 2 * alpha * w), rtol=1e-14, atol=0)
    assert np.allclose(Om.sum(axis=1), 1.0, rtol=0, atol=1e-14)


def test_zero_weight_edges_are_never_taken():
    # vertex 3's edges all weigh 0: always a root with one draw; the zero edge
    # {0, 2} never appears in a tree
    g = inputs.from_weighted_edge_list(5, [(0, 1, 1.0), (1, 2, 2.0), (0, 2, 0.0), (3, 0, 0.0),
                                           (3, 4, 0.0), (1, 4, 0.5)])
    res = oracle.sample(g, 1.3, 5, 0, 3000, per_tree=True)
    assert (res.parents[:, 3] == g.n).all() and (res.tree_visits[:, 3] == 1).all()
    assert not ((res.parents[:, 0] == 2) | (res.parents[:, 2] == 0)).any()
    assert not (res.parents[:, 4] == 3).any()
    assert oracle.root_threshold_w(1.3, 0.0) == 1 << 32


def test_weighted_eps_delta_guarantee():
    """(eps, delta) = (0.1, 0.1), tau = 576 on a weighted ER(1000) against the
    dense weighted forest matrix: no seed of 10 exceeds eps."""
    g = inputs.with_weights(inputs.erdos_renyi(1000, 0.01, 0), 2)
    Om = np.diag(oracle.forest_matrix(g, 1.0))
    assert np.allclose(oracle.forest_matrix(g, 1.0).sum(axis=1), 1.0, atol=1e-12)
    t = oracle.tau(g.m, g.n, 0.1, 0.1)
    assert t == 576
    for seed in range(10):
        res = oracle.sample(g, 1.0, seed, 0, t)
        assert np.abs(res.R / t - Om).max() < 0.1
