"""Pins for the oracle's UST sampler (Algorithm 3 of the paper).

What fixes the sampler, independently of its own code:
  * Cayley: K4 plus the universal vertex is K5, whose 5^3 = 125 spanning
    trees must come out equiprobable.
  * Weighted G*: edges of G weigh alpha and edges to u* weigh 1, so a uniform
    spanning tree of the weighted G* has P(T) proportional to
    alpha^(number of G-edges in T) (Section 4.1); checked against brute-force
    enumeration of all spanning trees.
  * Wilson's cycle-popping theorem: parents, visit counts and root counts do
    not depend on the order in which walks are started.
  * Structural validity of every sampled parent array.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import inputs


def _is_spanning_tree(g, parent):
    n = g.n
    adj = [set(g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]].tolist()) for v in range(n)]
    for v in range(n):
        p = int(parent[v])
        if p == n:
            continue
        if p < 0 or p > n or p not in adj[v]:
            return False
    # every vertex reaches u* by following parents (no cycles)
    state = np.zeros(n, np.int8)  # 0 new, 1 on stack, 2 done
    for v in range(n):
        path = []
        u = v
        while u != n and state[u] == 0:
            state[u] = 1
            path.append(u)
            u = int(parent[u])
        if u != n and state[u] == 1:
            return False
        for x in path:
            state[x] = 2
    return True


def _chi2_tree_test(g, alpha, n_trees, seed):
    trees = oracle.spanning_trees(g)
    weights = np.array([alpha ** k for _, k, _ in trees], np.float64)
    probs = weights / weights.sum()
    index = {t: i for i, (t, _, _) in enumerate(trees)}
    res = oracle.sample(g, alpha, seed, 0, n_trees, per_tree=True)
    counts = np.zeros(len(trees), np.int64)
    for row in res.parents:
        counts[index[tuple(int(x) for x in row)]] += 1
    chi2, p = stats.chisquare(counts, n_trees * probs)
    return len(trees), counts, p


def test_k5_cayley_uniform():
    g = inputs.from_edge_list(4, [(a, b) for a in range(4) for b in range(a + 1, 4)])
    ntrees, counts, p = _chi2_tree_test(g, 1.0, 125 * 400, seed=7)
    assert ntrees == 125  # Cayley: (n+1)^(n-1) with n+1 = 5
    assert p > 1e-3


@pytest.mark.parametrize("name,n,edges,alpha", [
    ("cycle4", 4, [(0, 1), (1, 2), (2, 3), (3, 0)], 2.0),
    ("path3", 3, [(0, 1), (1, 2)], 3.0),
    ("star", 4, [(0, 1), (0, 2), (0, 3)], 0.5),
    ("triangle_plus_isolated", 4, [(0, 1), (1, 2), (0, 2)], 1.5),
])
def test_weighted_tree_distribution(name, n, edges, alpha):
    g = inputs.from_edge_list(n, edges)
    ntrees, counts, p = _chi2_tree_test(g, alpha, 60000, seed=11)
    assert ntrees >= 3
    assert p > 1e-3, (name, counts)


def test_root_frequency_equals_exact_omega():
    """Kirchhoff (proof of Prop. unbiased): P[{u*, v} in T] = r(u*, v) in G* =
    Omega_vv; exact rationals vs the brute-force tree fraction vs sampling."""
    from fractions import Fraction
    g = inputs.from_edge_list(5, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2), (3, 4)])
    alpha = Fraction(1, 2)
    exact = oracle.exact_omega_diag(g, alpha)
    trees = oracle.spanning_trees(g)
    W = sum(alpha ** k for _, k, _ in trees)
    for v in range(g.n):
        frac = sum(alpha ** k for t, k, _ in trees if t[v] == g.n) / W
        assert frac == exact[v]
    n_trees = 200000
    res = oracle.sample(g, float(alpha), 3, 0, n_trees)
    for v in range(g.n):
        p = float(exact[v])
        sd = math.sqrt(p * (1 - p) / n_trees)
        assert abs(res.R[v] / n_trees - p) < 5 * sd


def test_sampled_parents_are_spanning_trees():
    g = inputs.erdos_renyi(60, 0.05, 1)
    res = oracle.sample(g, 1.0, 5, 0, 200, per_tree=True)
    for i in range(200):
        assert _is_spanning_tree(g, res.parents[i])
        # every vertex draws at least once, so steps >= n
        assert res.steps[i] == res.tree_visits[i].sum() >= g.n
        assert res.roots[i] == (res.parents[i] == g.n).sum()
        # isolated vertices are roots with exactly one draw
        iso = np.diff(g.row_ptr) == 0
        assert (res.parents[i][iso] == g.n).all()
        assert (res.tree_visits[i][iso] == 1).all()
    assert (res.R == (res.parents == g.n).sum(axis=0)).all()
    assert (res.visits == res.tree_visits.astype(np.uint64).sum(axis=0)).all()


def _digest(parents, n):
    tot = 0
    for v in range(n):
        tot = (tot + oracle.mix64((v << 32) | int(parents[v]))) & 0xFFFFFFFFFFFFFFFF
    return tot


def test_digest_definition():
    g = inputs.erdos_renyi(40, 0.1, 2)
    res = oracle.sample(g, 1.0, 9, 3, 5, per_tree=True)
    for i in range(5):
        assert int(res.digests[i]) == _digest(res.parents[i], g.n)


@pytest.mark.parametrize("gname", ["er", "ba", "grid"])
def test_order_independence(gname):
    """Cycle popping: same parents and visit counts for any start order."""
    if gname == "er":
        g = inputs.erdos_renyi(300, 0.02, 4)
    elif gname == "ba":
        g = inputs.barabasi_albert(400, 3, 4)
    else:
        g = inputs.grid_removed(20, 20, 0.12, 4)
    n = g.n
    orders = [None, np.arange(n), np.arange(n)[::-1].copy(), inputs.permutation(n, 99)]
    outs = [oracle.sample(g, 0.7, 21, 5, 12, order=o, per_tree=True) for o in orders]
    for o in outs[1:]:
        assert (o.parents == outs[0].parents).all()
        assert (o.tree_visits == outs[0].tree_visits).all()
        assert (o.R == outs[0].R).all()
        assert (o.digests == outs[0].digests).all()


def test_tree_ranges_sum():
    """Trees are pure functions of their index: split ranges sum exactly."""
    g = inputs.erdos_renyi(200, 0.03, 6)
    a = oracle.sample(g, 1.0, 1, 0, 30)
    b = oracle.sample(g, 1.0, 1, 30, 20)
    c = oracle.sample(g, 1.0, 1, 0, 50)
    assert (a.R + b.R == c.R).all()
    assert (a.visits + b.visits == c.visits).all()
    assert (np.concatenate([a.digests, b.digests]) == c.digests).all()


def test_streams_and_seeds_differ():
    g = inputs.erdos_renyi(200, 0.03, 6)
    a = oracle.sample(g, 1.0, 1, 0, 10)
    b = oracle.sample(g, 1.0, 1, 0, 10, stream=1)
    c = oracle.sample(g, 1.0, 2, 0, 10)
    assert (a.digests != b.digests).all()
    assert (a.digests != c.digests).all()


def test_degenerate_graphs():
    # no edges: every vertex is a root in every tree, Omega = I
    g = inputs.from_edge_list(7, [])
    r = oracle.sample(g, 1.0, 0, 0, 10, per_tree=True)
    assert (r.parents == 7).all() and (r.R == 10).all() and (r.steps == 7).all()
    # single vertex
    g1 = inputs.from_edge_list(1, [])
    r1 = oracle.sample(g1, 2.0, 0, 0, 3)
    assert (r1.R == 3).all()
    # empty graph (n = 0)
    g0 = inputs.from_edge_list(0, [])
    r0 = oracle.sample(g0, 1.0, 0, 0, 3)
    assert r0.R.shape == (0,)


# --------------------------------------------------------------------------
# Contract pins that no statistic can see.
# --------------------------------------------------------------------------
def _arrow(g, alpha, seed, stream, t, v, j):
    """The j-th arrow of v in tree t as the randomness contract defines it,
    built on the Philox block function pinned above (known-answer vectors and
    rocRAND): x0 < thr(d) -> u*, else neighbour floor(x1 d / 2^32)."""
    x = oracle.philox4x32_10([v, j, t, stream], [seed & 0xFFFFFFFF, seed >> 32])
    d = int(g.row_ptr[v + 1] - g.row_ptr[v])
    if int(x[0]) < oracle.root_threshold(alpha, d):
        return g.n
    return int(g.col_idx[g.row_ptr[v] + ((int(x[1]) * d) >> 32)])


def _cycle_popping(g, alpha, seed, stream, t):
    """Wilson's cycle popping (Wilson 1996, Theorem on stacks of arrows): pop
    any cycle of the top arrows until none is left; the top arrows then form
    the tree and top index + 1 is the number of arrows drawn at each vertex.
    A different algorithm from the walk-and-erase sampler."""
    n = g.n
    top = [0] * n
    arrow = [_arrow(g, alpha, seed, stream, t, v, 0) for v in range(n)]
    while True:
        cycle = None
        for s in range(n):
            seen = {}
            u = s
            while u != n and u not in seen:
                seen[u] = len(seen)
                u = arrow[u]
            if u != n:
                cycle = [u]
                w = arrow[u]
                while w != u:
                    cycle.append(w)
                    w = arrow[w]
                break
        if cycle is None:
            return arrow, [x + 1 for x in top]
        for v in cycle:
            top[v] += 1
            arrow[v] = _arrow(g, alpha, seed, stream, t, v, top[v])


@pytest.mark.parametrize("seed,alpha", [(0, 1.0), (5, 0.4), (77, 3.0)])
def test_matches_cycle_popping(seed, alpha):
    g = inputs.erdos_renyi(14, 0.3, seed + 1)
    res = oracle.sample(g, alpha, seed, 2, 25, stream=3, per_tree=True)
    for i in range(25):
        par, k = _cycle_popping(g, alpha, seed, 3, 2 + i)
        assert list(res.parents[i]) == par
        assert list(res.tree_visits[i]) == k


def test_root_test_is_strict_at_the_threshold():
    """Construct alpha so that thr(1) equals x0 of vertex 0's first arrow in
    tree 0 exactly: the contract's strict comparison sends that walk to the
    neighbour, not to u*."""
    x = oracle.philox4x32_10([0, 0, 0, 0], [0, 0])   # known-answer vector 1
    x0 = int(x[0])
    assert x0 == 0x6627E8D5
    alpha = 2.0**32 / (x0 + 0.5) - 1.0
    assert oracle.root_threshold(alpha, 1) == x0
    g = inputs.from_edge_list(2, [(0, 1)])
    res = oracle.sample(g, alpha, 0, 0, 1, order=np.array([0, 1]), per_tree=True)
    # vertex 0's first arrow goes to vertex 1 (x0 is not below thr)
    par, k = _cycle_popping(g, alpha, 0, 0, 0)
    assert _arrow(g, alpha, 0, 0, 0, 0, 0) == 1
    assert list(res.parents[0]) == par
    assert list(res.tree_visits[0]) == k
