"""Pins of the oracle's group forest closeness (Section 5): the group farness
f(S) = tr((L*_{-S})^{-1}) and the greedy of Algorithm 2.

- Lemma "a-vc" on 3-regular graphs: tr((L_{-S} + I)^{-1}) >= (n - k)/4 with
  equality exactly for vertex covers, and the closed form of f(S) it gives
  (block inversion around u*'s row, as in the proof of Theorem
  "GFC-NP-hard") for every vertex cover.
- The Schur-complement form of f(S) on random graphs and sets.
- The greedy: its f(S) trajectory equals direct inversion of every prefix
  (pins the downdate), every choice maximises the marginal gain computed by
  direct inversion (pins the gain formula), the first vertex is the one of
  highest individual forest closeness (the corollary's v_0), and the
  corollary's approximation bound holds against brute force.
- The lemma on f: non-increasing and supermodular.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import inputs


def _three_regular():
    k4 = [(a, b) for a in range(4) for b in range(a + 1, 4)]
    k33 = [(a, 3 + b) for a in range(3) for b in range(3)]
    cube = [(a, a ^ (1 << i)) for a in range(8) for i in range(3) if a < a ^ (1 << i)]
    petersen = ([(i, (i + 1) % 5) for i in range(5)] + [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
                + [(i, 5 + i) for i in range(5)])
    prism = [(i, (i + 1) % 4) for i in range(4)] + [(4 + i, 4 + (i + 1) % 4) for i in range(4)] + \
            [(i, 4 + i) for i in range(4)]
    return [("K4", 4, k4), ("K33", 6, k33), ("cube", 8, cube), ("petersen", 10, petersen),
            ("prism4", 8, prism)]


def _is_cover(S, edges):
    s = set(S)
    return all(a in s or b in s for a, b in edges)


def _t(n, k):
    """f(S) of a vertex cover S, |S| = k, of a 3-regular graph at alpha = 1:
    every vertex outside S has its three neighbours in S, so L_{-S} + I = 4I and
    block inversion around u*'s row (degree n) gives
    (n - k)/4 + (1 + (n - k)/16) / (n - (n - k)/4)."""
    return (n - k) / 4 + (1 + (n - k) / 16) / (n - (n - k) / 4)


@pytest.mark.parametrize("name,n,edges", _three_regular())
def test_lemma_vertex_cover_and_closed_form(name, n, edges):
    g = inputs.from_edge_list(n, edges, name)
    L = oracle.laplacian(g)
    covers = 0
    for k in range(1, n):
        for S in itertools.combinations(range(n), k):
            keep = [v for v in range(n) if v not in S]
            tr = float(np.trace(np.linalg.inv(L[np.ix_(keep, keep)] + np.eye(len(keep)))))
            assert tr >= (n - k) / 4 - 1e-12
            cover = _is_cover(S, edges)
            assert (abs(tr - (n - k) / 4) <= 1e-12) == cover, (S, tr)
            f = oracle.group_farness(g, 1.0, S)
            if cover:
                covers += 1
                assert abs(f - _t(n, k)) <= 1e-12, (S, f, _t(n, k))
            else:
                assert f > _t(n, k) + 1e-9, (S, f)
    assert covers > 0


def test_group_farness_schur_form():
    rng = np.random.default_rng(3)
    for gi, g in enumerate([inputs.barabasi_albert(40, 2, 1), inputs.erdos_renyi(35, 0.15, 2),
                            inputs.with_weights(inputs.erdos_renyi(30, 0.2, 4), 5)]):
        n = g.n
        for alpha in (0.3, 1.0, 4.0):
            for k in (1, 3, 10):
                S = rng.choice(n, k, replace=False)
                keep = np.setdiff1d(np.arange(n), S)
                A = (alpha * oracle.laplacian(g) + np.eye(n))[np.ix_(keep, keep)]
                Ai = np.linalg.inv(A)
                one = np.ones(len(keep))
                schur = n - one @ Ai @ one
                closed = np.trace(Ai) + (1 + one @ Ai @ Ai @ one) / schur
                assert abs(oracle.group_farness(g, alpha, S) - closed) <= 1e-10 * closed


@pytest.mark.parametrize("seed,alpha", [(1, 1.0), (2, 0.5), (3, 3.0)])
def test_greedy_trajectory_gains_and_first_vertex(seed, alpha):
    g = inputs.barabasi_albert(45, 2, seed)
    k = 6
    S, f = oracle.greedy_group(g, alpha, k)
    assert len(S) == k == len(set(S)) and all(0 <= v < g.n for v in S)
    # the downdate keeps M = (L*_{-S})^{-1}: f after each step by direct inversion
    for i in range(k):
        direct = oracle.group_farness(g, alpha, S[:i + 1])
        assert abs(f[i] - direct) <= 1e-10 * direct
    # every choice maximises the marginal gain f(S) - f(S + v), by direct inversion
    for i in range(1, k):
        base = oracle.group_farness(g, alpha, S[:i])
        gains = {v: base - oracle.group_farness(g, alpha, S[:i] + [v])
                 for v in range(g.n) if v not in S[:i]}
        best = max(gains.values())
        assert gains[S[i]] >= best - 1e-9 * abs(best)
    # the first vertex has the highest individual forest closeness (lowest Omega_vv)
    d = np.diag(oracle.forest_matrix(g, alpha))
    assert S[0] == int(np.argmin(d))


def test_greedy_bound_against_brute_force():
    for seed in (1, 2, 3):
        g = inputs.erdos_renyi(11, 0.35, seed)
        for k in (2, 3):
            S, f = oracle.greedy_group(g, 1.0, k)
            opt = min(oracle.group_farness(g, 1.0, T) for T in itertools.combinations(range(g.n), k))
            f0 = f[0]
            bound = 1 - k / (math.e * (k - 1))
            assert f0 - f[-1] >= bound * (f0 - opt) - 1e-12
            assert f[-1] >= opt - 1e-12


def test_group_farness_non_increasing_and_supermodular():
    g = inputs.erdos_renyi(14, 0.3, 6)
    rng = np.random.default_rng(8)
    for _ in range(60):
        T = list(rng.choice(g.n, rng.integers(2, 7), replace=False))
        S = T[:rng.integers(1, len(T))]
        v = int(rng.choice([x for x in range(g.n) if x not in T]))
        fS, fT = oracle.group_farness(g, 1.0, S), oracle.group_farness(g, 1.0, T)
        fSv, fTv = oracle.group_farness(g, 1.0, S + [v]), oracle.group_farness(g, 1.0, T + [v])
        assert fS >= fT - 1e-12 and fS >= fSv - 1e-12
        assert fS - fSv >= fT - fTv - 1e-12
