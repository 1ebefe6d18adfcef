"""Pins for the oracle's binary64 definitions: the forest matrix, forest
distance / farness, the augmented graph and the CG ground truth.

Checked against closed forms, a second factorisation, invariants that follow
from (alpha L + I) Omega = I, exact rational arithmetic and the Moore-Penrose
pseudoinverse (the paper's own cross-check tool in its experiments).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import inputs


def test_closed_form_empty_graph():
    g = inputs.from_edge_list(6, [])
    assert np.allclose(oracle.forest_matrix(g, 3.0), np.eye(6), atol=0, rtol=0)


@pytest.mark.parametrize("alpha", [0.1, 1.0, 2.5])
def test_closed_form_single_edge(alpha):
    g = inputs.from_edge_list(2, [(0, 1)])
    Om = oracle.forest_matrix(g, alpha)
    assert np.allclose(np.diag(Om), (1 + alpha) / (1 + 2 * alpha), rtol=1e-14)
    assert math.isclose(Om[0, 1], alpha / (1 + 2 * alpha), rel_tol=1e-14)


@pytest.mark.parametrize("n,alpha", [(5, 1.0), (12, 0.3), (30, 4.0)])
def test_closed_form_complete_graph(n, alpha):
    g = inputs.from_edge_list(n, [(a, b) for a in range(n) for b in range(a + 1, n)])
    Om = oracle.forest_matrix(g, alpha)
    want = 1.0 / n + (1.0 - 1.0 / n) / (alpha * n + 1.0)
    assert np.allclose(np.diag(Om), want, rtol=1e-13)


@pytest.mark.parametrize("n,alpha", [(3, 1.0), (10, 0.5), (25, 2.0)])
def test_closed_form_cycle(n, alpha):
    g = inputs.from_edge_list(n, [(i, (i + 1) % n) for i in range(n)])
    Om = oracle.forest_matrix(g, alpha)
    lam = 2.0 - 2.0 * np.cos(2.0 * np.pi * np.arange(n) / n)
    want = np.mean(1.0 / (1.0 + alpha * lam))
    assert np.allclose(np.diag(Om), want, rtol=1e-13)


def test_two_factorisations_agree_and_invariants():
    g = inputs.erdos_renyi(300, 0.02, 3)
    alpha = 1.0
    A = oracle.forest_matrix(g, alpha)
    B = oracle.forest_matrix_cholesky(g, alpha)
    assert np.abs(A - B).max() < 1e-12
    n = g.n
    deg = g.degrees
    assert np.abs(A @ np.ones(n) - 1.0).max() < 1e-12          # doubly stochastic
    assert np.abs(A - A.T).max() < 1e-13
    assert A.min() > -1e-15                                        # non-negative
    d = np.diag(A)
    assert (d >= 1.0 / (1.0 + alpha * deg) - 1e-14).all()
    assert (d <= 1.0 + 1e-14).all()
    iso = deg == 0
    assert np.allclose(d[iso], 1.0, rtol=0, atol=1e-14)
    assert (d[~iso] < 1.0).all()


def test_exact_rationals_match_dense():
    g = inputs.from_edge_list(6, [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (4, 5), (5, 3)])
    for alpha in (Fraction(1), Fraction(3, 4)):
        ex = oracle.exact_omega_diag(g, alpha)
        Om = oracle.forest_matrix(g, float(alpha))
        for v in range(g.n):
            assert abs(float(ex[v]) - Om[v, v]) < 1e-15


def test_farness_identity_vs_definition():
    g = inputs.erdos_renyi(200, 0.03, 8)
    for alpha in (0.2, 1.0, 5.0):
        Om = oracle.forest_matrix(g, alpha)
        f1 = oracle.farness_by_definition(Om)
        f2 = oracle.farness_by_identity(Om)
        assert np.abs(f1 - f2).max() < 1e-10 * np.abs(f1).max()


def test_augmented_graph_pseudoinverse_relations():
    """Prop. forest-resistance and the derived facts about the pivot u*."""
    g = inputs.erdos_renyi(40, 0.08, 5)
    n = g.n
    alpha = 0.8
    Om = oracle.forest_matrix(g, alpha)
    Ls = oracle.augmented_laplacian(g, alpha)
    # removing u*'s row and column of L* leaves exactly alpha L + I
    assert np.array_equal(Ls[:n, :n], alpha * oracle.laplacian(g) + np.eye(n))
    P = np.linalg.pinv(Ls)
    rho = oracle.forest_distance(Om)
    for u in range(0, n, 7):
        for v in range(1, n, 5):
            assert abs(oracle.effective_resistance(P, u, v) - rho[u, v]) < 1e-10
    # r_{G*}(u*, v) = Omega_vv: the edge-{u*, v} frequency targets Omega_vv
    for v in range(n):
        assert abs(oracle.effective_resistance(P, n, v) - Om[v, v]) < 1e-10
    # pivot column of L*^+ (mean-zero solution of L* x = e_u* - 1/(n+1) 1)
    assert abs(P[n, n] - n / (n + 1) ** 2) < 1e-12
    assert np.abs(P[:n, n] + 1.0 / (n + 1) ** 2).max() < 1e-12
    # the V-block of L*^+ is Omega shifted by a constant, not Omega itself
    shift = (n + 2) / (n + 1) ** 2
    assert np.abs(P[:n, :n] - (Om - shift)).max() < 1e-12


def test_cg_matches_dense():
    g = inputs.barabasi_albert(300, 3, 2)
    alpha = 1.0
    Om = oracle.forest_matrix(g, alpha)
    vs = [0, 17, 299, 150]
    d = oracle.omega_diag_cg(g, alpha, vs, rtol=1e-12)
    assert np.abs(d - Om[vs, vs]).max() < 1e-10
    B = inputs.gaussian(300 * 3, 1).reshape(300, 3)
    X, it = oracle.cg_solve(g, alpha, B, rtol=1e-10)
    Xd = np.linalg.solve(alpha * oracle.laplacian(g) + np.eye(300), B)
    assert np.abs(X - Xd).max() < 1e-8
    assert it > 1
