"""Pins for the estimator side of the oracle: tau, the (eps, delta) guarantee,
unbiasedness, expected work, and the output formulas.

Ground truth is the dense binary64 forest matrix on the 1000-vertex
Erdos-Renyi workload (G(1000, 0.01), alpha = 1).
"""
import math

import numpy as np
import pytest

import oracle
import inputs


@pytest.fixture(scope="module")
def er():
    g = inputs.erdos_renyi(1000, 0.01, 0)
    Om = oracle.forest_matrix(g, 1.0)
    return g, Om


@pytest.mark.parametrize("m,n,eps,delta,kappa", [
    (5012, 1000, 0.1, 0.1, 0.0), (999985, 200000, 0.1, 0.1, 0.0),
    (999985, 200000, 0.1, 0.1, 0.5), (1758240, 1000000, 0.05, 0.01, 0.0),
    (10, 1000, 0.3, 0.2, 0.1), (0, 1, 0.5, 0.5, 0.0)])
def test_tau_is_minimal_hoeffding_sample(m, n, eps, delta, kappa):
    """tau is the least integer with 2 max(m,n) exp(-2 tau ((1-kappa) eps)^2) <= delta
    (Hoeffding plus a union bound, proof of Theorem time-approx)."""
    t = oracle.tau(m, n, eps, delta, kappa)
    e1 = (1 - kappa) * eps
    bound = lambda tt: 2 * max(m, n) * math.exp(-2 * tt * e1 * e1)
    assert bound(t) <= delta * (1 + 1e-12)
    assert bound(t - 1) > delta * (1 - 1e-12)


def test_tau_rejects_bad_arguments():
    assert oracle.tau(10, 10, 0.0, 0.1) == 0
    assert oracle.tau(10, 10, 1.0, 0.1) == 0
    assert oracle.tau(10, 10, 0.1, 0.0) == 0
    assert oracle.tau(10, 10, 0.1, 1.0) == 0
    assert oracle.tau(10, 10, 0.1, 0.1, 1.0) == 0
    assert oracle.tau(10, 0, 0.1, 0.1) == 0


def test_tau_er1000():
    g = inputs.erdos_renyi(1000, 0.01, 0)
    assert oracle.tau(g.m, g.n, 0.1, 0.1) == 576


def test_eps_delta_guarantee(er):
    """Theorem time-approx: with tau(eps=0.1, delta=0.1), max_v |R/tau - Omega_vv|
    <= eps fails in at most a delta fraction of runs (expected: never)."""
    g, Om = er
    t = oracle.tau(g.m, g.n, 0.1, 0.1)
    d = np.diag(Om)
    fails = 0
    worst = 0.0
    for seed in range(40):
        r = oracle.sample(g, 1.0, seed, 0, t)
        err = np.abs(r.R / t - d).max()
        worst = max(worst, err)
        fails += err > 0.1
    assert fails <= 4
    assert worst < 0.1


def test_unbiased_and_clt(er):
    """Prop. unbiased: E[R/tau] = Omega_vv; per-vertex z-scores are N(0,1)."""
    g, Om = er
    d = np.diag(Om)
    t = 4000
    r = oracle.sample(g, 1.0, 1, 0, t)
    z = (r.R - t * d) / np.sqrt(t * d * (1 - d))
    assert abs(z.mean()) < 0.25
    assert 0.75 < z.var() < 1.3
    assert np.abs(z).max() < 5.0


def test_expected_work_identities(er):
    """Wilson's running-time identity on G* rooted at u*: E[k_v] =
    Omega_vv (1 + alpha d_v) (Green's function of the walk killed at u*), so
    E[steps per tree] = sum_v Omega_vv (1 + alpha d_v), between n and
    n + 2 alpha m (Prop. ust-wilson-time); E[roots per tree] = tr(Omega)."""
    g, Om = er
    d = np.diag(Om)
    deg = g.degrees
    t = 2000
    r = oracle.sample(g, 1.0, 2, 0, t, per_tree=True)
    ek = d * (1 + deg)
    assert g.n <= ek.sum() <= g.n + 2 * g.m
    steps = r.steps.astype(np.float64)
    assert abs(steps.mean() - ek.sum()) < 5 * steps.std() / math.sqrt(t)
    roots = r.roots.astype(np.float64)
    assert abs(roots.mean() - d.sum()) < 5 * roots.std() / math.sqrt(t)
    kv = r.tree_visits.astype(np.float64)
    zk = (kv.mean(axis=0) - ek) / (kv.std(axis=0) / math.sqrt(t) + 1e-12)
    assert np.abs(zk).max() < 5.5


def test_estimator_outputs(er):
    g, Om = er
    t = 300
    r = oracle.sample(g, 1.0, 4, 0, t)
    diag, far, clo = oracle.estimate(r.R, t)
    n = g.n
    # diag is R/tau; farness uses the doubly-stochastic identity with tr = S/tau
    assert np.array_equal(diag, r.R.astype(np.float64) / t)
    want = n * diag + diag.sum() - 2.0
    assert np.abs(far - want).max() < 1e-9
    assert np.allclose(clo, n / far, rtol=1e-15)
    # ranking: ascending diag <-> descending closeness
    assert (np.argsort(-clo, kind="stable") == np.argsort(diag, kind="stable")).all()
    # literal reading of Algorithm 1's last loop (minimum-norm solution x):
    # shifts every entry by the constant that separates L*^+ from Omega
    dl, _, _ = oracle.estimate(r.R, t, literal=True)
    Ls = oracle.augmented_laplacian(g, 1.0)
    P = np.linalg.pinv(Ls)
    shift_pinv = np.mean(np.diag(Om) - np.diag(P)[:n])
    assert np.abs((diag - dl) - shift_pinv).max() < 1e-12


def test_farness_estimate_tracks_definition(er):
    """The sampled farness approaches the definition-sum farness of the dense
    Omega at the rate of the diagonal error (n * eps)."""
    g, Om = er
    t = 2000
    r = oracle.sample(g, 1.0, 5, 0, t)
    _, far, _ = oracle.estimate(r.R, t)
    f_def = oracle.farness_by_definition(Om)
    diag_err = np.abs(r.R / t - np.diag(Om)).max()
    tr_err = abs(r.R.sum() / t - np.trace(Om))
    assert np.abs(far - f_def).max() <= g.n * diag_err + tr_err + 1e-6
