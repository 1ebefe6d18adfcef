"""Generators: determinism, simplicity, symmetry and exact edge counts.
Parity unpinned beyond self-consistency: the graphs are synthetic stand-ins
for the paper's datasets and have no external reference values."""
import numpy as np
import pytest

import inputs


def _check_simple_symmetric(g):
    n = g.n
    rp, ci = g.row_ptr, g.col_idx
    assert rp[0] == 0 and rp[-1] == ci.size and (np.diff(rp) >= 0).all()
    assert ci.min(initial=0) >= 0 and (ci.size == 0 or ci.max() < n)
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert (rows != ci).all()                                   # no self-loops
    for v in range(0, n, max(1, n // 500)):                     # sorted, no duplicates
        r = ci[rp[v]:rp[v + 1]]
        assert (np.diff(r) > 0).all()
    fwd = set(zip(rows.tolist(), ci.tolist())) if n < 5000 else None
    if fwd is not None:
        assert all((b, a) in fwd for a, b in fwd)
    else:
        key_f = np.sort(rows.astype(np.int64) * n + ci)
        key_b = np.sort(ci.astype(np.int64) * n + rows)
        assert np.array_equal(key_f, key_b)


def test_er_deterministic_and_simple():
    a = inputs.erdos_renyi(1000, 0.01, 0)
    b = inputs.erdos_renyi(1000, 0.01, 0)
    c = inputs.erdos_renyi(1000, 0.01, 1)
    assert np.array_equal(a.col_idx, b.col_idx) and np.array_equal(a.row_ptr, b.row_ptr)
    assert not np.array_equal(a.row_ptr, c.row_ptr)
    _check_simple_symmetric(a)
    assert abs(a.m - 4995) < 5 * 70


def test_ba_edge_count_and_shape():
    g = inputs.barabasi_albert(20000, 5, 0)
    assert g.m == 15 + 5 * (20000 - 6)
    _check_simple_symmetric(g)
    assert g.degrees.min() >= 5
    assert g.degrees.max() > 100                                  # heavy tail


def test_grid_exact_edge_count():
    g = inputs.grid_removed(1000, 1000, 0.12, 0)
    assert g.n == 10**6
    assert g.m == 1998000 - 239760 == 1758240
    _check_simple_symmetric(g)
    assert g.degrees.max() <= 4
    assert (g.degrees == 0).sum() > 0                             # disconnected


def test_rmat_simple():
    g = inputs.rmat(5000, 8, 3)
    _check_simple_symmetric(g)
    assert g.m <= 8 * 5000
    sizes = inputs.rmat_batch_sizes(256, 0)
    assert min(sizes) >= 2**10 and max(sizes) <= 2**17


def test_gaussian_moments():
    x = inputs.gaussian(200000, 5)
    assert abs(x.mean()) < 0.01 and abs(x.std() - 1) < 0.01
    assert np.array_equal(x, inputs.gaussian(200000, 5))


def test_csr_builder_matches_numpy():
    """The C CSR builder (count, scatter, per-row sort and dedupe) gives the same
    graph as a numpy unique over symmetrised keys, with self-loops, repeated
    edges, both orientations and isolated vertices in the list."""
    rng = np.random.default_rng(3)
    for n, m in ((1, 0), (5, 12), (200, 3000), (5000, 20000)):
        us = rng.integers(0, n, m, dtype=np.int32)
        vs = rng.integers(0, n, m, dtype=np.int32)
        a = inputs.csr_from_edges(n, us, vs)
        b = inputs.csr_from_edges_numpy(n, us, vs)
        assert np.array_equal(a.row_ptr, b.row_ptr)
        assert np.array_equal(a.col_idx, b.col_idx)
        _check_simple_symmetric(a)
    with pytest.raises(ValueError):
        inputs.csr_from_edges(4, np.array([0, 4], np.int32), np.array([1, 2], np.int32))
