"""GPU parity on weighted graphs (Section 2 allows non-negative edge weights):
the HIP path against the CPU oracle, through the C-ABI.

The weighted step is integer work decided by binary64 arithmetic that both
sides carry out in the same order (running row sums in CSR order, the root
threshold of the weighted degree, u = (x1 * W) * 2^-32), so the bar is
bit-exactness, as for unit weights.
"""
import sys

import numpy as np
import pytest

import oracle
import inputs

pytestmark = pytest.mark.gpu

SAMPLERS = ["lane", "coop", "lds", "hyb", "tile"]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _compare(fc, g, alpha, seed, t0, count, stream=0, per_tree=True, sampler=None):
    _say(f"weighted parity {sampler} {g.name or g.n} alpha={alpha} seed={seed} "
         f"trees=[{t0},{t0 + count}) stream={stream}")
    got = fc.sample(g, alpha=alpha, seed=seed, tree_begin=t0, tree_count=count, stream_id=stream,
                    want_visits=True, want_digests=True, want_steps=True,
                    want_parents=per_tree, want_tree_visits=per_tree, sampler=sampler)
    if sampler:
        assert got["stats"]["sampler"] == ("wilson_" + sampler if g.n and count else "")
    ref = oracle.sample(g, alpha, seed, t0, count, stream=stream, per_tree=per_tree)
    if per_tree:
        for i in range(count):
            assert np.array_equal(got["parents"][i], ref.parents[i]), f"parents differ in tree {t0 + i}"
            assert np.array_equal(got["tree_visits"][i], ref.tree_visits[i]), f"visits differ in tree {t0 + i}"
    assert np.array_equal(got["tree_digests"], ref.digests)
    assert np.array_equal(got["tree_steps"], ref.steps)
    assert np.array_equal(got["root_counts"], ref.R)
    assert np.array_equal(got["visit_counts"], ref.visits)
    st = got["stats"]
    assert st["walk_steps"] == int(ref.steps.sum())
    assert st["roots"] == int(ref.roots.sum())
    return got, ref


def _small(case):
    W = inputs.from_weighted_edge_list
    if case == "edge":
        return W(2, [(0, 1, 2.5)], "w_edge")
    if case == "triangle":
        return W(3, [(0, 1, 0.25), (1, 2, 4.0), (0, 2, 1.0)], "w_triangle")
    if case == "star_extreme":  # weights across the whole accepted range in one row
        return W(6, [(0, 1, 2.0**-64), (0, 2, 1.0), (0, 3, 2.0**64), (0, 4, 0.0), (0, 5, 3.5)],
                 "w_star_extreme")
    if case == "star_extreme_dense":  # the same extremes among many ordinary weights
        edges = [(0, v, 1.0 + (v % 5)) for v in range(1, 40)]
        edges[6] = (0, 7, 2.0**-64)
        edges[20] = (0, 21, 2.0**64)
        edges[29] = (0, 30, 0.0)
        return W(40, edges + [(7, 8, 2.0), (21, 22, 2.0**63)], "w_star_extreme_dense")
    if case == "zero_component":  # vertex 3 only has zero-weight edges: always a root
        return W(5, [(0, 1, 1.5), (1, 2, 0.5), (2, 3, 0.0), (3, 4, 0.0), (0, 2, 2.0)],
                 "w_zero_component")
    if case == "all_zero":
        return W(4, [(0, 1, 0.0), (1, 2, 0.0), (2, 3, 0.0)], "w_all_zero")
    if case == "k6":
        edges = [(a, b, 0.5 + ((3 * a + 5 * b) % 7)) for a in range(6) for b in range(a + 1, 6)]
        return W(6, edges, "w_k6")
    if case == "path_isolated":
        return W(5, [(0, 1, 3.0), (1, 2, 0.125), (2, 3, 7.0)], "w_path_isolated")
    raise ValueError(case)


# Expected walk steps per tree are at most n + alpha * (sum of weighted
# degrees): with weights near 2^64 alpha must be tiny for trees to finish.
_ALPHAS = {"star_extreme": (2.0**-70, 2.0**-66), "star_extreme_dense": (2.0**-72, 2.0**-67)}


@pytest.mark.parametrize("sampler", SAMPLERS)
@pytest.mark.parametrize("case", ["edge", "triangle", "star_extreme", "star_extreme_dense",
                                  "zero_component", "all_zero", "k6", "path_isolated"])
def test_small_weighted_graphs(gpu_lib, case, sampler):
    g = _small(case)
    for alpha in _ALPHAS.get(case, (0.3, 1.0, 7.0)):
        _compare(gpu_lib, g, alpha, 11, 0, 64, sampler=sampler)


@pytest.mark.parametrize("sampler", SAMPLERS)
def test_weighted_er1000_bit_exact(gpu_lib, sampler):
    """ER(1000, 0.01) with log-uniform weights in [0.1, 10), alpha = 1: 600 trees."""
    g = inputs.with_weights(inputs.erdos_renyi(1000, 0.01, 0), 3)
    _compare(gpu_lib, g, 1.0, 5, 0, 600, sampler=sampler)


@pytest.mark.parametrize("sampler", SAMPLERS)
def test_unit_weights_equal_unweighted(gpu_lib, sampler):
    """Weights all 1: the same trees as the unweighted graph (degrees < 2^21)."""
    fc = gpu_lib
    g = inputs.barabasi_albert(20_000, 4, 1)
    gw = inputs.CSRGraph(g.n, g.row_ptr, g.col_idx, "ba20k_unit", np.ones(len(g.col_idx)))
    a = fc.sample(g, alpha=0.7, seed=3, tree_count=40, want_digests=True, want_visits=True,
                  sampler=sampler)
    b = fc.sample(gw, alpha=0.7, seed=3, tree_count=40, want_digests=True, want_visits=True,
                  sampler=sampler)
    assert np.array_equal(a["tree_digests"], b["tree_digests"])
    assert np.array_equal(a["root_counts"], b["root_counts"])
    assert np.array_equal(a["visit_counts"], b["visit_counts"])


@pytest.mark.parametrize("sampler", SAMPLERS)
def test_weighted_ba200k_subset_bit_exact(gpu_lib, sampler):
    """BA(200000, 5) with log-uniform weights, alpha = 1: 32 trees and a later
    range (the LDS sampler draws first arrows ahead at this size)."""
    g = inputs.with_weights(inputs.barabasi_albert(200_000, 5, 0), 0)
    got, _ = _compare(gpu_lib, g, 1.0, 0, 0, 32, per_tree=True, sampler=sampler)
    if sampler == "lds":
        assert got["stats"]["ms_predraw"] > 0.0
    _compare(gpu_lib, g, 1.0, 0, 4000, 16, per_tree=False, sampler=sampler)


@pytest.mark.parametrize("sampler", SAMPLERS)
def test_weighted_rmat_heavy_tail_bit_exact(gpu_lib, sampler):
    """R-MAT 2^14 (rows up to thousands of entries: deep weighted searches),
    weights spanning four decades."""
    g = inputs.with_weights(inputs.rmat(1 << 14, 8, 3), 9, lo=1e-2, hi=1e2)
    _compare(gpu_lib, g, 1.0, 1, 0, 32, per_tree=False, sampler=sampler)


def test_weighted_grid_device_graph(gpu_lib):
    """Weights travel with a device graph; the automatic sampler choice."""
    fc = gpu_lib
    g = inputs.with_weights(inputs.grid_removed(60, 70, 0.12, 1), 2)
    dg = fc.to_device(g)
    got = fc.sample(dg, alpha=0.5, seed=9, tree_count=100, want_digests=True, want_visits=True)
    ref = oracle.sample(g, 0.5, 9, 0, 100)
    assert np.array_equal(got["tree_digests"], ref.digests)
    assert np.array_equal(got["root_counts"], ref.R)
    assert np.array_equal(got["visit_counts"], ref.visits)


def test_weighted_estimators_bit_exact(gpu_lib):
    fc = gpu_lib
    g = inputs.with_weights(inputs.erdos_renyi(1000, 0.01, 0), 1)
    out = fc.farness(g, alpha=1.0, seed=0, tau=800)
    ref = oracle.sample(g, 1.0, 0, 0, 800)
    d, f, c = oracle.estimate(ref.R, 800)
    assert np.array_equal(out["root_counts"], ref.R)
    assert np.array_equal(out["diag"], d)
    assert np.array_equal(out["farness"], f)
    assert np.array_equal(out["closeness"], c)
    # the (eps, delta) guarantee against the dense weighted forest matrix
    Om = oracle.forest_matrix(g, 1.0)
    est = fc.diag_estimate(g, alpha=1.0, eps=0.1, delta=0.1, seed=2)
    assert np.abs(est["diag"] - np.diag(Om)).max() < 0.1


@pytest.fixture(params=[1, 0], ids=["lds_counters", "global_counters"])
def counters(request, gpu_lib):
    gpu_lib.set_option("coop_lds_counts", request.param)
    yield request.param
    gpu_lib.set_option("coop_lds_counts", 1)


def test_weighted_batch(gpu_lib, counters):
    """Weighted and unweighted jobs on the same CSR arrays in one batch: each
    job equals the oracle on its own graph."""
    fc = gpu_lib
    base = [inputs.rmat(1 << 10, 8, 21), inputs.barabasi_albert(3000, 3, 5)]
    gs, dgs = [], []
    for i, g in enumerate(base):
        dg = fc.to_device(g)
        for wseed in (None, 1, 2):
            gw = g if wseed is None else inputs.with_weights(g, wseed)
            dgw = dg if wseed is None else fc.DeviceGraph(
                dg.n, dg.row_ptr, dg.col_idx, fc.to_device(gw).weights)
            gs.append(gw)
            dgs.append(dgw)
    jobs = [{"graph": dg, "alpha": 0.5 + i, "stream_id": i, "tree_begin": i, "tree_count": 24,
             "digests": True} for i, dg in enumerate(dgs)]
    b = fc.Batch(jobs, seed=77)
    st = b.run()
    _say(f"weighted batch: {st['sampler']} trees={st['tau']}")
    for i, j in enumerate(jobs):
        ref = oracle.sample(gs[i], j["alpha"], 77, j["tree_begin"], 24, stream=i)
        got = b.result(i)
        assert np.array_equal(got["root_counts"], ref.R), i
        assert np.array_equal(got["tree_digests"], ref.digests), i
    b.close()


def test_weight_validation(gpu_lib):
    fc = gpu_lib
    base = inputs.from_edge_list(3, [(0, 1), (1, 2)])  # entries: 0->1, 1->0, 1->2, 2->1

    def run(w, alpha=1.0):
        g = inputs.CSRGraph(3, base.row_ptr, base.col_idx, "", np.asarray(w, np.float64))
        got = fc.sample(g, alpha=alpha, tree_count=2, want_digests=True)
        ref = oracle.sample(g, alpha, 0, 0, 2)
        assert np.array_equal(got["tree_digests"], ref.digests)

    for w in ([-1.0, -1.0, 1.0, 1.0], [np.nan, np.nan, 1.0, 1.0], [np.inf, np.inf, 1.0, 1.0],
              [2.0**-70, 2.0**-70, 1.0, 1.0], [2.0**65, 2.0**65, 1.0, 1.0],
              [1.0, 2.0, 1.0, 1.0]):
        with pytest.raises(fc.FCError) as e:
            run(w)
        assert e.value.code == fc.FC_ERR_GRAPH, w
    # the accepted range is closed; -0 counts as 0.  (With alpha = 1 the first
    # graph's walk between vertices 1 and 2 would take about 2^32 steps before
    # vertex 1 steps to 0 or u*: alpha must be tiny next to 2^-64.)
    run([2.0**-64, 2.0**-64, 2.0**64, 2.0**64], alpha=2.0**-70)
    run([0.0, -0.0, 1.0, 1.0])
    with pytest.raises(ValueError):
        run([1.0, 1.0, 1.0])


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_weighted_solve_matches_dense(gpu_lib, precision):
    """(alpha L_w + I) X = B with the weighted Laplacian, against a dense solve."""
    fc = gpu_lib
    g = inputs.with_weights(inputs.barabasi_albert(700, 3, 4), 6)
    alpha, k = 1.3, 9
    B = inputs.gaussian(g.n * k, 17).reshape(g.n, k)
    out = fc.solve(g, alpha, B, rtol=1e-10, precision=precision)
    A = alpha * oracle.laplacian(g) + np.eye(g.n)
    Xd = np.linalg.solve(A, B)
    assert (out["relres"] <= 1e-10).all(), out["relres"]
    cond = np.linalg.cond(A)
    assert np.abs(out["X"] - Xd).max() / np.abs(Xd).max() <= 2 * cond * 1e-10
    R = B - A @ out["X"]
    assert np.allclose(np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0), out["relres"],
                       rtol=1e-3, atol=1e-15)
