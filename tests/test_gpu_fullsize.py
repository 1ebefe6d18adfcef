"""GPU parity at the full workload sizes, in the launch configurations the
benchmark times, on outputs the oracle can recompute one by one.

- R-MAT batch: 256 graphs x alpha {0.1, 1, 10} x 512 trees in one autotuned
  persistent launch; root counts of 16 jobs spread over the graph sizes
  against the oracle and against per-job sampling.
- R-MAT 2^22, 1024 trees: per-tree digests of three trees against the
  oracle, and the estimate of Omega_vv against CG on sampled vertices
  within the Hoeffding radius.
- 1000 x 1000 grid with 12% of the edges removed, 1024 trees at alpha = 1
  and 2: per-tree digests and walk steps of sampled trees against the oracle.
- Weighted BA(200000, 5), 4096 trees: per-tree digests and steps of sampled
  trees against the oracle.
(BA(200000, 5) with 4096 trees is in test_gpu_parity.py.)
"""
import sys

import numpy as np
import pytest

import oracle
import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_rmat_batch_full_size_subset_bit_exact(gpu_lib):
    fc = gpu_lib
    gs = inputs.rmat_batch(256, 8, 0)
    dgs = [fc.to_device(g) for g in gs]
    alphas = (0.1, 1.0, 10.0)
    jobs = [{"graph": dg, "alpha": a, "stream_id": gi * 3 + ai, "tree_count": 512}
            for gi, dg in enumerate(dgs) for ai, a in enumerate(alphas)]
    b = fc.Batch(jobs, seed=0, trusted=False, autotune=True)
    st = b.run()
    _say(f"full batch: {st['sampler']} ms={st['ms_sample']:.1f} trees={st['tau']}")
    order = np.argsort([g.n for g in gs], kind="stable")
    picks = [int(order[i]) for i in np.linspace(0, len(gs) - 1, 16).astype(int)]
    for k, gi in enumerate(picks):
        ai = k % 3
        j = gi * 3 + ai
        _say(f"job {j}: n={gs[gi].n} alpha={alphas[ai]}")
        ref = oracle.sample(gs[gi], alphas[ai], 0, 0, 512, stream=j)
        got = b.result(j)["root_counts"]
        assert np.array_equal(got, ref.R), j
        one = fc.sample(dgs[gi], alpha=alphas[ai], seed=0, tree_begin=0, tree_count=512,
                        stream_id=j)
        assert np.array_equal(one["root_counts"], got), j
    assert st["tau"] == 256 * 3 * 512
    b.close()


def test_rmat22_digests_and_estimate(gpu_lib):
    fc = gpu_lib
    g = inputs.rmat(1 << 22, 8, 0)
    dg = fc.to_device(g)
    got = fc.sample(dg, alpha=1.0, seed=0, tree_begin=0, tree_count=1024, want_digests=True,
                    want_steps=True, trusted=False)
    _say(f"rmat22: sampler={got['stats']['sampler']} ms={got['stats']['ms_sample']:.1f}")
    for t in (0, 511, 1023):
        ref = oracle.sample(g, 1.0, 0, t, 1)
        assert got["tree_digests"][t] == ref.digests[0], t
        assert got["tree_steps"][t] == ref.steps[0], t
    R = got["root_counts"].astype(np.float64)
    assert int(R.sum()) == got["stats"]["roots"]
    rng = np.random.default_rng(5)
    vs = rng.choice(g.n, 6, replace=False)
    om = oracle.omega_diag_cg(g, 1.0, vs, rtol=1e-9)
    # Hoeffding radius at delta = 1e-6 over the sampled vertices, 1024 trees
    assert np.abs(R[vs] / 1024 - om).max() < np.sqrt(np.log(2 * len(vs) / 1e-6) / (2 * 1024))


@pytest.mark.parametrize("alpha", [0.5, 1.0, 2.0])
def test_grid_full_size_sampled(gpu_lib, alpha):
    """The road-like workload in the benchmark's launch (1000 x 1000 grid, 12%
    of edges removed, 1024 trees in one call, the automatic choice: the tile
    sampler): trees 0..7 and 1023 against the oracle one by one; all 1024
    trees' digests, steps and root counts against the global-counter sampler
    with and without its re-pops (three schedules, one set of trees)."""
    fc = gpu_lib
    g = inputs.grid_removed(1000, 1000, 0.12, 0)
    dg = fc.to_device(g)
    got = fc.sample(dg, alpha=alpha, seed=0, tree_begin=0, tree_count=1024, want_digests=True,
                    want_steps=True, trusted=True)
    _say(f"grid alpha={alpha}: sampler={got['stats']['sampler']} ms={got['stats']['ms_sample']:.1f}")
    assert got["stats"]["sampler"] == "wilson_tile"
    ref = oracle.sample(g, alpha, 0, 0, 8)
    assert np.array_equal(got["tree_digests"][:8], ref.digests)
    assert np.array_equal(got["tree_steps"][:8], ref.steps)
    ref = oracle.sample(g, alpha, 0, 1023, 1)
    assert got["tree_digests"][1023] == ref.digests[0]
    assert got["tree_steps"][1023] == ref.steps[0]
    assert int(got["root_counts"].astype(np.int64).sum()) == got["stats"]["roots"]
    for repop in (2, 0):
        fc.set_option("coop_repop", repop)
        try:
            other = fc.sample(dg, alpha=alpha, seed=0, tree_begin=0, tree_count=1024,
                              want_digests=True, want_steps=True, trusted=True, sampler="coop")
        finally:
            fc.set_option("coop_repop", 2)
        _say(f"grid alpha={alpha}: global counters, re-pops {repop}: "
             f"ms={other['stats']['ms_sample']:.1f}")
        assert np.array_equal(other["tree_digests"], got["tree_digests"])
        assert np.array_equal(other["tree_steps"], got["tree_steps"])
        assert np.array_equal(other["root_counts"], got["root_counts"])


def test_weighted_ba200k_full_size_sampled(gpu_lib):
    """The weighted workload of the benchmark (BA(200000, 5), log-uniform
    weights in [0.1, 10), alpha = 1, 4096 trees in one call, the LDS sampler
    with first arrows drawn ahead): per-tree digests and steps of sampled trees
    against the oracle, and the totals against the root counts."""
    fc = gpu_lib
    g = inputs.with_weights(inputs.barabasi_albert(200_000, 5, 0), 0)
    dg = fc.to_device(g)
    got = fc.sample(dg, alpha=1.0, seed=0, tree_begin=0, tree_count=4096, want_digests=True,
                    want_steps=True)
    st = got["stats"]
    _say(f"weighted ba200k: sampler={st['sampler']} ms={st['ms_sample']:.1f} predraw={st['ms_predraw']:.1f}")
    assert st["sampler"] == "wilson_lds" and st["ms_predraw"] > 0.0
    for t in (0, 1, 2047, 4095):
        ref = oracle.sample(g, 1.0, 0, t, 1)
        assert got["tree_digests"][t] == ref.digests[0], t
        assert got["tree_steps"][t] == ref.steps[0], t
    assert int(got["root_counts"].astype(np.int64).sum()) == st["roots"]
    assert int(got["tree_steps"].sum()) == st["walk_steps"]
