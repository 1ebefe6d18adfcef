"""GPU parity: the HIP path against the CPU oracle, through the C-ABI.

Sampling is integer work, so the bar is bit-exactness: parent arrays, per
vertex visit counts, root counts, per-tree digests and step counts.  The
estimators are one or two correctly rounded binary64 operations on exact
integers, so they must be bit-equal too.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


SAMPLERS = ["lane", "coop", "lds", "hyb", "tile"]


def _compare(fc, g, alpha, seed, t0, count, stream=0, per_tree=True, sampler="lane"):
    _say(f"parity {sampler} {g.name or g.n} alpha={alpha} seed={seed} "
         f"trees=[{t0},{t0 + count}) stream={stream}")
    got = fc.sample(g, alpha=alpha, seed=seed, tree_begin=t0, tree_count=count, stream_id=stream,
                    want_visits=True, want_digests=True, want_steps=True,
                    want_parents=per_tree, want_tree_visits=per_tree, sampler=sampler)
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
    assert st["digest_sum"] == int(ref.digests.sum(dtype=np.uint64))
    return got, ref


def test_thresholds_match_oracle(gpu_lib):
    fc = gpu_lib
    for alpha in (0.1, 0.5, 1.0, 2.0, 10.0, 1e-17, 3.3e5):
        thr = fc.thresholds(alpha, 5000)
        ref = np.array([oracle.root_threshold(alpha, d) for d in range(5001)], np.uint64)
        assert np.array_equal(thr, ref), alpha


@pytest.mark.parametrize("sampler", SAMPLERS)
def test_er1000_all_trees_bit_exact(gpu_lib, sampler):
    """ER(1000, 0.01), alpha = 1, seed 0: all 2000 trees."""
    g = inputs.erdos_renyi(1000, 0.01, 0)
    _compare(gpu_lib, g, 1.0, 0, 0, 2000, sampler=sampler)


def test_er1000_estimators_bit_exact(gpu_lib):
    fc = gpu_lib
    g = inputs.erdos_renyi(1000, 0.01, 0)
    out = fc.farness(g, alpha=1.0, seed=0, tau=2000)
    ref = oracle.sample(g, 1.0, 0, 0, 2000)
    d, f, c = oracle.estimate(ref.R, 2000)
    assert np.array_equal(out["root_counts"], ref.R)
    assert np.array_equal(out["diag"], d)
    assert np.array_equal(out["farness"], f)
    assert np.array_equal(out["closeness"], c)
    # Algorithm 1 with tau from (eps, delta) and the literal last-loop reading
    out2 = fc.diag_estimate(g, alpha=1.0, eps=0.1, delta=0.1, seed=0, literal=True)
    t = oracle.tau(g.m, g.n, 0.1, 0.1)
    assert out2["tau"] == t == 576
    ref2 = oracle.sample(g, 1.0, 0, 0, t)
    dl, _, _ = oracle.estimate(ref2.R, t, literal=True)
    assert np.array_equal(out2["diag"], dl)
    # and the (eps, delta) guarantee against the dense forest matrix
    Om = oracle.forest_matrix(g, 1.0)
    direct = fc.diag_estimate(g, alpha=1.0, eps=0.1, delta=0.1, seed=0)
    assert np.abs(direct["diag"] - np.diag(Om)).max() < 0.1


@pytest.mark.parametrize("sampler", SAMPLERS)
@pytest.mark.parametrize("case", ["single_vertex", "isolated", "edge", "star", "path", "k6",
                                  "triangle_isolated", "ragged_er", "two_components"])
def test_small_and_degenerate_graphs(gpu_lib, case, sampler):
    E = {
        "single_vertex": (1, []),
        "isolated": (37, []),
        "edge": (2, [(0, 1)]),
        "star": (65, [(0, i) for i in range(1, 65)]),
        "path": (130, [(i, i + 1) for i in range(129)]),
        "k6": (6, [(a, b) for a in range(6) for b in range(a + 1, 6)]),
        "triangle_isolated": (5, [(0, 1), (1, 2), (0, 2)]),
        "two_components": (9, [(0, 1), (1, 2), (2, 3), (5, 6), (6, 7), (7, 8), (8, 5)]),
    }
    if case == "ragged_er":
        g = inputs.erdos_renyi(333, 0.03, 9)
    else:
        n, e = E[case]
        g = inputs.from_edge_list(n, e, case)
    for alpha in (0.3, 1.0, 7.0):
        _compare(gpu_lib, g, alpha, 1234567890123, 17, 97, stream=3, sampler=sampler)


@pytest.mark.parametrize("shape", ["full", "lean"])
@pytest.mark.parametrize("case", ["path5000", "bundle200x100"])
def test_long_peel_chains_bit_exact(gpu_lib, case, shape):
    """Arrow forests with thousands of peel levels (alpha = 50: roots are rare):
    a path of 5000 vertices (single-wave levels in many 63-level batches and
    register windows) and 200 disjoint paths of 100 vertices (about 200 entries
    per level: the register-held middle levels for a hundred levels), in both
    register shapes of the LDS sampler, against the oracle."""
    fc = gpu_lib
    if case == "path5000":
        g = inputs.from_edge_list(5000, [(i, i + 1) for i in range(4999)], case)
    else:
        g = inputs.from_edge_list(20_000, [(100 * p + i, 100 * p + i + 1) for p in range(200)
                                           for i in range(99)], case)
    try:
        if shape == "lean":
            fc.set_option("lds_lean", 1)
            fc.set_option("lds_threads", 256)
        for repop in (3, 0):
            fc.set_option("lds_repop", repop)
            _compare(fc, g, 50.0, 31, 0, 12, per_tree=False, sampler="lds")
    finally:
        fc.set_option("lds_lean", 0)
        fc.set_option("lds_threads", 0)
        fc.set_option("lds_repop", 3)


def test_empty_graph_and_zero_trees(gpu_lib):
    fc = gpu_lib
    g0 = inputs.from_edge_list(0, [])
    r = fc.sample(g0, alpha=1.0, tree_count=5, want_digests=True)
    assert r["root_counts"].size == 0
    out = fc.diag_estimate(g0, alpha=1.0, tau=10)
    assert out["diag"].size == 0
    g = inputs.erdos_renyi(50, 0.1, 2)
    r = fc.sample(g, alpha=1.0, tree_count=0, want_visits=True)
    assert (r["root_counts"] == 0).all() and (r["visit_counts"] == 0).all()


def test_tree_ranges_streams_and_device_graph(gpu_lib):
    fc = gpu_lib
    g = inputs.barabasi_albert(3000, 4, 5)
    a = fc.sample(g, alpha=0.8, seed=9, tree_begin=0, tree_count=40, want_digests=True)
    b = fc.sample(g, alpha=0.8, seed=9, tree_begin=40, tree_count=25, want_digests=True)
    c = fc.sample(g, alpha=0.8, seed=9, tree_begin=0, tree_count=65, want_digests=True)
    assert np.array_equal(a["root_counts"] + b["root_counts"], c["root_counts"])
    assert np.array_equal(np.concatenate([a["tree_digests"], b["tree_digests"]]), c["tree_digests"])
    dg = fc.to_device(g)
    d = fc.sample(dg, alpha=0.8, seed=9, tree_begin=0, tree_count=65, want_digests=True)
    assert np.array_equal(d["tree_digests"], c["tree_digests"])
    ref = oracle.sample(g, 0.8, 9, 0, 65, stream=0)
    assert np.array_equal(c["root_counts"], ref.R)
    s1 = fc.sample(g, alpha=0.8, seed=9, tree_count=10, stream_id=1, want_digests=True)
    ref1 = oracle.sample(g, 0.8, 9, 0, 10, stream=1)
    assert np.array_equal(s1["tree_digests"], ref1.digests)


@pytest.mark.parametrize("sampler", SAMPLERS)
def test_counter_words_at_their_limits(gpu_lib, sampler):
    """The last tree ids of the 32-bit range, the largest stream id and a
    64-bit seed with every bit set: the Philox counter and key words at their
    extremes (BA(20000, 3): the LDS sampler also draws the first arrows
    ahead here).  A range past 2^32 is rejected."""
    fc = gpu_lib
    g = inputs.barabasi_albert(20_000, 3, 3)
    _compare(fc, g, 1.0, (1 << 64) - 1, (1 << 32) - 6, 6, stream=(1 << 32) - 1, sampler=sampler)
    with pytest.raises(fc.FCError) as e:
        fc.sample(g, alpha=1.0, tree_begin=(1 << 32) - 2, tree_count=3, sampler=sampler)
    assert e.value.code == fc.FC_ERR_ARG


@pytest.mark.parametrize("sampler", SAMPLERS)
def test_root_test_boundary(gpu_lib, sampler):
    """alpha chosen so that thr(1) equals x0 of vertex 0's first arrow in tree
    0 (seed 0): both sides must take the strict comparison."""
    x0 = int(oracle.philox4x32_10([0, 0, 0, 0], [0, 0])[0])
    alpha = 2.0**32 / (x0 + 0.5) - 1.0
    assert oracle.root_threshold(alpha, 1) == x0
    g = inputs.from_edge_list(2, [(0, 1)])
    _compare(gpu_lib, g, alpha, 0, 0, 4, sampler=sampler)


def test_graph_validation_errors(gpu_lib):
    fc = gpu_lib

    def bad(n, rp, ci):
        g = inputs.CSRGraph(n, np.asarray(rp, np.int32), np.asarray(ci, np.int32))
        with pytest.raises(fc.FCError) as e:
            fc.sample(g, alpha=1.0, tree_count=1)
        return e.value.code

    assert bad(3, [0, 1, 1, 1], [1]) == fc.FC_ERR_GRAPH            # asymmetric
    assert bad(2, [0, 1, 2], [0, 1]) == fc.FC_ERR_GRAPH            # self-loops
    assert bad(3, [0, 2, 3, 4], [2, 1, 0, 0]) == fc.FC_ERR_GRAPH   # unsorted row
    assert bad(2, [0, 1, 2], [1, 5]) == fc.FC_ERR_GRAPH            # column out of range
    assert bad(2, [0, 2, 1], [1, 0]) == fc.FC_ERR_GRAPH            # row_ptr decreasing
    assert bad(2, [1, 1, 2], [1, 0]) == fc.FC_ERR_GRAPH            # row_ptr[0] != 0
    with pytest.raises(fc.FCError) as e:
        fc.sample(inputs.erdos_renyi(10, 0.3, 1), alpha=0.0, tree_count=1)
    assert e.value.code == fc.FC_ERR_ARG
    with pytest.raises(fc.FCError) as e:
        fc.diag_estimate(inputs.erdos_renyi(10, 0.3, 1), alpha=1.0, eps=1.5)
    assert e.value.code == fc.FC_ERR_ARG


@pytest.mark.parametrize("sampler", SAMPLERS)
def test_ba200k_tree_subset_bit_exact(gpu_lib, sampler):
    """BA(200000, 5), alpha = 1: the first 48 trees and a later range."""
    g = inputs.barabasi_albert(200_000, 5, 0)
    _compare(gpu_lib, g, 1.0, 0, 0, 48, sampler=sampler)
    _compare(gpu_lib, g, 1.0, 0, 4000, 16, per_tree=False, sampler=sampler)


@pytest.mark.parametrize("sampler", ["lane", "coop", "hyb"])
@pytest.mark.parametrize("alpha", [0.5, 1.0, 2.0])
def test_grid_tree_subset_bit_exact(gpu_lib, alpha, sampler):
    """1000 x 1000 grid with 12% of edges removed: 16 trees per alpha."""
    g = inputs.grid_removed(1000, 1000, 0.12, 0)
    _compare(gpu_lib, g, alpha, 0, 100, 16, per_tree=sampler == "coop", sampler=sampler)


@pytest.mark.parametrize("sampler", SAMPLERS)
def test_draw_limit_reports_overflow(gpu_lib, sampler):
    """The per-vertex draw-count limit (forced down with option max_draws)
    turns into FC_ERR_OVERFLOW; at the largest count the oracle sees, the run
    succeeds and matches it."""
    fc = gpu_lib
    g = inputs.erdos_renyi(200, 0.05, 3)
    ref = oracle.sample(g, 1.0, 9, 0, 8, per_tree=True)
    kmax = int(ref.tree_visits.max())
    assert kmax >= 2
    fc.set_option("max_draws", kmax - 1)
    try:
        with pytest.raises(fc.FCError) as e:
            fc.sample(g, alpha=1.0, seed=9, tree_begin=0, tree_count=8, sampler=sampler)
        assert e.value.code == fc.FC_ERR_OVERFLOW
        fc.set_option("max_draws", kmax)
        got = fc.sample(g, alpha=1.0, seed=9, tree_begin=0, tree_count=8, want_digests=True,
                        sampler=sampler)
        assert np.array_equal(got["tree_digests"], ref.digests)
    finally:
        fc.set_option("max_draws", 0)


def test_lds_sampler_rejects_graphs_too_large_and_auto_falls_back(gpu_lib):
    """10^6 vertices need at least 610 KiB of 4-bit counters: forcing the
    LDS-counter sampler fails cleanly; the automatic choice is the tile
    sampler (the grid's row-major ids keep 98% of the edges inside a tile),
    or global counters when no share of crossing edges is accepted."""
    fc = gpu_lib
    g = inputs.grid_removed(1000, 1000, 0.12, 0)
    with pytest.raises(fc.FCError) as e:
        fc.sample(g, alpha=1.0, seed=0, tree_begin=0, tree_count=2, sampler="lds")
    assert e.value.code == fc.FC_ERR_UNSUPPORTED
    ref = oracle.sample(g, 1.0, 0, 0, 2, per_tree=False)
    got = fc.sample(g, alpha=1.0, seed=0, tree_begin=0, tree_count=2, want_digests=True)
    assert got["stats"]["sampler"] == "wilson_tile"
    assert np.array_equal(got["tree_digests"], ref.digests)
    fc.set_option("tile_cross_permille", 0)
    try:
        got = fc.sample(g, alpha=1.0, seed=0, tree_begin=0, tree_count=2, want_digests=True)
    finally:
        fc.set_option("tile_cross_permille", 100)
    assert got["stats"]["sampler"] == "wilson_coop"
    assert np.array_equal(got["tree_digests"], ref.digests)


@pytest.mark.parametrize("threads,wg", [(64, 8), (256, 2), (512, 1), (1024, 2), (128, 0)])
def test_lds_launch_shapes_bit_exact(gpu_lib, threads, wg):
    """LDS-counter sampler with other workgroup sizes and residency caps."""
    fc = gpu_lib
    fc.set_option("lds_threads", threads)
    fc.set_option("lds_wg_per_cu", wg)
    try:
        g = inputs.barabasi_albert(20_000, 3, 7)
        _compare(fc, g, 1.5, 77, 9, 40, sampler="lds")
        g2 = inputs.grid_removed(120, 90, 0.12, 3)
        _compare(fc, g2, 2.0, 78, 0, 20, sampler="lds")
    finally:
        fc.set_option("lds_threads", 0)
        fc.set_option("lds_wg_per_cu", 0)


@pytest.mark.parametrize("mib", [0, 1, 32768], ids=["off", "over_budget", "default"])
def test_lds_first_arrows_drawn_ahead_or_in_place(gpu_lib, mib):
    """The LDS sampler's first arrows, drawn by the vertex-major pre-draw
    kernel (the default when every tree's words fit the budget) or by each
    tree's workgroup (budget 0, a budget too small: 40 trees of 20000 vertices
    need 6.1 MiB, more than 1 MiB, or fewer than 16384 non-isolated vertices),
    give the oracle's trees."""
    fc = gpu_lib
    fc.set_option("predraw_mib", mib)

    def drawn_ahead(g, trees):
        non_isolated = int((np.diff(g.row_ptr) > 0).sum())
        return mib > 0 and non_isolated >= 16384 and 8 * g.n * trees <= mib << 20

    try:
        g = inputs.barabasi_albert(20_000, 3, 7)
        got, _ = _compare(fc, g, 1.5, 77, 9, 40, sampler="lds")
        assert (got["stats"]["ms_predraw"] > 0.0) == drawn_ahead(g, 40)
        # isolated vertices and a tree range not starting at 0
        g2 = inputs.rmat(40_000, 8, 5)
        got, _ = _compare(fc, g2, 0.3, 5, 1000, 6, stream=7, sampler="lds")
        assert (got["stats"]["ms_predraw"] > 0.0) == drawn_ahead(g2, 6)
        # too small to draw ahead
        g3 = inputs.rmat(3000, 8, 5)
        got, _ = _compare(fc, g3, 0.3, 5, 1000, 33, stream=7, sampler="lds")
        assert got["stats"]["ms_predraw"] == 0.0
    finally:
        fc.set_option("predraw_mib", 32768)


def test_lds_counter_classes_and_size_limit(gpu_lib):
    """A star whose centre has degree 70000 needs a 32-bit field (the widest
    class); BA(250000, 3) needs 161.8 KB of fields and bitmap, just inside
    gfx950's 160 KiB of LDS; BA(262000, 3) is beyond it and runs on global
    counters.  All three match the oracle tree for tree."""
    fc = gpu_lib
    star = inputs.from_edge_list(70001, [(0, i) for i in range(1, 70001)], "star70000")
    got, _ = _compare(fc, star, 0.5, 21, 0, 12, per_tree=True, sampler="lds")
    near = inputs.barabasi_albert(250_000, 3, 1)
    got = fc.sample(near, alpha=1.0, seed=2, tree_begin=0, tree_count=8, want_digests=True)
    assert got["stats"]["sampler"] == "wilson_lds"
    assert np.array_equal(got["tree_digests"], oracle.sample(near, 1.0, 2, 0, 8).digests)
    over = inputs.barabasi_albert(262_000, 3, 1)
    got = fc.sample(over, alpha=1.0, seed=2, tree_begin=0, tree_count=8, want_digests=True)
    assert got["stats"]["sampler"] == "wilson_coop"
    assert np.array_equal(got["tree_digests"], oracle.sample(over, 1.0, 2, 0, 8).digests)


@pytest.mark.parametrize("cap", [0, 1, 100, 5000])
def test_hybrid_hot_prefix_sizes_bit_exact(gpu_lib, cap):
    """Hybrid sampler with at most `cap` vertices in LDS (0: every counter and
    settled bit global; the rest: a split between LDS and global memory that
    falls inside different degree classes)."""
    fc = gpu_lib
    fc.set_option("hyb_hot_cap", cap)
    try:
        _compare(fc, inputs.barabasi_albert(20_000, 3, 7), 1.5, 77, 9, 24, sampler="hyb")
        _compare(fc, inputs.rmat(1 << 14, 8, 12), 1.0, 5, 0, 16, sampler="hyb")
        _compare(fc, inputs.grid_removed(120, 90, 0.12, 3), 2.0, 78, 0, 12, sampler="hyb")
    finally:
        fc.set_option("hyb_hot_cap", 0x7FFFFFFF)


def test_auto_choice_prefers_lds_counters(gpu_lib):
    """Without a sampler flag a tree that fits uses LDS counters; the option
    turns that off."""
    fc = gpu_lib
    g = inputs.barabasi_albert(70_000, 4, 5)
    got = fc.sample(g, alpha=1.0, seed=3, tree_begin=0, tree_count=8, want_digests=True)
    assert got["stats"]["sampler"] == "wilson_lds"
    fc.set_option("coop_lds_counts", 0)
    try:
        got2 = fc.sample(g, alpha=1.0, seed=3, tree_begin=0, tree_count=8, want_digests=True)
        assert got2["stats"]["sampler"] == "wilson_coop"
    finally:
        fc.set_option("coop_lds_counts", 1)
    assert np.array_equal(got["tree_digests"], got2["tree_digests"])


@pytest.mark.parametrize("repop", [0, 2], ids=["repop_off", "repop_on"])
@pytest.mark.parametrize("case", ["ba20k", "grid", "matching", "path", "cycles", "w64"])
def test_coop_repop_bit_exact(gpu_lib, repop, case):
    """The global-counter sampler with and without popping re-formed 2-cycles
    within their round (option coop_repop): the same trees as the oracle,
    unweighted and weighted; a perfect matching has one count bit per word (the
    pass mark then fills it), "w64" forces 64-bit words and a global settled
    bitmap (the filter then sits alone in LDS)."""
    fc = gpu_lib
    g = {"ba20k": lambda: inputs.barabasi_albert(20_000, 3, 4),
         "grid": lambda: inputs.grid_removed(90, 110, 0.12, 2),
         "matching": lambda: inputs.from_edge_list(2000, [(2 * i, 2 * i + 1) for i in range(1000)]),
         "path": lambda: inputs.from_edge_list(3000, [(i, i + 1) for i in range(2999)]),
         "cycles": lambda: inputs.from_edge_list(
             999, [(i, 3 * (i // 3) + (i + 1) % 3) for i in range(999)]),
         "w64": lambda: inputs.barabasi_albert(5000, 4, 9)}[case]()
    fc.set_option("coop_repop", repop)
    if case == "w64":
        fc.set_option("coop_word32", 0)
        fc.set_option("coop_lds_bits", 0)
    try:
        for gg, alpha in ((g, 1.0), (inputs.with_weights(g, 7), 2.0)):
            _compare(fc, gg, alpha, 3, 0, 40, per_tree=True, sampler="coop")
    finally:
        fc.set_option("coop_repop", 2)
        fc.set_option("coop_word32", 1)
        fc.set_option("coop_lds_bits", 1)


@pytest.mark.parametrize("shape", [(64, 1, 1, 1, 1), (256, 3, 0, 1, 1), (448, 1, 1, 0, 0),
                                   (512, 2, 0, 0, 0), (512, 4, 1, 1, 0), (256, 2, 1, 0, 1)])
def test_coop_launch_shapes_bit_exact(gpu_lib, shape):
    """Workgroup sampler under other launch shapes, with the settled bitmap
    in LDS or global memory, with or without the in-arrow bitmap, 32- and
    64-bit tree words: identical results."""
    fc = gpu_lib
    threads, wg, lds, w32, inb = shape
    fc.set_option("coop_threads", threads)
    fc.set_option("coop_wg_per_cu", wg)
    fc.set_option("coop_lds_bits", lds)
    fc.set_option("coop_word32", w32)
    fc.set_option("coop_in_bits", inb)
    try:
        g = inputs.barabasi_albert(20_000, 3, 7)
        _compare(fc, g, 1.5, 77, 9, 40, sampler="coop")
        g2 = inputs.grid_removed(120, 90, 0.12, 3)
        _compare(fc, g2, 2.0, 78, 0, 20, sampler="coop")
    finally:
        fc.set_option("coop_threads", 512)
        fc.set_option("coop_wg_per_cu", 3)
        fc.set_option("coop_lds_bits", 1)
        fc.set_option("coop_word32", 1)
        fc.set_option("coop_in_bits", 1)


def test_set_option_rejects_bad_values(gpu_lib):
    fc = gpu_lib
    for key, val in (("coop_threads", 100), ("coop_threads", 1024), ("coop_wg_per_cu", 0),
                     ("lanes_per_wave", 65), ("nonsense", 1), ("coop_lds_bits", 2),
                     ("coop_lds_counts", 2), ("lds_threads", 1088), ("lds_threads", 96),
                     ("lds_wg_per_cu", -1), ("lds_wg_per_cu", 65), ("hyb_hot_cap", -1),
                     ("coop_repop", 3), ("coop_repop", -1),
                     ("max_draws", -1),
                     ("max_draws", 1 << 31)):
        with pytest.raises(fc.FCError) as e:
            fc.set_option(key, val)
        assert e.value.code == fc.FC_ERR_ARG


@pytest.mark.parametrize("sampler", SAMPLERS)
def test_rmat_heavy_tail_bit_exact(gpu_lib, sampler):
    """R-MAT (2^15 vertices, edge factor 8) at alpha = 10 and 0.1: hubs,
    isolated vertices and many popping rounds."""
    g = inputs.rmat(1 << 15, 8, 11)
    for alpha in (10.0, 0.1):
        _compare(gpu_lib, g, alpha, 5, 0, 24, sampler=sampler)


def test_ba200k_full_run_sampled(gpu_lib):
    """The benchmark's configuration (BA(200000, 5), alpha = 1, 4096 trees):
    per-tree digests and steps of trees 0..63 and of a spread of later tree
    ids recomputed by the oracle, exact totals, and the estimate against CG on
    sampled vertices."""
    fc = gpu_lib
    g = inputs.barabasi_albert(200_000, 5, 0)
    dg = fc.to_device(g)
    got = fc.sample(dg, alpha=1.0, seed=0, tree_begin=0, tree_count=4096, want_digests=True,
                    want_steps=True, trusted=True)
    _say(f"full run sampler={got['stats']['sampler']} ms={got['stats']['ms_sample']:.1f}")
    # the benchmark's launch: LDS counters, first arrows drawn ahead
    assert got["stats"]["sampler"] == "wilson_lds" and got["stats"]["ms_predraw"] > 0.0
    # every tree of the first 64 (a quarter of the trees the first wave of
    # workgroups samples), then a spread of later ones
    ref = oracle.sample(g, 1.0, 0, 0, 64)
    assert np.array_equal(got["tree_digests"][:64], ref.digests)
    assert np.array_equal(got["tree_steps"][:64], ref.steps)
    for t in (777, 2048, 4095):
        ref = oracle.sample(g, 1.0, 0, t, 1)
        assert got["tree_digests"][t] == ref.digests[0], t
        assert got["tree_steps"][t] == ref.steps[0], t
    R = got["root_counts"].astype(np.float64)
    assert int(R.sum()) == got["stats"]["roots"]
    rng = np.random.default_rng(3)
    vs = rng.choice(g.n, 64, replace=False)
    om = oracle.omega_diag_cg(g, 1.0, vs, rtol=1e-9)  # Section 6.1's protocol, 64 vertices
    # Hoeffding radius at delta = 1e-6 over 64 vertices with 4096 trees
    assert np.abs(R[vs] / 4096 - om).max() < np.sqrt(np.log(2 * 64 / 1e-6) / (2 * 4096))


# --------------------------------------------------------------------------
# Batches (many graphs x alphas in one persistent launch)
# --------------------------------------------------------------------------
def _batch_graphs():
    sizes = inputs.rmat_batch_sizes(6, 5, lo_exp=7.0, hi_exp=12.0)
    gs = [inputs.rmat(nn, 8, 100 + i) for i, nn in enumerate(sizes)]
    gs.append(inputs.barabasi_albert(5000, 3, 2))
    # 100000 vertices need more than a third of the LDS for their counters:
    # with LDS counters the batch runs as two launch groups
    gs.append(inputs.barabasi_albert(100_000, 3, 4))
    gs.append(inputs.grid_removed(40, 50, 0.12, 1))
    gs.append(inputs.from_edge_list(3, [(0, 1)], "edge_plus_isolated"))
    return gs


@pytest.fixture(params=[1, 0], ids=["lds_counters", "global_counters"])
def counters(request, gpu_lib):
    """Runs a test with the workgroup kernels' in-arrow counters in LDS (the
    default) and in global tree words."""
    gpu_lib.set_option("coop_lds_counts", request.param)
    yield "lbatch" if request.param else "batch"
    gpu_lib.set_option("coop_lds_counts", 1)


def test_batch_matches_oracle_and_single_runs(gpu_lib, counters):
    fc = gpu_lib
    gs = _batch_graphs()
    dgs = [fc.to_device(g) for g in gs]
    alphas = (0.1, 1.0, 10.0)
    jobs = []
    for gi, dg in enumerate(dgs):
        for ai, a in enumerate(alphas):
            jobs.append({"graph": dg, "alpha": a, "stream_id": gi * len(alphas) + ai,
                         "tree_begin": 3 * ai, "tree_count": 20 + 5 * ai, "digests": True})
    # edge jobs: no trees, and an empty graph
    jobs.append({"graph": dgs[0], "alpha": 1.0, "tree_count": 0})
    jobs.append({"graph": fc.to_device(inputs.from_edge_list(0, [])), "alpha": 1.0, "tree_count": 4})
    b = fc.Batch(jobs, seed=4242)
    st = b.run()
    _say(f"batch run: {st['sampler']} ms={st['ms_sample']:.2f} trees={st['tau']}")
    assert st["sampler"].split(":")[0] == counters
    if counters == "lbatch":
        assert "+" in st["sampler"]  # two launch groups
    total_steps = 0
    for i, j in enumerate(jobs[:-2]):
        g = gs[i // len(alphas)]
        ref = oracle.sample(g, j["alpha"], 4242, j["tree_begin"], j["tree_count"],
                            stream=j["stream_id"])
        got = b.result(i)
        assert np.array_equal(got["root_counts"], ref.R), i
        assert np.array_equal(got["tree_digests"], ref.digests), i
        total_steps += int(ref.steps.sum())
        one = fc.sample(dgs[i // len(alphas)], alpha=j["alpha"], seed=4242,
                        tree_begin=j["tree_begin"], tree_count=j["tree_count"],
                        stream_id=j["stream_id"], want_digests=True, sampler="coop")
        assert np.array_equal(one["root_counts"], got["root_counts"])
    assert st["walk_steps"] == total_steps
    b.close()


def test_batch_graph_replays_and_autotune(gpu_lib, counters):
    """Replays of the captured launch, with eager work and synchronisation
    between them, each equal to the eager single-job result."""
    import torch
    fc = gpu_lib
    all_gs = _batch_graphs()
    gs = all_gs[:4] + [all_gs[7]]  # small R-MAT graphs and BA(80000, 3): two launch groups
    dgs = [fc.to_device(g) for g in gs]
    jobs = [{"graph": dg, "alpha": 1.0, "stream_id": i, "tree_count": 33, "digests": True}
            for i, dg in enumerate(dgs)]
    eager = [fc.sample(dg, alpha=1.0, seed=7, tree_count=33, stream_id=i, want_digests=True)
             for i, dg in enumerate(dgs)]
    for tune in (False, True):
        b = fc.Batch(jobs, seed=7, autotune=tune)
        assert b.run()["sampler"].split(":")[0] == counters
        for rep in range(3):
            b.reset()
            x = torch.randn(1 << 20, device="cuda:0")  # unrelated eager work in between
            x.mul_(2.0).sum().item()
            torch.cuda.synchronize()
            b.run()
            for i in range(len(jobs)):
                got = b.result(i)
                assert np.array_equal(got["root_counts"], eager[i]["root_counts"]), (tune, rep, i)
                assert np.array_equal(got["tree_digests"], eager[i]["tree_digests"]), (tune, rep, i)
        # without a reset the counts accumulate
        b.run()
        assert np.array_equal(b.result(0)["root_counts"], 2 * eager[0]["root_counts"])
        b.close()


def test_batch_autotune_cached_and_repop_values(gpu_lib):
    """A batch created again with the same job shapes takes the cached launch
    shape (the same shape string, the same trees); every lds_repop value,
    tuned (3) or fixed (0, 1, 2), gives the eager trees."""
    fc = gpu_lib
    gs = _batch_graphs()[:3]
    dgs = [fc.to_device(g) for g in gs]
    jobs = [{"graph": dg, "alpha": 2.0, "stream_id": i, "tree_count": 40, "digests": True}
            for i, dg in enumerate(dgs)]
    eager = [fc.sample(dg, alpha=2.0, seed=3, tree_count=40, stream_id=i, want_digests=True)
             for i, dg in enumerate(dgs)]
    try:
        for repop in (3, 2, 1, 0):
            fc.set_option("lds_repop", repop)
            shapes = []
            for _ in range(2):
                b = fc.Batch(jobs, seed=3, autotune=True)
                shapes.append(b.run()["sampler"])
                for i in range(len(jobs)):
                    got = b.result(i)
                    assert np.array_equal(got["tree_digests"], eager[i]["tree_digests"]), (repop, i)
                    assert np.array_equal(got["root_counts"], eager[i]["root_counts"]), (repop, i)
                b.close()
            assert shapes[0] == shapes[1], shapes
        with pytest.raises(fc.FCError):
            fc.set_option("lds_repop", 4)
    finally:
        fc.set_option("lds_repop", 3)


_TUNE_CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import paper_2101_06192_amd as fc
import inputs
gs = [inputs.rmat(n, 8, 40 + i) for i, n in enumerate((700, 1500, 2900))]
dgs = [fc.to_device(g) for g in gs]
jobs = [{"graph": dg, "alpha": 0.7, "stream_id": i, "tree_count": 37, "digests": True}
        for i, dg in enumerate(dgs)]
b = fc.Batch(jobs, seed=11, autotune=True)
st = b.run()
d = [int(x) for i in range(len(jobs)) for x in b.result(i)["tree_digests"]]
print(st["sampler"], sum(d) % (1 << 61))
b.close()
"""


def test_batch_tune_cache_on_disk(gpu_lib, tmp_path):
    """FC_TUNE_CACHE: a process appends its tuned choice to the file; a later
    process with the same job shapes reads it back instead of tuning (nothing
    appended) and samples the same trees."""
    import os
    import subprocess
    import sys as _sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    path = tmp_path / "tune.txt"
    env = dict(os.environ, FC_TUNE_CACHE=str(path))
    outs = []
    for _ in range(2):
        r = subprocess.run([_sys.executable, "-c", _TUNE_CHILD, root], env=env, capture_output=True,
                           text=True, timeout=240)
        assert r.returncode == 0, r.stderr[-2000:]
        outs.append(r.stdout.strip().splitlines()[-1])
        if len(outs) == 1:
            lines = path.read_text().splitlines()
            assert len(lines) >= 1
    assert path.read_text().splitlines() == lines  # read back, not tuned again
    assert outs[0] == outs[1]


@pytest.mark.parametrize("weighted", [False, True], ids=["unweighted", "weighted"])
@pytest.mark.parametrize("repop", [2, 0], ids=["repop", "no_repop"])
def test_lds_lean_shape_bit_exact(gpu_lib, weighted, repop):
    """The LDS sampler's lean register shape (option lds_lean, 256- and 512-thread
    workgroups): every tree against the oracle on an R-MAT graph at alpha = 10
    (long peel chains: the single-wave and middle levels) and on a BA graph; then
    an untuned batch in the lean shape against the eager runs."""
    fc = gpu_lib
    gs = [inputs.rmat(3000, 8, 7), inputs.barabasi_albert(20_000, 5, 3)]
    if weighted:
        gs = [inputs.with_weights(g, 5) for g in gs]
    try:
        fc.set_option("lds_repop", repop)
        fc.set_option("lds_lean", 1)
        for threads, g, alpha, count in ((256, gs[0], 10.0, 40), (512, gs[1], 1.0, 24)):
            fc.set_option("lds_threads", threads)
            _compare(fc, g, alpha, 77, 5, count, stream=2, per_tree=False, sampler="lds")
        fc.set_option("lds_threads", 256)
        dgs = [fc.to_device(g) for g in gs]
        jobs = [{"graph": dg, "alpha": a, "stream_id": i, "tree_count": 30, "digests": True}
                for i, dg in enumerate(dgs) for a in (1.0, 10.0)]
        b = fc.Batch(jobs, seed=9)
        st = b.run()
        _say(f"lean batch: {st['sampler']}")
        for i, j in enumerate(jobs):
            one = fc.sample(j["graph"], alpha=j["alpha"], seed=9, tree_count=30,
                            stream_id=j["stream_id"], want_digests=True, sampler="coop")
            got = b.result(i)
            assert np.array_equal(got["tree_digests"], one["tree_digests"]), i
            assert np.array_equal(got["root_counts"], one["root_counts"]), i
        b.close()
        with pytest.raises(fc.FCError):
            fc.set_option("lds_lean", 2)
    finally:
        fc.set_option("lds_lean", 0)
        fc.set_option("lds_threads", 0)
        fc.set_option("lds_repop", 3)


def test_batch_rejects_host_graphs_and_bad_alpha(gpu_lib):
    fc = gpu_lib
    g = inputs.erdos_renyi(30, 0.2, 1)
    with pytest.raises(TypeError):
        fc.Batch([{"graph": g, "alpha": 1.0, "tree_count": 2}])
    with pytest.raises(fc.FCError) as e:
        fc.Batch([{"graph": fc.to_device(g), "alpha": -1.0, "tree_count": 2}])
    assert e.value.code == fc.FC_ERR_ARG


# --------------------------------------------------------------------------
# Linear solves (alpha L + I) X = B, binary64 and binary32-refined
# --------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
@pytest.mark.parametrize("k", [1, 5, 37, 64])
def test_solve_matches_dense(gpu_lib, precision, k):
    fc = gpu_lib
    g = inputs.barabasi_albert(700, 3, 4)
    alpha = 1.3
    B = inputs.gaussian(g.n * k, 10 + k).reshape(g.n, k)
    out = fc.solve(g, alpha, B, rtol=1e-10, precision=precision)
    A = alpha * oracle.laplacian(g) + np.eye(g.n)
    Xd = np.linalg.solve(A, B)
    assert (out["relres"] <= 1e-10).all(), out["relres"]
    # relative residual bound -> error bound: |x - x*| <= cond(A) rtol |x*|
    cond = np.linalg.cond(A)
    err = np.abs(out["X"] - Xd).max() / np.abs(Xd).max()
    assert err <= 2 * cond * 1e-10, (err, cond)
    # the residual reported is the true binary64 residual
    R = B - A @ out["X"]
    assert np.allclose(np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0), out["relres"],
                       rtol=1e-3, atol=1e-15)


def test_solve_precisions_agree_and_initial_guess(gpu_lib):
    fc = gpu_lib
    g = inputs.grid_removed(30, 40, 0.12, 2)
    B = inputs.gaussian(g.n * 8, 3).reshape(g.n, 8)
    a = fc.solve(g, 2.0, B, rtol=1e-11, precision="fp64")
    b = fc.solve(g, 2.0, B, rtol=1e-11, precision="fp32_refined")
    assert np.abs(a["X"] - b["X"]).max() < 1e-8 * np.abs(a["X"]).max()
    # warm start from the solution: no iterations needed
    c = fc.solve(g, 2.0, B, X0=a["X"], rtol=1e-9, precision="fp32_refined")
    assert c["iters"] == 0 and (c["relres"] <= 1e-9).all()
    # zero right-hand side column stays zero
    B[:, 3] = 0.0
    d = fc.solve(g, 2.0, B, rtol=1e-9)
    assert (d["X"][:, 3] == 0.0).all()


def test_solve_omega_diagonal(gpu_lib):
    """Columns e_v give Omega e_v: the diagonal matches the dense forest matrix."""
    fc = gpu_lib
    g = inputs.erdos_renyi(1000, 0.01, 0)
    vs = np.arange(0, 1000, 16)[:64]
    B = np.zeros((g.n, len(vs)))
    B[vs, np.arange(len(vs))] = 1.0
    out = fc.solve(g, 1.0, B, rtol=1e-9, precision="fp32_refined")
    Om = oracle.forest_matrix(g, 1.0)
    assert np.abs(out["X"][vs, np.arange(len(vs))] - np.diag(Om)[vs]).max() < 1e-8


def test_solve_argument_errors(gpu_lib):
    fc = gpu_lib
    g = inputs.erdos_renyi(50, 0.1, 1)
    with pytest.raises(fc.FCError) as e:
        fc.solve(g, 1.0, np.ones((50, 65)))
    assert e.value.code == fc.FC_ERR_UNSUPPORTED
    with pytest.raises(fc.FCError) as e:
        fc.solve(g, 0.0, np.ones((50, 2)))
    assert e.value.code == fc.FC_ERR_ARG
    with pytest.raises(fc.FCError) as e:
        fc.solve(g, 1.0, np.ones((50, 2)), rtol=0.0)
    assert e.value.code == fc.FC_ERR_ARG


def _heavy_pairs_graph():
    """BA(1800, 3) with unit weights and 100 separate pairs of weight 10^4:
    a pair's walk bounces thousands of times, so its 2-cycle re-forms pass
    after pass."""
    ba = inputs.barabasi_albert(1800, 3, 11)
    deg = np.diff(ba.row_ptr)
    src = np.repeat(np.arange(ba.n), deg)
    edges = [(int(a), int(b), 1.0) for a, b in zip(src, ba.col_idx) if a < b]
    edges += [(1800 + 2 * i, 1801 + 2 * i, 1e4) for i in range(100)]
    return inputs.from_weighted_edge_list(2000, edges, "ba1800_heavy_pairs")


@pytest.mark.parametrize("sampler", ["lds", "coop"])
def test_repop_overflow_and_pass_limit(gpu_lib, sampler):
    """The re-pop's two exits besides running out of pairs: a perfect matching
    at alpha = 100, where nearly every pair forms again, so a pass outgrows its
    half of the peel buffer (the pass is dropped and its pairs wait for the next
    round); and pairs of weight 10^4, which keep re-forming past the last
    allowed pass.  Both give the oracle's trees."""
    fc = gpu_lib
    matching = inputs.from_edge_list(2000, [(2 * i, 2 * i + 1) for i in range(1000)], "matching2000")
    _compare(fc, matching, 100.0, 5, 0, 12, per_tree=True, sampler=sampler)
    _compare(fc, _heavy_pairs_graph(), 1.0, 6, 0, 12, per_tree=True, sampler=sampler)


@pytest.mark.parametrize("repop", [0, 2], ids=["repop_off", "repop_on"])
@pytest.mark.parametrize("case", ["er1000", "ba20k", "grid", "rmat", "small"])
def test_lds_repop_bit_exact(gpu_lib, repop, case):
    """The LDS sampler with and without popping re-formed 2-cycles within their
    round (option lds_repop): the same trees as the oracle, unweighted and
    weighted."""
    fc = gpu_lib
    g = {"er1000": lambda: inputs.erdos_renyi(1000, 0.01, 0),
         "ba20k": lambda: inputs.barabasi_albert(20_000, 5, 2),
         "grid": lambda: inputs.grid_removed(60, 70, 0.12, 1),
         "rmat": lambda: inputs.rmat(1 << 12, 8, 5),
         "small": lambda: inputs.from_edge_list(4, [(0, 1), (1, 2), (2, 3), (0, 3)])}[case]()
    fc.set_option("lds_repop", repop)
    try:
        for gg, alpha in ((g, 1.0), (inputs.with_weights(g, 7), 0.5)):
            _compare(fc, gg, alpha, 3, 0, 40, per_tree=True, sampler="lds")
    finally:
        fc.set_option("lds_repop", 3)
