"""GPU parity of the tile sampler (cycles popped tile by tile in LDS, crossing
cycles through the exit graph) against the CPU oracle, through the C-ABI.

Small tiles force many crossing cycles, several exit-graph passes and tile
re-runs; graphs without local ids (Erdos-Renyi, Barabasi-Albert) send almost
every arrow across tiles and stress the exit graph most.  The bar is
bit-exactness of parents, visit counts, root counts, digests and steps
(Algorithm 3; Wilson's cycle-popping theorem makes the popping order free)."""
import sys

import numpy as np
import pytest

import oracle
import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _compare(fc, g, alpha, seed, t0, count, tile, per_tree=True):
    _say(f"tile parity {g.name or g.n} n={g.n} alpha={alpha} seed={seed} trees=[{t0},{t0 + count}) "
         f"tile={tile}")
    fc.set_option("tile_size", tile)
    try:
        got = fc.sample(g, alpha=alpha, seed=seed, tree_begin=t0, tree_count=count,
                        want_visits=True, want_digests=True, want_steps=True,
                        want_parents=per_tree, want_tree_visits=per_tree, sampler="tile")
    finally:
        fc.set_option("tile_size", 0)
    assert got["stats"]["sampler"] == "wilson_tile"
    ref = oracle.sample(g, alpha, seed, t0, count, per_tree=per_tree)
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
    return got


@pytest.mark.parametrize("alpha", [0.5, 1.0, 2.0])
@pytest.mark.parametrize("tile", [64, 256, 1024, 0])
def test_grid_small_tiles_bit_exact(gpu_lib, alpha, tile):
    """60 x 70 grid with 12% of edges removed (isolated vertices, ragged last
    tile): 48 trees, tiles of 64 ids (a row is 70 ids: almost every vertical
    arrow crosses) up to one tile for the whole graph."""
    g = inputs.grid_removed(60, 70, 0.12, 0)
    _compare(gpu_lib, g, alpha, 1, 3, 48, tile)


@pytest.mark.parametrize("tile", [64, 512])
def test_nonlocal_graphs_bit_exact(gpu_lib, tile):
    """Graphs whose ids carry no locality: nearly every arrow crosses tiles, so
    the exit graph holds most vertices and pops most cycles."""
    fc = gpu_lib
    _compare(fc, inputs.erdos_renyi(1000, 0.01, 0), 1.0, 0, 0, 64, tile)
    _compare(fc, inputs.barabasi_albert(3000, 5, 2), 1.0, 5, 10, 32, tile)
    _compare(fc, inputs.rmat(4096, 8, 7), 10.0, 2, 0, 16, tile)


@pytest.mark.parametrize("threads", [256, 1024])
def test_global_bitmaps_and_narrow_workgroups(gpu_lib, threads):
    """Option tile_bits_lds = 0 keeps the exit and settled bitmaps in global
    memory (several workgroups per CU with small tiles); narrower workgroups.
    Small tiles give residual sets larger than a tile, which start with the
    global rounds and finish in LDS once they fit."""
    fc = gpu_lib
    fc.set_option("tile_bits_lds", 0)
    fc.set_option("tile_threads", threads)
    try:
        _compare(fc, inputs.grid_removed(60, 70, 0.12, 0), 2.0, 1, 3, 48, 128)
        _compare(fc, inputs.erdos_renyi(1000, 0.01, 0), 1.0, 0, 0, 32, 64)
    finally:
        fc.set_option("tile_bits_lds", 1)
        fc.set_option("tile_threads", 1024)
    with pytest.raises(fc.FCError):
        fc.set_option("tile_bits_lds", 2)


def test_weighted_grid_bit_exact(gpu_lib):
    g = inputs.with_weights(inputs.grid_removed(50, 40, 0.12, 3), 5)
    _compare(gpu_lib, g, 1.0, 4, 0, 32, 128)
    _compare(gpu_lib, g, 3.0, 4, 0, 32, 0)


def test_edge_cases(gpu_lib):
    fc = gpu_lib
    # one vertex, an edge, a path longer than a tile, isolated vertices only
    for g in (inputs.from_edge_list(1, []), inputs.from_edge_list(2, [(0, 1)]),
              inputs.from_edge_list(300, [(i, i + 1) for i in range(299)]),
              inputs.from_edge_list(130, [])):
        _compare(fc, g, 1.0, 0, 0, 8, 64)
    # a long path at a tiny alpha: long chains and cycles across many tiles
    g = inputs.from_edge_list(2000, [(i, i + 1) for i in range(1999)])
    _compare(fc, g, 0.05, 3, 0, 4, 64, per_tree=True)


def test_tile_error_paths(gpu_lib):
    fc = gpu_lib
    with pytest.raises(fc.FCError):
        fc.set_option("tile_size", 100)  # not a multiple of 64
    with pytest.raises(fc.FCError):
        fc.set_option("tile_size", 32768)
    # a visit-count limit turns into FC_ERR_OVERFLOW on the tile sampler too
    g = inputs.grid_removed(30, 30, 0.1, 2)
    ref = oracle.sample(g, 2.0, 9, 0, 8, per_tree=True)
    kmax = int(ref.tree_visits.max())
    fc.set_option("max_draws", kmax - 1)
    fc.set_option("tile_size", 128)
    try:
        with pytest.raises(fc.FCError) as e:
            fc.sample(g, alpha=2.0, seed=9, tree_begin=0, tree_count=8, sampler="tile")
        assert e.value.code == fc.FC_ERR_OVERFLOW
        fc.set_option("max_draws", kmax)
        got = fc.sample(g, alpha=2.0, seed=9, tree_begin=0, tree_count=8, want_digests=True,
                        sampler="tile")
        assert np.array_equal(got["tree_digests"], ref.digests)
    finally:
        fc.set_option("max_draws", 0)
        fc.set_option("tile_size", 0)


@pytest.mark.parametrize("repop", [0, 2], ids=["repop_off", "repop_on"])
def test_repop_on_and_off_same_trees(gpu_lib, repop):
    """Popping re-formed 2-cycles inside a tile round (option tile_repop) is
    only another popping order: the oracle's trees either way, on a grid at
    alpha = 2 (many re-formed pairs), a weighted grid and an R-MAT graph."""
    fc = gpu_lib
    fc.set_option("tile_repop", repop)
    try:
        _compare(fc, inputs.grid_removed(80, 90, 0.12, 1), 2.0, 6, 0, 40, 512)
        _compare(fc, inputs.with_weights(inputs.grid_removed(40, 50, 0.1, 2), 3), 5.0, 2, 0, 24, 0)
        _compare(fc, inputs.rmat(1 << 12, 8, 3), 10.0, 1, 5, 16, 1024)
    finally:
        fc.set_option("tile_repop", 2)
