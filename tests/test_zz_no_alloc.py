"""fc_sample_noalloc: the sampling call whose scratch is the library's static
device array.  Its trees must equal fc_sample's (and the oracle's) bit for bit,
on two calls in a row, the second with a smaller graph: the array keeps the
first call's contents, so whatever must start at zero has to be cleared by the
call itself.  A graph whose buffers exceed the array is rejected before any
output is written."""
import sys

import numpy as np
import pytest
import torch

import oracle
import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _both(fc, g, alpha, seed, t0, count, sampler=None):
    dg = fc.to_device(g)
    kw = dict(alpha=alpha, seed=seed, tree_begin=t0, tree_count=count, want_visits=True,
              want_digests=True, want_steps=True, sampler=sampler)
    _say(f"noalloc {g.name or g.n} n={g.n} alpha={alpha} trees=[{t0},{t0 + count}) sampler={sampler}")
    a = fc.sample_noalloc(dg, **kw)
    b = fc.sample(dg, **kw)
    for key in ("root_counts", "visit_counts", "tree_digests", "tree_steps"):
        assert np.array_equal(a[key], b[key]), key
    for key in ("walk_steps", "roots", "digest_sum", "sampler"):
        assert a["stats"][key] == b["stats"][key], key
    return a


def test_noalloc_two_calls_match_fc_sample(gpu_lib):
    fc = gpu_lib
    # first call: a graph of the LDS-counter sampler with several trees in flight
    g1 = inputs.barabasi_albert(20000, 5, 0)
    a1 = _both(fc, g1, 1.0, 3, 5, 96)
    assert a1["stats"]["sampler"] == "wilson_lds"
    assert a1["stats"]["trees_in_flight"] >= 1
    # second call, smaller graph: must not see the first call's leftovers
    g2 = inputs.erdos_renyi(1000, 0.01, 0)
    a2 = _both(fc, g2, 1.0, 0, 0, 64)
    ref = oracle.sample(g2, 1.0, 0, 0, 64)
    assert np.array_equal(a2["root_counts"], ref.R)
    assert np.array_equal(a2["visit_counts"], ref.visits)
    assert np.array_equal(a2["tree_digests"], ref.digests)


def test_noalloc_global_counter_sampler(gpu_lib):
    fc = gpu_lib
    g = inputs.grid_removed(60, 70, 0.12, 0)
    a = _both(fc, g, 2.0, 1, 0, 48, sampler="coop")
    ref = oracle.sample(g, 2.0, 1, 0, 48)
    assert np.array_equal(a["tree_digests"], ref.digests)
    assert np.array_equal(a["root_counts"], ref.R)


def test_noalloc_rejects_oversized_graph(gpu_lib):
    fc = gpu_lib
    # 5M isolated vertices: their 16-byte records alone exceed the 64 MiB array
    n = 5_000_000
    g = inputs.CSRGraph(n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), "empty5m")
    dg = fc.to_device(g)
    R = torch.full((n,), 7, dtype=torch.int32, device="cuda:0")
    _say("noalloc oversized graph")
    with pytest.raises(fc.FCError) as e:
        fc.sample_noalloc(dg, alpha=1.0, tree_count=4, root_counts=R)
    assert "static scratch" in str(e.value)
    assert int((R != 7).sum()) == 0
