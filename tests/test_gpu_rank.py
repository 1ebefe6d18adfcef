"""GPU parity of the ranking output (Section 6, "Vertex Ranking") against the
oracle, through the C-ABI: the ranking is integer work (a permutation) and
Kendall's counts are exact integers, so both must be bit-exact; tau-b is one
binary64 expression of the counts, so it must be bit-equal too."""
import math
import sys

import numpy as np
import pytest

import oracle
import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _scores(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "random":
        return rng.standard_normal(n) * 10.0 ** rng.integers(-30, 30, n)
    if kind == "ties":
        return rng.integers(0, max(1, n // 50), n) / 7.0
    if kind == "constant":
        return np.full(n, 0.25)
    if kind == "special":
        base = np.array([0.0, -0.0, np.inf, -np.inf, 5e-324, -5e-324, 1.0, -1.0, 1e308, -1e308])
        return base[rng.integers(0, base.size, n)]
    raise ValueError(kind)


@pytest.mark.parametrize("descending", [False, True], ids=["asc", "desc"])
@pytest.mark.parametrize("kind", ["random", "ties", "constant", "special"])
@pytest.mark.parametrize("n", [0, 1, 2, 255, 256, 4095, 4096, 4097, 10000, 200_000])
def test_rank_bit_exact(gpu_lib, n, kind, descending):
    s = _scores(kind, n, n + 13)
    got = gpu_lib.rank(s, descending=descending)
    order, rank = oracle.ranking(s, descending)
    assert np.array_equal(got["order"], order)
    assert np.array_equal(got["rank"], rank)


def test_rank_large_ragged(gpu_lib):
    """2^21 + 12345 scores with ties (several 4096-key tiles, a ragged last tile)."""
    n = (1 << 21) + 12345
    s = _scores("ties", n, 5)
    got = gpu_lib.rank(s)
    order, _ = oracle.ranking(s)
    assert np.array_equal(got["order"], order)


def test_rank_rejects_nan(gpu_lib):
    with pytest.raises(gpu_lib.FCError) as e:
        gpu_lib.rank([1.0, float("nan"), 2.0])
    assert e.value.code == gpu_lib.FC_ERR_ARG


@pytest.mark.parametrize("n,kind", [(0, "random"), (1, "random"), (2, "ties"), (3, "ties"),
                                    (255, "random"), (256, "ties"), (257, "special"),
                                    (1000, "ties"), (5000, "ties"), (5000, "special"),
                                    (20000, "random"), (20000, "ties")])
def test_kendall_bit_exact(gpu_lib, n, kind):
    a = _scores(kind, n, n)
    b = a + _scores("ties", n, n + 1) if kind != "special" else _scores(kind, n, n + 1)
    got = gpu_lib.kendall_tau(a, b)
    ref = oracle.kendall_counts(a, b)
    assert got["counts"] == ref
    t = oracle.kendall_tau_b(a, b)
    assert (math.isnan(t) and math.isnan(got["tau_b"])) or got["tau_b"] == t


def test_kendall_full_size_closed_forms(gpu_lib):
    """n = 200000 with ties: b = a gives n_d = 0 and every tie count equal to
    sum over tie groups of t(t - 1)/2; b = -a mirrors n_c and n_d."""
    n = 200_000
    a = _scores("ties", n, 3)
    _, cnt = np.unique(a, return_counts=True)
    ties = int((cnt.astype(np.int64) * (cnt - 1) // 2).sum())
    n0 = n * (n - 1) // 2
    same = gpu_lib.kendall_tau(a, a)
    assert same["counts"] == (n0 - ties, 0, ties, ties, ties)
    assert same["tau_b"] == 1.0
    opp = gpu_lib.kendall_tau(a, -a)
    assert opp["counts"] == (0, n0 - ties, ties, ties, ties)
    assert opp["tau_b"] == -1.0


def test_kendall_rejects_nan_and_size(gpu_lib):
    with pytest.raises(gpu_lib.FCError) as e:
        gpu_lib.kendall_tau([1.0, 2.0], [float("nan"), 1.0])
    assert e.value.code == gpu_lib.FC_ERR_ARG
    with pytest.raises(ValueError):
        gpu_lib.kendall_tau([1.0, 2.0], [1.0])


def test_ranking_of_the_estimate(gpu_lib):
    """The paper's use: rank the vertices by the estimated closeness and
    compare with the ground-truth ranking (dense Omega) by Kendall's tau-b."""
    fc = gpu_lib
    g = inputs.erdos_renyi(1000, 0.01, 0)
    out = fc.farness(g, alpha=1.0, seed=0, tau=2000)
    ref = oracle.sample(g, 1.0, 0, 0, 2000)
    d, f, c = oracle.estimate(ref.R, 2000)
    got = fc.rank(out["closeness"], descending=True)
    order, rank = oracle.ranking(c, descending=True)
    assert np.array_equal(got["order"], order) and np.array_equal(got["rank"], rank)
    truth = np.diag(oracle.forest_matrix(g, 1.0))
    kt = fc.kendall_tau(out["diag"], truth)
    assert kt["counts"] == oracle.kendall_counts(d, truth)
    assert kt["tau_b"] == oracle.kendall_tau_b(d, truth)
    _say(f"ER(1000) tau=2000: KT of the estimate vs the dense ground truth {kt['tau_b']:.4f}")
    assert kt["tau_b"] > 0.8


@pytest.mark.parametrize("n,kind", [(3, "ties"), (1000, "ties"), (20000, "random")])
def test_kendall_pair_kernel_bit_exact(gpu_lib, n, kind):
    """The tiled all-pairs kernel (option kendall_pairs) against the oracle."""
    a = _scores(kind, n, n + 3)
    b = a + _scores("ties", n, n + 4)
    gpu_lib.set_option("kendall_pairs", 1)
    try:
        got = gpu_lib.kendall_tau(a, b)
    finally:
        gpu_lib.set_option("kendall_pairs", 0)
    assert got["counts"] == oracle.kendall_counts(a, b)
    t = oracle.kendall_tau_b(a, b)
    assert (math.isnan(t) and math.isnan(got["tau_b"])) or got["tau_b"] == t


@pytest.mark.parametrize("kind", ["random", "ties", "special"])
def test_kendall_merge_equals_pairs_full_size(gpu_lib, kind):
    """n = 200000, beyond the oracle's reach: the merge-sort counts equal the
    all-pairs counts exactly."""
    n = 200_000
    a = _scores(kind, n, 21)
    b = _scores(kind, n, 22) + (a if kind != "special" else 0.0)
    merge = gpu_lib.kendall_tau(a, b)
    gpu_lib.set_option("kendall_pairs", 1)
    try:
        pairs = gpu_lib.kendall_tau(a, b)
    finally:
        gpu_lib.set_option("kendall_pairs", 0)
    assert merge["counts"] == pairs["counts"]
    assert merge["tau_b"] == pairs["tau_b"]


def test_kendall_merge_large_closed_forms(gpu_lib):
    """n = 2^21 + 777 (22 merge levels, ragged runs): b = a and b = -a."""
    n = (1 << 21) + 777
    a = _scores("ties", n, 9)
    _, cnt = np.unique(a, return_counts=True)
    ties = int((cnt.astype(np.int64) * (cnt - 1) // 2).sum())
    n0 = n * (n - 1) // 2
    assert gpu_lib.kendall_tau(a, a)["counts"] == (n0 - ties, 0, ties, ties, ties)
    assert gpu_lib.kendall_tau(a, -a)["counts"] == (0, n0 - ties, ties, ties, ties)
    # a random permutation of 2^15 against the identity, no ties: the oracle's pairs
    perm = np.random.default_rng(4).permutation(1 << 15).astype(np.float64)
    ident = np.arange(1 << 15, dtype=np.float64)
    assert gpu_lib.kendall_tau(ident, perm)["counts"] == oracle.kendall_counts(ident, perm)
