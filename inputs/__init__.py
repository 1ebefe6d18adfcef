"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

Nothing here computes any part of the forest-closeness method: it only
builds graphs (and Gaussian right-hand sides) from a seed.  The random
streams are SplitMix64 (see ``graphgen.c``); the graph families stand in for
the paper's complex networks (Barabasi-Albert, R-MAT, Erdos-Renyi) and road
networks (grid with edges removed), as described in the experiments section
of the paper (its datasets are not available here).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(
                f"{_LIB_PATH} is missing: run __graft_entry__.build() first")
        lib = ctypes.CDLL(_LIB_PATH)
        i32p = ctypes.POINTER(ctypes.c_int32)
        f64p = ctypes.POINTER(ctypes.c_double)
        lib.gg_er_edges.restype = ctypes.c_int64
        lib.gg_er_edges.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64,
                                    i32p, i32p, ctypes.c_int64]
        lib.gg_ba_edges.restype = ctypes.c_int64
        lib.gg_ba_edges.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                    i32p, i32p, ctypes.c_int64]
        lib.gg_grid_edges.restype = ctypes.c_int64
        lib.gg_grid_edges.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                      ctypes.c_uint64, i32p, i32p, ctypes.c_int64]
        lib.gg_rmat_edges.restype = ctypes.c_int64
        lib.gg_rmat_edges.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                      i32p, i32p]
        lib.gg_permutation.restype = None
        lib.gg_permutation.argtypes = [ctypes.c_int32, ctypes.c_uint64, i32p]
        lib.gg_uniforms.restype = None
        lib.gg_uniforms.argtypes = [ctypes.c_int64, ctypes.c_uint64, f64p]
        lib.gg_normals.restype = None
        lib.gg_normals.argtypes = [ctypes.c_int64, ctypes.c_uint64, f64p]
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.gg_csr.restype = ctypes.c_int64
        lib.gg_csr.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, i64p, i32p, i64p]
        _lib = lib
    return _lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _pf64(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class CSRGraph:
    """Simple undirected graph in CSR form: both directions stored, rows sorted
    ascending, no self-loops, no duplicate edges (the input contract of the
    library, section "Definitions and Notation" of the paper: finite, simple,
    undirected)."""

    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col_idx: np.ndarray  # int32[2m]
    name: str = ""
    weights: np.ndarray | None = None  # float64[2m] aligned with col_idx (symmetric), or None

    @property
    def m(self) -> int:
        return int(self.col_idx.shape[0]) // 2

    @property
    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


def csr_from_edges(n: int, us: np.ndarray, vs: np.ndarray, name: str = "") -> CSRGraph:
    """Symmetrise, drop self-loops and duplicates, sort rows (in C: a count, a
    scatter and a sort of every row)."""
    lib = _load()
    us = np.ascontiguousarray(us, dtype=np.int32)
    vs = np.ascontiguousarray(vs, dtype=np.int32)
    m = int(us.shape[0])
    raw = ctypes.c_int64(0)
    if lib.gg_csr(int(n), m, _p32(us), _p32(vs), None, None, ctypes.byref(raw)) < 0:
        raise ValueError("edge endpoint out of range")
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col = np.empty(max(raw.value, 1), dtype=np.int32)
    nnz = lib.gg_csr(int(n), m, _p32(us), _p32(vs),
                     row_ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p32(col),
                     ctypes.byref(raw))
    if nnz < 0:
        raise MemoryError("CSR construction failed")
    if nnz >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    return CSRGraph(n, row_ptr.astype(np.int32), np.ascontiguousarray(col[:nnz]), name)


def csr_from_edges_numpy(n: int, us: np.ndarray, vs: np.ndarray, name: str = "") -> CSRGraph:
    """The same CSR as csr_from_edges, with numpy (kept to check it)."""
    us = np.asarray(us, dtype=np.int64)
    vs = np.asarray(vs, dtype=np.int64)
    keep = us != vs
    us, vs = us[keep], vs[keep]
    src = np.concatenate([us, vs])
    dst = np.concatenate([vs, us])
    key = np.unique(src * n + dst)
    src = (key // n).astype(np.int32)
    dst = (key % n).astype(np.int32)
    counts = np.bincount(src, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    return CSRGraph(n, row_ptr.astype(np.int32), np.ascontiguousarray(dst), name)


def erdos_renyi(n: int, p: float, seed: int = 0) -> CSRGraph:
    lib = _load()
    cap = int(n * (n - 1) // 2 * p * 1.5 + 64 + 10 * math.sqrt(n * n * p + 1))
    cap = min(cap, n * (n - 1) // 2 + 1)
    us = np.empty(cap, np.int32)
    vs = np.empty(cap, np.int32)
    m = lib.gg_er_edges(n, p, seed, _p32(us), _p32(vs), cap)
    if m < 0:
        raise RuntimeError("ER edge buffer overflow")
    return csr_from_edges(n, us[:m], vs[:m], f"er_n{n}_p{p}_s{seed}")


def barabasi_albert(n: int, m: int, seed: int = 0) -> CSRGraph:
    lib = _load()
    cap = m * (m + 1) // 2 + m * (n - m - 1)
    us = np.empty(cap, np.int32)
    vs = np.empty(cap, np.int32)
    e = lib.gg_ba_edges(n, m, seed, _p32(us), _p32(vs), cap)
    if e != cap:
        raise RuntimeError("BA generation failed")
    return csr_from_edges(n, us, vs, f"ba_n{n}_m{m}_s{seed}")


def grid_removed(rows: int, cols: int, remove_frac: float, seed: int = 0) -> CSRGraph:
    lib = _load()
    cap = rows * (cols - 1) + (rows - 1) * cols
    us = np.empty(cap, np.int32)
    vs = np.empty(cap, np.int32)
    e = lib.gg_grid_edges(rows, cols, remove_frac, seed, _p32(us), _p32(vs), cap)
    if e < 0:
        raise RuntimeError("grid generation failed")
    return csr_from_edges(rows * cols, us[:e], vs[:e],
                          f"grid_{rows}x{cols}_rm{remove_frac}_s{seed}")


RMAT_ABC = (0.57, 0.19, 0.19)


def rmat(n: int, edge_factor: int = 8, seed: int = 0, abc=RMAT_ABC) -> CSRGraph:
    lib = _load()
    draws = edge_factor * n
    us = np.empty(draws, np.int32)
    vs = np.empty(draws, np.int32)
    e = lib.gg_rmat_edges(n, draws, abc[0], abc[1], abc[2], seed, _p32(us), _p32(vs))
    if e != draws:
        raise RuntimeError("R-MAT generation failed")
    return csr_from_edges(n, us, vs, f"rmat_n{n}_ef{edge_factor}_s{seed}")


def rmat_batch_sizes(count: int, seed: int = 0, lo_exp: float = 10.0,
                     hi_exp: float = 17.0) -> list:
    """Vertex counts n_g = round(2^(lo + (hi-lo) U_g)), log-uniform."""
    lib = _load()
    u = np.empty(count, np.float64)
    lib.gg_uniforms(count, seed, _pf64(u))
    return [int(round(2.0 ** (lo_exp + (hi_exp - lo_exp) * x))) for x in u]


def rmat_batch(count: int, edge_factor: int = 8, seed: int = 0, lo_exp: float = 10.0,
               hi_exp: float = 17.0) -> list:
    sizes = rmat_batch_sizes(count, seed, lo_exp, hi_exp)
    return [rmat(nn, edge_factor, seed * 1000003 + 17 * g + 1) for g, nn in enumerate(sizes)]


def permutation(n: int, seed: int) -> np.ndarray:
    lib = _load()
    p = np.empty(n, np.int32)
    lib.gg_permutation(n, seed, _p32(p))
    return p


def gaussian(count: int, seed: int = 0) -> np.ndarray:
    lib = _load()
    out = np.empty(count, np.float64)
    lib.gg_normals(count, seed, _pf64(out))
    return out


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 (Steele, Lea and Flood 2014) on a uint64 array (wrapping)."""
    z = x + np.uint64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def with_weights(g: CSRGraph, seed: int = 0, lo: float = 0.1, hi: float = 10.0) -> CSRGraph:
    """The graph with a seeded edge weight on every edge, log-uniform in
    [lo, hi): a function of the unordered pair {u, v} and the seed only, so both
    stored directions carry the same value."""
    with np.errstate(over="ignore"):
        deg = np.diff(g.row_ptr).astype(np.int64)
        v = np.repeat(np.arange(g.n, dtype=np.uint64), deg)
        u = g.col_idx.astype(np.uint64)
        a, b = np.minimum(u, v), np.maximum(u, v)
        key = (a << np.uint64(32)) | b
        h = _splitmix64(key ^ _splitmix64(np.full(key.shape, seed, np.uint64)))
    unif = (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    w = lo * np.power(hi / lo, unif)
    return CSRGraph(g.n, g.row_ptr, g.col_idx, (g.name + "_w") if g.name else "", w)


def from_weighted_edge_list(n: int, edges, name: str = "") -> CSRGraph:
    """Small hand-written weighted graphs (tests): edges (u, v, w)."""
    g = from_edge_list(n, [(a, b) for a, b, _ in edges], name)
    wt = {(min(a, b), max(a, b)): float(w) for a, b, w in edges}
    deg = np.diff(g.row_ptr)
    v = np.repeat(np.arange(n), deg)
    w = np.array([wt[(min(int(x), int(y)), max(int(x), int(y)))] for x, y in zip(v, g.col_idx)],
                 np.float64)
    return CSRGraph(g.n, g.row_ptr, g.col_idx, name, w)


def from_edge_list(n: int, edges, name: str = "") -> CSRGraph:
    """Small hand-written graphs (tests)."""
    if len(edges) == 0:
        return CSRGraph(n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), name)
    e = np.asarray(edges, dtype=np.int64)
    return csr_from_edges(n, e[:, 0], e[:, 1], name)


# Named workloads (sizes as used by the tests and the benchmark).
def workload(name: str) -> CSRGraph:
    if name == "er1000":
        return erdos_renyi(1000, 0.01, 0)
    if name == "ba200k":
        return barabasi_albert(200_000, 5, 0)
    if name == "grid1000":
        return grid_removed(1000, 1000, 0.12, 0)
    if name == "ba2m":
        return barabasi_albert(2_000_000, 8, 0)
    if name == "rmat22":
        return rmat(1 << 22, 8, 0)
    raise KeyError(name)
