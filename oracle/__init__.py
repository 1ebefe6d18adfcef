"""CPU oracle for the forest-closeness sampling path -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The product path (``paper_2101_06192_amd``)
never imports it and shares no code with it.

Two halves:

* ``liboracle.so`` (``fc_oracle.c``): the paper's UST sampler (Algorithm 3)
  under the Philox arrow-stack contract, the sample size tau of Algorithm 1
  and the estimators of Algorithm 1 / the farness identity.  It is the
  bit-exact parity target of the GPU path.
* plain numpy binary64 definitions of what the sampler estimates: the forest
  matrix Omega = (alpha L + I)^{-1} (Section 2, "Forest Distance /
  Closeness"), forest distances and farness by their definitions, the
  augmented graph G* and its Laplacian (Section 4.1), a conjugate-gradient
  ground truth as in the paper's experimental protocol (Section 6.1), and
  brute-force spanning-tree enumeration with exact rational arithmetic.
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "fc_oracle.c")
_lib = None


def build(cc: str = "gcc") -> str:
    """Compile the C oracle (single-threaded, no FMA contraction)."""
    import subprocess
    cmd = [cc, "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
           SRC_PATH, "-o", LIB_PATH, "-lm"]
    subprocess.run(cmd, check=True)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} missing: build the oracle first")
        lib = ctypes.CDLL(LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        f64p = ctypes.POINTER(ctypes.c_double)
        lib.orc_philox4x32_10.restype = None
        lib.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        lib.orc_root_threshold.restype = ctypes.c_uint64
        lib.orc_root_threshold.argtypes = [ctypes.c_double, ctypes.c_int64]
        lib.orc_mix64.restype = ctypes.c_uint64
        lib.orc_mix64.argtypes = [ctypes.c_uint64]
        lib.orc_tau.restype = ctypes.c_uint32
        lib.orc_tau.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double]
        lib.orc_sample.restype = ctypes.c_int
        lib.orc_sample.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_double, ctypes.c_uint64,
                                   ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, i32p,
                                   u32p, u64p, i32p, u32p, u64p, u64p, u32p]
        lib.orc_sample_w.restype = ctypes.c_int
        lib.orc_sample_w.argtypes = [ctypes.c_int32, i32p, i32p, f64p, ctypes.c_double,
                                     ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_uint32, i32p, u32p, u64p, i32p, u32p, u64p, u64p,
                                     u32p]
        lib.orc_root_threshold_w.restype = ctypes.c_uint64
        lib.orc_root_threshold_w.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.orc_kendall_counts.restype = None
        lib.orc_kendall_counts.argtypes = [ctypes.c_int64, f64p, f64p,
                                           np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")]
        lib.orc_estimate.restype = None
        lib.orc_estimate.argtypes = [ctypes.c_int32, u32p, ctypes.c_uint32, ctypes.c_int,
                                     f64p, f64p, f64p]
        _lib = lib
    return _lib


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


# --------------------------------------------------------------------------
# C oracle wrappers
# --------------------------------------------------------------------------
def philox4x32_10(ctr, key) -> np.ndarray:
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib.orc_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                          _ptr(out, ctypes.c_uint32))
    return out


def _weights(g):
    """The graph's edge weights as float64 aligned with col_idx, or None."""
    w = getattr(g, "weights", None)
    return None if w is None else np.ascontiguousarray(w, dtype=np.float64)


def root_threshold_w(alpha: float, W: float) -> int:
    return int(_load().orc_root_threshold_w(float(alpha), float(W)))


def root_threshold(alpha: float, d: int) -> int:
    return int(_load().orc_root_threshold(float(alpha), int(d)))


def mix64(z: int) -> int:
    return int(_load().orc_mix64(int(z) & 0xFFFFFFFFFFFFFFFF))


def tau(m: int, n: int, eps: float, delta: float, kappa: float = 0.0) -> int:
    return int(_load().orc_tau(int(m), int(n), float(eps), float(delta), float(kappa)))


class SampleResult:
    """Outputs of ``sample``; per-tree arrays are present when requested."""

    def __init__(self, R, visits, parents, tree_visits, digests, steps, roots):
        self.R = R
        self.visits = visits
        self.parents = parents
        self.tree_visits = tree_visits
        self.digests = digests
        self.steps = steps
        self.roots = roots


def sample(g, alpha: float, seed: int, t_begin: int, count: int, stream: int = 0,
           order=None, per_tree: bool = False) -> SampleResult:
    """Run the oracle sampler on trees [t_begin, t_begin + count) (with the
    graph's edge weights when it has them)."""
    lib = _load()
    n = int(g.n)
    R = np.zeros(n, np.uint32)
    visits = np.zeros(n, np.uint64)
    digests = np.zeros(count, np.uint64)
    steps = np.zeros(count, np.uint64)
    roots = np.zeros(count, np.uint32)
    parents = np.zeros((count, n), np.int32) if per_tree else None
    tvis = np.zeros((count, n), np.uint32) if per_tree else None
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, np.int32)
    ordr = None if order is None else np.ascontiguousarray(order, dtype=np.int32)
    w = _weights(g)
    if w is not None and w.size == 0:
        w = np.zeros(1, np.float64)
    rc = lib.orc_sample_w(n, _ptr(rp, ctypes.c_int32), _ptr(ci, ctypes.c_int32),
                          _ptr(w, ctypes.c_double), float(alpha), int(seed), int(stream),
                          int(t_begin), int(count), _ptr(ordr, ctypes.c_int32),
                          _ptr(R, ctypes.c_uint32), _ptr(visits, ctypes.c_uint64),
                          _ptr(parents, ctypes.c_int32), _ptr(tvis, ctypes.c_uint32),
                          _ptr(digests, ctypes.c_uint64), _ptr(steps, ctypes.c_uint64),
                          _ptr(roots, ctypes.c_uint32))
    if rc != 0:
        raise ValueError(f"orc_sample failed ({rc})")
    return SampleResult(R, visits, parents, tvis, digests, steps, roots)


def estimate(R: np.ndarray, tau_: int, literal: bool = False):
    """(diag, farness, closeness) from root counts (Algorithm 1 last loop and
    the farness identity of Section 4.2)."""
    lib = _load()
    R = np.ascontiguousarray(R, dtype=np.uint32)
    n = R.shape[0]
    d = np.zeros(n, np.float64)
    f = np.zeros(n, np.float64)
    c = np.zeros(n, np.float64)
    lib.orc_estimate(n, _ptr(R, ctypes.c_uint32), int(tau_), int(bool(literal)),
                     _ptr(d, ctypes.c_double), _ptr(f, ctypes.c_double), _ptr(c, ctypes.c_double))
    return d, f, c


# --------------------------------------------------------------------------
# binary64 definitions (numpy)
# --------------------------------------------------------------------------
def laplacian(g) -> np.ndarray:
    """L = diag(deg) - A (Section 2; weighted degree and adjacency when the
    graph has edge weights)."""
    n = g.n
    L = np.zeros((n, n), np.float64)
    rp, ci = g.row_ptr, g.col_idx
    w = _weights(g)
    for v in range(n):
        for j in range(rp[v], rp[v + 1]):
            wj = 1.0 if w is None else float(w[j])
            L[v, ci[j]] -= wj
            L[v, v] += wj
    return L


def forest_matrix(g, alpha: float) -> np.ndarray:
    """Omega = (alpha L + I)^{-1} by a dense binary64 solve."""
    n = g.n
    A = alpha * laplacian(g) + np.eye(n)
    return np.linalg.solve(A, np.eye(n))


def forest_matrix_cholesky(g, alpha: float) -> np.ndarray:
    """Same matrix through an explicit Cholesky factorisation (a second route)."""
    n = g.n
    A = alpha * laplacian(g) + np.eye(n)
    C = np.linalg.cholesky(A)
    Y = np.linalg.solve(C, np.eye(n))
    return Y.T @ Y


def forest_distance(Om: np.ndarray) -> np.ndarray:
    """rho(u, v) = Omega_uu + Omega_vv - 2 Omega_uv (Eq. forest-dist-pair)."""
    d = np.diag(Om)
    return d[:, None] + d[None, :] - 2.0 * Om


def farness_by_definition(Om: np.ndarray) -> np.ndarray:
    """rho(v) = sum over w != v of rho(v, w) (Definition forest-dist-vertex)."""
    D = forest_distance(Om)
    np.fill_diagonal(D, 0.0)
    return D.sum(axis=1)


def farness_by_identity(Om: np.ndarray) -> np.ndarray:
    """rho(v) = n Omega_vv + tr(Omega) - 2 (Eq. eq-fdistu-tr)."""
    n = Om.shape[0]
    return n * np.diag(Om) + np.trace(Om) - 2.0


def augmented_laplacian(g, alpha: float) -> np.ndarray:
    """Laplacian of G* (Section 4.1): edges of G weighted alpha, u* (last
    index) joined to every vertex with weight 1."""
    n = g.n
    Ls = np.zeros((n + 1, n + 1), np.float64)
    Ls[:n, :n] = alpha * laplacian(g)
    for v in range(n):
        Ls[v, v] += 1.0
        Ls[n, n] += 1.0
        Ls[v, n] -= 1.0
        Ls[n, v] -= 1.0
    return Ls


def effective_resistance(Lpinv: np.ndarray, u: int, v: int) -> float:
    """r(u, v) = L+_uu + L+_vv - 2 L+_uv (Eq. eff-res)."""
    return float(Lpinv[u, u] + Lpinv[v, v] - 2.0 * Lpinv[u, v])


def _operator(g, alpha: float):
    """alpha L + I as a scipy sparse matrix (with the edge weights, if any)."""
    import scipy.sparse as sp
    n = g.n
    w = _weights(g)
    vals = np.ones(g.col_idx.size) if w is None else w
    A = sp.csr_matrix((vals, g.col_idx.astype(np.int64), g.row_ptr.astype(np.int64)), shape=(n, n))
    deg = np.asarray(A.sum(axis=1)).ravel()
    return (sp.diags(1.0 + alpha * deg) - alpha * A).tocsr()


def cg_solve(g, alpha: float, b: np.ndarray, rtol: float = 1e-9, maxiter: int = 100000):
    """Jacobi-preconditioned conjugate gradients in binary64 for
    (alpha L + I) x = b, stopped at ||r||_2 / ||b||_2 <= rtol per column
    (the ground-truth protocol of the experiments, Section 6.1)."""
    b = np.asarray(b, np.float64)
    single = b.ndim == 1
    B = b[:, None] if single else b
    deg = np.diff(g.row_ptr).astype(np.float64)
    minv = 1.0 / (1.0 + alpha * deg)
    A = _operator(g, alpha)
    X = np.zeros_like(B)
    R = B.copy()
    Z = minv[:, None] * R
    P = Z.copy()
    rz = np.einsum("ij,ij->j", R, Z)
    bn = np.linalg.norm(B, axis=0)
    bn[bn == 0] = 1.0
    it = 0
    active = np.linalg.norm(R, axis=0) / bn > rtol
    while active.any() and it < maxiter:
        AP = A @ P
        pap = np.einsum("ij,ij->j", P, AP)
        a = np.where(active, rz / np.where(pap == 0, 1, pap), 0.0)
        X += a * P
        R -= a * AP
        Z = minv[:, None] * R
        rz_new = np.einsum("ij,ij->j", R, Z)
        beta = np.where(active, rz_new / np.where(rz == 0, 1, rz), 0.0)
        P = Z + beta * P
        rz = rz_new
        it += 1
        active = np.linalg.norm(R, axis=0) / bn > rtol
    return (X[:, 0] if single else X), it


def omega_diag_cg(g, alpha: float, vertices, rtol: float = 1e-9) -> np.ndarray:
    """Omega_vv for selected v by solving (alpha L + I) x = e_v with CG."""
    vertices = np.asarray(vertices)
    B = np.zeros((g.n, len(vertices)))
    B[vertices, np.arange(len(vertices))] = 1.0
    X, _ = cg_solve(g, alpha, B, rtol)
    return X[vertices, np.arange(len(vertices))]


# --------------------------------------------------------------------------
# exact / brute-force tools for tiny graphs
# --------------------------------------------------------------------------
def augmented_edges(g):
    """Edge list of G*: (u, v, is_star_edge, w) with w the G-edge weight (1 for
    unweighted graphs and for the star edges); u* has id n."""
    out = []
    wts = _weights(g)
    for v in range(g.n):
        for j in range(g.row_ptr[v], g.row_ptr[v + 1]):
            w = int(g.col_idx[j])
            if v < w:
                out.append((v, w, False, 1.0 if wts is None else float(wts[j])))
    for v in range(g.n):
        out.append((v, g.n, True, 1.0))
    return out


def spanning_trees(g):
    """All spanning trees of G* (brute force over n-edge subsets).  Each tree
    is returned as its parent array rooted at u* (= n)."""
    n = g.n
    E = augmented_edges(g)
    trees = []
    for sub in itertools.combinations(range(len(E)), n):
        parent_uf = list(range(n + 1))

        def find(x):
            while parent_uf[x] != x:
                parent_uf[x] = parent_uf[parent_uf[x]]
                x = parent_uf[x]
            return x
        ok = True
        for e in sub:
            a, b = E[e][0], E[e][1]
            ra, rb = find(a), find(b)
            if ra == rb:
                ok = False
                break
            parent_uf[ra] = rb
        if not ok:
            continue
        adj = {x: [] for x in range(n + 1)}
        for e in sub:
            a, b = E[e][0], E[e][1]
            adj[a].append(b)
            adj[b].append(a)
        par = [-1] * n
        seen = {n}
        stack = [n]
        while stack:
            x = stack.pop()
            for y in adj[x]:
                if y not in seen:
                    seen.add(y)
                    par[y] = x
                    stack.append(y)
        wprod = Fraction(1)
        for e in sub:
            if not E[e][2]:
                wprod *= Fraction(E[e][3])
        trees.append((tuple(par), sum(1 for e in sub if not E[e][2]), wprod))
    return trees


def exact_omega_diag(g, alpha: Fraction):
    """Omega_vv as exact rationals by Gauss-Jordan elimination over Q."""
    n = g.n
    alpha = Fraction(alpha)
    A = [[Fraction(0)] * n for _ in range(n)]
    wts = _weights(g)
    for v in range(n):
        for j in range(g.row_ptr[v], g.row_ptr[v + 1]):
            w = Fraction(1) if wts is None else Fraction(float(wts[j]))
            A[v][int(g.col_idx[j])] -= alpha * w
            A[v][v] += alpha * w
        A[v][v] += 1
    M = [row[:] + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(A)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [x / piv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [M[v][n + v] for v in range(n)]


# --------------------------------------------------------------------------
# Ranking output (Section 6, "Vertex Ranking"; footnote on the accuracy
# paragraph: the top vertices of the forest closeness ranking are those with
# the lowest Omega_vv).
# --------------------------------------------------------------------------
def ranking(score, descending: bool = False):
    """Vertices sorted by score (ascending, or descending), ties by vertex id
    ascending; returns (order, rank) with order[rank[v]] = v.  -0 and +0 tie;
    NaN is not a score."""
    s = np.asarray(score, dtype=np.float64)
    if np.isnan(s).any():
        raise ValueError("NaN score")
    key = -s if descending else s
    order = np.lexsort((np.arange(s.size), key)).astype(np.int32)
    rank = np.empty_like(order)
    rank[order] = np.arange(s.size, dtype=np.int32)
    return order, rank


def kendall_counts(a, b):
    """Pair counts over i < j: (concordant, discordant, tied in a, tied in b,
    tied in both); the two 'tied in' counts include the pairs tied in both."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    assert a.shape == b.shape
    out = np.zeros(5, np.int64)
    L = _load()
    L.orc_kendall_counts(a.size, _ptr(a, ctypes.c_double), _ptr(b, ctypes.c_double), out)
    return tuple(int(x) for x in out)


def kendall_tau_b(a, b) -> float:
    """Kendall's tau-b: (n_c - n_d) / sqrt((n_0 - n_a)(n_0 - n_b)) with n_0 the
    number of pairs and n_a, n_b the pairs tied in a and in b; NaN when either
    vector is constant.  Evaluated in binary64 from the exact integer counts:
    the product of the two differences, its square root, one division."""
    nc, nd, ta, tb, _ = kendall_counts(a, b)
    n = len(a)
    n0 = n * (n - 1) // 2
    d1, d2 = n0 - ta, n0 - tb
    if d1 == 0 or d2 == 0:
        return float("nan")
    return float(nc - nd) / math.sqrt(float(d1) * float(d2))


# --------------------------------------------------------------------------
# Group forest closeness (Section 5): f(S) = tr((L*_{-S})^{-1}), L* the
# Laplacian of G* with the rows and columns of S removed; the greedy
# maximiser of the group forest closeness 1/f(S) (Algorithm 2).
# --------------------------------------------------------------------------
def group_farness(g, alpha: float, S) -> float:
    """tr((L*_{-S})^{-1}) by a dense inverse (Section 5's definition)."""
    Ls = augmented_laplacian(g, alpha)
    keep = np.setdiff1d(np.arange(g.n + 1), np.asarray(list(S), dtype=np.int64))
    return float(np.trace(np.linalg.inv(Ls[np.ix_(keep, keep)])))


def greedy_group(g, alpha: float, k: int):
    """Algorithm 2, step by step: P = pinv(L*); the first vertex minimises
    n P[v, v] + tr(P); M = inverse of L* without that vertex; then, while
    |S| < k, the vertex v of V \\ S maximising |M e_v|^2 / (e_v^T M e_v) joins S
    and M <- (M - M e_v e_v^T M / (e_v^T M e_v)) without row and column v.
    Ties go to the smallest vertex id.  Returns (S in order of choice,
    [f(S) after each choice])."""
    n = g.n
    Ls = augmented_laplacian(g, alpha)
    P = np.linalg.pinv(Ls)
    score = n * np.diag(P)[:n] + np.trace(P)
    v = int(np.flatnonzero(score == score.min())[0])
    idx = [x for x in range(n + 1) if x != v]          # row/column i of M is vertex idx[i]
    M = np.linalg.inv(Ls[np.ix_(idx, idx)])
    S = [v]
    f = [float(np.trace(M))]
    while len(S) < k:
        cand = [i for i, x in enumerate(idx) if x < n]   # V \ S (u* is not a candidate)
        gain = np.array([(M[:, i] @ M[:, i]) / M[i, i] for i in cand])
        best = cand[int(np.flatnonzero(gain == gain.max())[0])]
        col = M[:, best].copy()
        M = M - np.outer(col, col) / col[best]
        keep = [i for i in range(len(idx)) if i != best]
        M = M[np.ix_(keep, keep)]
        S.append(idx[best])
        idx = [idx[i] for i in keep]
        f.append(float(np.trace(M)))
    return S, f
