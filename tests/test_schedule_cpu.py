"""The workgroup samplers' popping schedule, modelled on the CPU: every cycle of
the current arrows popped at once, round after round, and a 2-cycle that the
new arrows close again popped within its round (pass after pass over the
vertices just redrawn).  Wilson's cycle-popping theorem (Section 4's UST
sampling rests on it) says any order of popping cycles ends in the same tree
with the same number of arrows drawn at every vertex; here that is checked
against the oracle's sequential walk (Algorithm 3) tree by tree, with the
arrows of the randomness contract (Philox4x32-10 on (v, k_v, t, stream),
root test on x0, neighbour from x1), unweighted and weighted.  The model is
test code: it shares nothing with the device kernels."""
import numpy as np
import pytest

import oracle
import inputs


class _Arrows:
    """The k-th arrow of vertex v in tree t (u* = n)."""

    def __init__(self, g, alpha, seed, stream):
        self.g, self.n, self.stream = g, g.n, stream
        self.key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], np.uint32)
        self.rp = np.asarray(g.row_ptr, np.int64)
        self.ci = np.asarray(g.col_idx, np.int64)
        self.w = None if g.weights is None else np.asarray(g.weights, np.float64)
        deg = np.diff(self.rp)
        if self.w is None:
            self.thr = [oracle.root_threshold(alpha, int(d)) for d in deg]
        else:
            self.S, self.thr = [], []
            for v in range(self.n):
                s, run = [], 0.0
                for x in self.w[self.rp[v]:self.rp[v + 1]]:
                    run += float(x)  # binary64, in CSR order
                    s.append(run)
                self.S.append(s)
                self.thr.append(oracle.root_threshold_w(alpha, run) if s else 0)

    def __call__(self, v, k, t):
        x = oracle.philox4x32_10([v, k, t, self.stream], self.key)
        d = int(self.rp[v + 1] - self.rp[v])
        if d == 0 or int(x[0]) < self.thr[v]:
            return self.n
        if self.w is None:
            i = (int(x[1]) * d) >> 32
        else:
            S = self.S[v]
            u = (float(int(x[1])) * S[-1]) * 2.0 ** -32
            i = next(j for j, s in enumerate(S) if u < s)
        return int(self.ci[self.rp[v] + i])


def _schedule_tree(g, arrows, t, repop):
    """Parents and per-vertex arrow counts of tree t by the round schedule."""
    n = g.n
    k = np.ones(n, np.int64)
    tgt = np.array([arrows(v, 0, t) for v in range(n)] + [n], np.int64)
    settled = np.zeros(n + 1, bool)
    settled[n] = True
    settled[:n] = tgt[:n] == n
    while True:
        # settle every vertex whose arrows lead to u* or to a settled vertex
        changed = True
        while changed:
            nxt = ~settled[:n] & settled[tgt[:n]]
            changed = bool(nxt.any())
            settled[:n] |= nxt
        U = np.flatnonzero(~settled[:n])
        if U.size == 0:
            return tgt[:n].copy(), k
        # the cycles among the unsettled vertices: what Kahn peeling cannot remove
        indeg = np.zeros(n + 1, np.int64)
        np.add.at(indeg, tgt[U], 1)
        alive = np.zeros(n + 1, bool)
        alive[U] = True
        stack = [v for v in U if indeg[v] == 0]
        while stack:
            v = stack.pop()
            alive[v] = False
            w = tgt[v]
            if alive[w]:
                indeg[w] -= 1
                if indeg[w] == 0:
                    stack.append(w)
        cyc = np.flatnonzero(alive[:n])
        assert cyc.size > 0  # unsettled vertices always lead into a cycle
        for v in cyc:
            tgt[v] = arrows(int(v), int(k[v]), t)
            k[v] += 1
            settled[v] = tgt[v] == n
        if not repop:
            continue
        cur = [int(v) for v in cyc if not settled[v]]
        while cur:
            pairs = set()
            for u in cur:
                w = int(tgt[u])
                if w < n and not settled[w] and tgt[w] == u:
                    pairs.add((min(u, w), max(u, w)))
            cur = []
            for a, b in sorted(pairs):
                for v in (a, b):
                    tgt[v] = arrows(v, int(k[v]), t)
                    k[v] += 1
                    settled[v] = tgt[v] == n
                    if not settled[v]:
                        cur.append(v)


def _graphs():
    heavy = [(0, 1, 1.0), (1, 2, 1.0), (2, 3, 1.0), (3, 0, 1.0), (4, 5, 500.0), (5, 6, 1.0),
             (6, 4, 0.5), (7, 8, 900.0), (3, 7, 1.0)]
    return [
        ("er40", inputs.erdos_renyi(40, 0.1, 3), 1.0),
        ("ba50", inputs.barabasi_albert(50, 2, 4), 2.0),
        ("grid", inputs.grid_removed(6, 7, 0.1, 5), 0.7),
        ("matching", inputs.from_edge_list(30, [(2 * i, 2 * i + 1) for i in range(15)]), 8.0),
        ("ba40w", inputs.with_weights(inputs.barabasi_albert(40, 3, 6), 2), 1.5),
        ("heavy", inputs.from_weighted_edge_list(10, heavy, "heavy"), 1.0),
    ]


@pytest.mark.parametrize("repop", [False, True], ids=["rounds", "rounds_repop"])
@pytest.mark.parametrize("name,g,alpha", _graphs(), ids=[c[0] for c in _graphs()])
def test_round_schedule_equals_wilson(name, g, alpha, repop):
    seed, stream, t0, count = 0x1234_5678_9ABC, 3, 5, 6
    arrows = _Arrows(g, alpha, seed, stream)
    ref = oracle.sample(g, alpha, seed, t0, count, stream=stream, per_tree=True)
    for i in range(count):
        parents, k = _schedule_tree(g, arrows, t0 + i, repop)
        assert np.array_equal(parents, ref.parents[i]), (name, i)
        assert np.array_equal(k, ref.tree_visits[i]), (name, i)
