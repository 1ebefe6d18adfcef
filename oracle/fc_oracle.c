/*
 * CPU ORACLE for the forest-closeness sampling path -- TEST INFRASTRUCTURE.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this code.  The product library never calls it, and it shares no
 * code, header, table or constant generator with the GPU path.
 *
 * It is deliberately plain and slow: one thread, one tree at a time, the
 * steps of the paper's UST sampler (Algorithm 3, appendix "Algorithmic
 * Details") in the paper's order, with an explicit walk list P and an
 * explicit chronological loop erasure LE(P).
 *
 * Method summary (paper, Section 4.1 and Algorithm 1):
 *   - G* is G plus a universal vertex u* joined to every vertex by an edge of
 *     weight 1; the edges of G get weight alpha.  u* is the id n here and is
 *     never stored.
 *   - A random walk on G* leaves v to u* with probability 1/(1 + alpha d_v)
 *     and otherwise to a uniform neighbour (unit weights).  With edge weights
 *     w (Section 2 allows non-negative weights), G's edges weigh alpha w and
 *     the walk leaves v to u* with probability 1/(1 + alpha W_v), W_v the
 *     weighted degree, and to neighbour u with probability alpha w_vu / (1 +
 *     alpha W_v) (a random walk on a weighted graph moves along an edge with
 *     probability proportional to its weight).
 *   - tau uniform spanning trees of G* rooted at u* are sampled; R[v] counts
 *     the trees that contain the edge {u*, v}; R[v]/tau estimates Omega_vv,
 *     Omega = (alpha L + I)^{-1}.
 *
 * Randomness contract (one reading where the paper is silent; both sides
 * implement it independently):
 *   - Every vertex v owns a stack of arrows; the j-th arrow (j = 0, 1, ...)
 *     drawn at v in tree t is a pure function of (seed, stream, t, v, j).
 *     k_v counts the arrows drawn at v in the current tree (its visits).
 *   - x = Philox4x32-10(counter = (v, j, t, stream), key = (seed_lo, seed_hi)).
 *   - step to u* iff x0 < thr(d_v), thr(d) = floor(2^32 * fl(1 / fl(fl(alpha d) + 1)))
 *     in IEEE binary64 round-to-nearest with no fused multiply-add, thr(0) = 2^32;
 *     otherwise to col_idx[row_ptr[v] + floor(x1 * d_v / 2^32)].
 *   - With weights: W_v = the binary64 sum of v's row weights in CSR order,
 *     thr as above with W_v for d_v (thr = 2^32 when W_v = 0); otherwise u =
 *     fl(x1 W_v) 2^-32 and the step goes to the first neighbour in CSR order
 *     whose running binary64 weight sum exceeds u.  With unit weights and
 *     degrees below 2^21 this is exactly the unweighted rule (the sums are
 *     exact integers and so is x1 * d).
 *   Wilson's cycle-popping argument (Wilson 1996, the paper's reference for
 *   the sampler) makes the tree and every k_v independent of the order in
 *   which walks are started; the tests check that property on this code.
 *
 * Build: cc -O2 -std=c11 -ffp-contract=off -shared -fPIC fc_oracle.c -o liboracle.so
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#pragma STDC FP_CONTRACT OFF

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 block function (Salmon, Moraes, Dror and Shaw, "Parallel    */
/* random numbers: as easy as 1, 2, 3", SC 2011, Section 3.3).  Each of the  */
/* ten rounds multiplies words 0 and 2 by fixed odd constants, XORs the high */
/* halves of the products with words 1 and 3 and with the round key, and     */
/* permutes; the key advances by the Weyl constants (golden ratio and        */
/* sqrt(3) - 1, scaled to 32 bits) between rounds.                            */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Root threshold of a vertex of degree d (see the contract above). */
uint64_t orc_root_threshold(double alpha, int64_t d) {
    if (d == 0) return (uint64_t)1 << 32;
    double ad = alpha * (double)d;
    double den = ad + 1.0;
    double p = 1.0 / den;
    return (uint64_t)(p * 4294967296.0);
}

/* SplitMix64 output function (Steele, Lea and Flood 2014), used for the
 * order-independent per-tree digest sum_v mix64((v << 32) | parent(v)). */
uint64_t orc_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/*
 * Sample size (Algorithm 1, setting tau; proof of Theorem "time-approx"):
 * tau = ceil( ln(2 max(m, n) / delta) / (2 (1-kappa)^2 eps^2) ).
 * The paper writes log(2m/delta); we read log as the natural logarithm
 * (Hoeffding's bound) and take max(m, n) so the union bound also covers all n
 * estimates when m < n.  Returns 0 on invalid arguments.
 */
uint32_t orc_tau(int64_t m, int64_t n, double eps, double delta, double kappa) {
    if (!(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 1.0) ||
        !(kappa >= 0.0 && kappa < 1.0) || n < 1 || m < 0)
        return 0;
    double events = (double)(m > n ? m : n);
    double e1 = (1.0 - kappa) * eps;
    double t = log(2.0 * events / delta) / (2.0 * e1 * e1);
    double c = ceil(t);
    if (c > 4294967295.0) return 0;
    return (uint32_t)c;
}

/* Root threshold of a vertex of weighted degree W (W = 0: always u*). */
uint64_t orc_root_threshold_w(double alpha, double W) {
    if (W == 0.0) return (uint64_t)1 << 32;
    double aw = alpha * W;
    double den = aw + 1.0;
    double p = 1.0 / den;
    return (uint64_t)(p * 4294967296.0);
}

/* One random step of the walk on G* from v, using arrow j of v in tree t
 * (weights == NULL: unit weights). */
static int32_t orc_successor(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                             const double *weights, double alpha, const uint32_t key[2],
                             uint32_t stream, uint32_t t, int32_t v, uint32_t j) {
    uint32_t ctr[4] = {(uint32_t)v, j, t, stream};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    if (!weights) {
        int64_t d = (int64_t)row_ptr[v + 1] - row_ptr[v];
        if ((uint64_t)x[0] < orc_root_threshold(alpha, d)) return n; /* to u* */
        uint64_t idx = ((uint64_t)x[1] * (uint64_t)d) >> 32;
        return col_idx[row_ptr[v] + (int64_t)idx];
    }
    double W = 0.0;
    for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) W += weights[e];
    if ((uint64_t)x[0] < orc_root_threshold_w(alpha, W)) return n;   /* to u* */
    /* the neighbour whose weight interval [sum before it, sum through it)
     * contains u, a point of [0, W) */
    double u = ((double)x[1] * W) * (1.0 / 4294967296.0);
    double s = 0.0;
    for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
        s += weights[e];
        if (u < s) return col_idx[e];
    }
    return -1; /* unreachable: u < W */
}

/* Stable ascending-degree order of V (Algorithm 3: "reordering of V according
 * to ascending degree"); ties broken by vertex id. */
static void orc_degree_order(int32_t n, const int32_t *row_ptr, int32_t *order) {
    int64_t dmax = 0;
    for (int32_t v = 0; v < n; ++v) {
        int64_t d = (int64_t)row_ptr[v + 1] - row_ptr[v];
        if (d > dmax) dmax = d;
    }
    int64_t *cnt = (int64_t *)calloc((size_t)dmax + 2, sizeof(int64_t));
    for (int32_t v = 0; v < n; ++v) cnt[row_ptr[v + 1] - row_ptr[v] + 1]++;
    for (int64_t d = 1; d <= dmax + 1; ++d) cnt[d] += cnt[d - 1];
    for (int32_t v = 0; v < n; ++v) order[cnt[row_ptr[v + 1] - row_ptr[v]]++] = v;
    free(cnt);
}

typedef struct {
    int32_t *data;
    int64_t len, cap;
} orc_vec;

static void orc_push(orc_vec *a, int32_t x) {
    if (a->len == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 1024;
        a->data = (int32_t *)realloc(a->data, sizeof(int32_t) * (size_t)a->cap);
    }
    a->data[a->len++] = x;
}

/*
 * Sample trees t = t_begin .. t_begin+count-1 of G* rooted at u* and
 * accumulate R (Algorithm 3, called tau times by Algorithm 1).
 *
 *   order        : start order v_1..v_n, or NULL for ascending degree
 *   R            : uint32[n], accumulated: R[v] += [ {u*, v} in tree ]
 *   visits       : uint64[n] or NULL, accumulated: += k_v of each tree
 *   parents      : int32[count * n] or NULL: parent of v in tree i (u* = n)
 *   tree_visits  : uint32[count * n] or NULL: k_v of tree i
 *   digests      : uint64[count] or NULL: sum_v mix64((v << 32) | parent(v))
 *   steps        : uint64[count] or NULL: sum_v k_v (random-successor calls)
 *   roots        : uint32[count] or NULL: number of v with parent u*
 * Returns 0, or -1 on invalid arguments / allocation failure.
 */
int orc_sample_w(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                 const double *weights, double alpha, uint64_t seed, uint32_t stream,
                 uint32_t t_begin, uint32_t count, const int32_t *order, uint32_t *R,
                 uint64_t *visits, int32_t *parents, uint32_t *tree_visits, uint64_t *digests,
                 uint64_t *steps, uint32_t *roots) {
    if (n < 0 || !(alpha > 0.0) || !R) return -1;
    if (n == 0 || count == 0) return 0;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const int32_t ustar = n;
    int32_t *ord = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint8_t *in_tree = (uint8_t *)malloc((size_t)n + 1);
    int32_t *parent = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint32_t *k = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!ord || !in_tree || !parent || !k || !pos) {
        free(ord); free(in_tree); free(parent); free(k); free(pos);
        return -1;
    }
    if (order) memcpy(ord, order, sizeof(int32_t) * (size_t)n);
    else orc_degree_order(n, row_ptr, ord);
    for (int64_t v = 0; v <= n; ++v) pos[v] = -1;
    orc_vec P = {0, 0, 0}, LE = {0, 0, 0};

    for (uint32_t i = 0; i < count; ++i) {
        const uint32_t t = t_begin + i;
        /* R[v] <- 0 is the caller's; T <- {u*} */
        memset(in_tree, 0, (size_t)n + 1);
        in_tree[ustar] = 1;
        for (int32_t v = 0; v < n; ++v) { parent[v] = -1; k[v] = 0; }

        for (int32_t q = 0; q < n; ++q) {
            const int32_t s = ord[q];
            if (in_tree[s]) continue;          /* walk from v_i to T is empty */
            /* P <- random walk on G* from v_i until it first hits T */
            P.len = 0;
            orc_push(&P, s);
            int32_t u = s;
            for (;;) {
                int32_t w = orc_successor(n, row_ptr, col_idx, weights, alpha, key, stream, t, u,
                                          k[u]);
                k[u] += 1;
                orc_push(&P, w);
                if (in_tree[w]) break;
                u = w;
            }
            /* LE(P): chronological loop erasure of P */
            LE.len = 0;
            for (int64_t j = 0; j < P.len; ++j) {
                int32_t x = P.data[j];
                if (pos[x] >= 0) {             /* loop closed at x: erase it */
                    for (int64_t r = pos[x] + 1; r < LE.len; ++r) pos[LE.data[r]] = -1;
                    LE.len = pos[x] + 1;
                } else {
                    pos[x] = LE.len;
                    orc_push(&LE, x);
                }
            }
            for (int64_t r = 0; r < LE.len; ++r) pos[LE.data[r]] = -1;
            /* T <- T u LE(P); LE(P) ends at the first vertex of T it met */
            for (int64_t r = 0; r + 1 < LE.len; ++r) {
                int32_t a = LE.data[r];
                parent[a] = LE.data[r + 1];
                in_tree[a] = 1;
            }
            /* last vertex of LE(P) is u*: count the vertex just before it */
            if (LE.data[LE.len - 1] == ustar) R[LE.data[LE.len - 2]] += 1;
        }

        uint64_t dig = 0, st = 0;
        uint32_t nr = 0;
        for (int32_t v = 0; v < n; ++v) {
            dig += orc_mix64(((uint64_t)(uint32_t)v << 32) | (uint64_t)(uint32_t)parent[v]);
            st += k[v];
            nr += (parent[v] == ustar);
            if (visits) visits[v] += k[v];
        }
        if (parents) memcpy(parents + (size_t)i * n, parent, sizeof(int32_t) * (size_t)n);
        if (tree_visits) memcpy(tree_visits + (size_t)i * n, k, sizeof(uint32_t) * (size_t)n);
        if (digests) digests[i] = dig;
        if (steps) steps[i] = st;
        if (roots) roots[i] = nr;
    }
    free(P.data); free(LE.data);
    free(ord); free(in_tree); free(parent); free(k); free(pos);
    return 0;
}

/* Unit weights (the paper's unweighted graphs). */
int orc_sample(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, double alpha,
               uint64_t seed, uint32_t stream, uint32_t t_begin, uint32_t count,
               const int32_t *order, uint32_t *R, uint64_t *visits, int32_t *parents,
               uint32_t *tree_visits, uint64_t *digests, uint64_t *steps, uint32_t *roots) {
    return orc_sample_w(n, row_ptr, col_idx, NULL, alpha, seed, stream, t_begin, count, order, R,
                        visits, parents, tree_visits, digests, steps, roots);
}

/*
 * Estimators (Algorithm 1, last loop; farness identity of Section 4.2).
 *   diag[v]      = R[v] / tau                               (estimates Omega_vv)
 *   farness[v]   = (n R[v] + S) / tau - 2,  S = sum_w R[w]   (n Omega_vv + tr Omega - 2)
 *   closeness[v] = n / farness[v]                            (Definition of forest closeness)
 * The integer numerators are exact (below 2^53), so each output is one or
 * two correctly rounded binary64 operations.
 * literal != 0 selects the paper's line read with the minimum-norm solution
 * of its linear system, which subtracts (n+2)/(n+1)^2 from every diag entry.
 */
void orc_estimate(int32_t n, const uint32_t *R, uint32_t tau, int literal, double *diag,
                  double *farness, double *closeness) {
    uint64_t S = 0;
    for (int32_t v = 0; v < n; ++v) S += R[v];
    const double shift = (double)((int64_t)n + 2) / ((double)((int64_t)n + 1) * (double)((int64_t)n + 1));
    for (int32_t v = 0; v < n; ++v) {
        double dv = (double)R[v] / (double)tau;
        if (literal) dv = dv - shift;
        if (diag) diag[v] = dv;
        uint64_t num = (uint64_t)n * (uint64_t)R[v] + S;
        double fv = (double)num / (double)tau - 2.0;
        if (farness) farness[v] = fv;
        if (closeness) closeness[v] = (double)n / fv;
    }
}

/* ------------------------------------------------------------------------ */
/* Kendall's rank correlation of two score vectors (Section 6, "Vertex       */
/* Ranking": the ranking of the estimate against the ground truth).  Over    */
/* all pairs i < j: concordant when a and b order the pair the same way,     */
/* discordant when oppositely, and otherwise tied in a, in b or in both.     */
/* Plain O(n^2) loop over the pairs; comparisons only, no differences.       */
/* counts = {concordant, discordant, tied in a (both included), tied in b    */
/* (both included), tied in both}.                                           */
/* ------------------------------------------------------------------------ */
void orc_kendall_counts(int64_t n, const double *a, const double *b, int64_t counts[5]) {
    int64_t nc = 0, nd = 0, ta = 0, tb = 0, tab = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            int sa = (a[i] < a[j]) ? 1 : (a[i] > a[j]) ? -1 : 0;
            int sb = (b[i] < b[j]) ? 1 : (b[i] > b[j]) ? -1 : 0;
            if (sa == 0) ta += 1;
            if (sb == 0) tb += 1;
            if (sa == 0 && sb == 0) tab += 1;
            if (sa * sb > 0) nc += 1;
            if (sa * sb < 0) nd += 1;
        }
    }
    counts[0] = nc;
    counts[1] = nd;
    counts[2] = ta;
    counts[3] = tb;
    counts[4] = tab;
}
