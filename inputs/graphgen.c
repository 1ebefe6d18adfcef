/*
 * Seeded synthetic graph generators.
 *
 * This module produces inputs only.  It holds none of the forest-closeness
 * arithmetic: no spanning-tree sampling, no Philox stream, no estimator.
 * Both the CPU oracle and the GPU path consume what it writes, so that the
 * two sides see identical graphs.
 *
 * Randomness comes from SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), one sequential stream per
 * generator call, seeded by the caller.  Every function writes an undirected
 * edge list (u[i], v[i]); the Python side turns it into a symmetric CSR with
 * sorted rows, self-loops dropped and duplicates removed.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s; } gg_rng;

static uint64_t gg_next(gg_rng *r) {
    uint64_t z = (r->s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Uniform integer in [0, bound), bound >= 1 (multiply-high, bias < bound/2^64). */
static uint64_t gg_below(gg_rng *r, uint64_t bound) {
    return (uint64_t)(((unsigned __int128)gg_next(r) * bound) >> 64);
}

/* Uniform double in [0, 1) with 53 random bits. */
static double gg_unit(gg_rng *r) {
    return (double)(gg_next(r) >> 11) * (1.0 / 9007199254740992.0);
}

static void gg_seed(gg_rng *r, uint64_t seed, uint64_t salt) {
    r->s = seed ^ (salt * 0xD1342543DE82EF95ull);
    (void)gg_next(r);
}

/* Fisher-Yates permutation of [0, n). */
void gg_permutation(int32_t n, uint64_t seed, int32_t *perm) {
    gg_rng r;
    gg_seed(&r, seed, 0x5045524Dull);
    for (int32_t i = 0; i < n; ++i) perm[i] = i;
    for (int32_t i = n - 1; i > 0; --i) {
        int32_t j = (int32_t)gg_below(&r, (uint64_t)i + 1);
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
}

/*
 * Erdos-Renyi G(n, p): pair (i, j), i < j, in lexicographic order, is kept
 * iff the next uniform draw is < p.  Returns the edge count, or -1 if cap is
 * exceeded.
 */
int64_t gg_er_edges(int32_t n, double p, uint64_t seed,
                    int32_t *us, int32_t *vs, int64_t cap) {
    gg_rng r;
    gg_seed(&r, seed, 0x4552ull);
    int64_t m = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = i + 1; j < n; ++j)
            if (gg_unit(&r) < p) {
                if (m >= cap) return -1;
                us[m] = i; vs[m] = j; ++m;
            }
    return m;
}

/*
 * Barabasi-Albert with m edges per new vertex.  Seed graph: the clique on the
 * first m+1 vertices.  Each later vertex picks m distinct earlier vertices,
 * each pick a uniform entry of the list of edge endpoints added so far
 * (probability proportional to degree), repeats rejected.  Vertex ids are
 * then relabelled by a seeded permutation so that ids carry no age or degree
 * information.  Edge count: m(m+1)/2 + m(n-m-1).
 */
int64_t gg_ba_edges(int32_t n, int32_t m, uint64_t seed,
                    int32_t *us, int32_t *vs, int64_t cap) {
    if (n < m + 1 || m < 1) return -1;
    int64_t need = (int64_t)m * (m + 1) / 2 + (int64_t)m * (n - m - 1);
    if (need > cap) return -1;
    gg_rng r;
    gg_seed(&r, seed, 0x4241ull);
    int32_t *ends = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * need));
    int32_t *pick = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    if (!ends || !pick) { free(ends); free(pick); return -1; }
    int64_t e = 0, ne = 0;
    for (int32_t i = 0; i <= m; ++i)
        for (int32_t j = i + 1; j <= m; ++j) {
            us[e] = i; vs[e] = j; ++e;
            ends[ne++] = i; ends[ne++] = j;
        }
    for (int32_t v = m + 1; v < n; ++v) {
        int64_t avail = ne;           /* only endpoints of earlier edges */
        int32_t got = 0;
        while (got < m) {
            int32_t c = ends[gg_below(&r, (uint64_t)avail)];
            int dup = 0;
            for (int32_t q = 0; q < got; ++q) dup |= (pick[q] == c);
            if (!dup) pick[got++] = c;
        }
        for (int32_t q = 0; q < m; ++q) {
            us[e] = v; vs[e] = pick[q]; ++e;
            ends[ne++] = v; ends[ne++] = pick[q];
        }
    }
    free(ends); free(pick);
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!perm) return -1;
    gg_permutation(n, seed ^ 0xB5ull, perm);
    for (int64_t i = 0; i < e; ++i) { us[i] = perm[us[i]]; vs[i] = perm[vs[i]]; }
    free(perm);
    return e;
}

/*
 * rows x cols grid, row-major ids, 4-neighbour edges listed horizontal first
 * (row by row), then vertical.  Exactly floor(remove_frac * E) edges are
 * removed: the first that many slots of a seeded Fisher-Yates shuffle of the
 * edge indices.  Surviving edges keep their original order.
 */
int64_t gg_grid_edges(int32_t rows, int32_t cols, double remove_frac, uint64_t seed,
                      int32_t *us, int32_t *vs, int64_t cap) {
    int64_t eh = (int64_t)rows * (cols - 1), ev = (int64_t)(rows - 1) * cols;
    int64_t E = eh + ev;
    int64_t drop = (int64_t)floor(remove_frac * (double)E);
    if (E - drop > cap || drop < 0 || drop > E) return -1;
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)E);
    uint8_t *gone = (uint8_t *)calloc((size_t)E, 1);
    if (!idx || !gone) { free(idx); free(gone); return -1; }
    for (int64_t i = 0; i < E; ++i) idx[i] = i;
    gg_rng r;
    gg_seed(&r, seed, 0x47524944ull);
    for (int64_t i = 0; i < drop; ++i) {
        int64_t j = i + (int64_t)gg_below(&r, (uint64_t)(E - i));
        int64_t t = idx[i]; idx[i] = idx[j]; idx[j] = t;
        gone[idx[i]] = 1;
    }
    int64_t m = 0;
    for (int64_t e = 0; e < E; ++e) {
        if (gone[e]) continue;
        int32_t a, b;
        if (e < eh) {
            int32_t rr = (int32_t)(e / (cols - 1)), cc = (int32_t)(e % (cols - 1));
            a = rr * cols + cc; b = a + 1;
        } else {
            int64_t f = e - eh;
            int32_t rr = (int32_t)(f / cols), cc = (int32_t)(f % cols);
            a = rr * cols + cc; b = a + cols;
        }
        us[m] = a; vs[m] = b; ++m;
    }
    free(idx); free(gone);
    return m;
}

/*
 * R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004): each of `draws` edges
 * descends `scale = ceil(log2 n)` levels, choosing quadrant a / b / c / d;
 * an edge with an endpoint >= n is redrawn.  Self-loops and duplicates are
 * left in; the CSR builder removes them.  Ids are relabelled by a seeded
 * permutation.
 */
int64_t gg_rmat_edges(int32_t n, int64_t draws, double a, double b, double c,
                      uint64_t seed, int32_t *us, int32_t *vs) {
    if (n < 1) return -1;
    int32_t scale = 0;
    while (((int64_t)1 << scale) < n) ++scale;
    gg_rng r;
    gg_seed(&r, seed, 0x524D4154ull);
    double ab = a + b, abc = a + b + c;
    for (int64_t i = 0; i < draws; ++i) {
        int32_t u, v;
        do {
            u = 0; v = 0;
            for (int32_t l = 0; l < scale; ++l) {
                double x = gg_unit(&r);
                int32_t bu = (x >= ab), bv = (x >= a && x < ab) || (x >= abc);
                u = (u << 1) | bu; v = (v << 1) | bv;
            }
        } while (u >= n || v >= n);
        us[i] = u; vs[i] = v;
    }
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!perm) return -1;
    gg_permutation(n, seed ^ 0x52ull, perm);
    for (int64_t i = 0; i < draws; ++i) { us[i] = perm[us[i]]; vs[i] = perm[vs[i]]; }
    free(perm);
    return draws;
}

/* Uniform doubles in [0,1) (for log-uniform graph sizes of a batch). */
void gg_uniforms(int64_t count, uint64_t seed, double *out) {
    gg_rng r;
    gg_seed(&r, seed, 0x554E49ull);
    for (int64_t i = 0; i < count; ++i) out[i] = gg_unit(&r);
}

/* Standard normal N(0,1) values by the Box-Muller transform. */
void gg_normals(int64_t count, uint64_t seed, double *out) {
    gg_rng r;
    gg_seed(&r, seed, 0x4E4F524Dull);
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t i = 0; i < count; i += 2) {
        double u1 = 1.0 - gg_unit(&r);   /* (0, 1] */
        double u2 = gg_unit(&r);
        double rad = sqrt(-2.0 * log(u1));
        out[i] = rad * cos(two_pi * u2);
        if (i + 1 < count) out[i + 1] = rad * sin(two_pi * u2);
    }
}

/*
 * Simple symmetric CSR from an undirected edge list: both directions of every
 * edge u != v, rows sorted ascending, duplicates dropped.  Pass 1 (row_ptr and
 * col_idx NULL) returns the number of directed entries before deduplication in
 * *raw and fills nothing; pass 2 fills row_ptr (n + 1 entries, int64) and
 * col_idx (room for *raw entries) and returns the final entry count.  Returns
 * -1 on an id out of [0, n) or a failed allocation.
 */
static int gg_cmp_i32(const void *a, const void *b) {
    const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

int64_t gg_csr(int32_t n, int64_t m, const int32_t *us, const int32_t *vs, int64_t *row_ptr,
               int32_t *col_idx, int64_t *raw) {
    int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!deg) return -1;
    for (int64_t i = 0; i < m; ++i) {
        const int32_t u = us[i], v = vs[i];
        if (u < 0 || v < 0 || u >= n || v >= n) { free(deg); return -1; }
        if (u == v) continue;
        ++deg[u];
        ++deg[v];
    }
    int64_t total = 0;
    for (int32_t v = 0; v < n; ++v) total += deg[v];
    *raw = total;
    if (!row_ptr || !col_idx) { free(deg); return total; }
    /* scatter into rows (deg becomes the fill cursor) */
    int64_t *start = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!start) { free(deg); return -1; }
    start[0] = 0;
    for (int32_t v = 0; v < n; ++v) start[v + 1] = start[v] + deg[v];
    for (int32_t v = 0; v < n; ++v) deg[v] = start[v];
    for (int64_t i = 0; i < m; ++i) {
        const int32_t u = us[i], v = vs[i];
        if (u == v) continue;
        col_idx[deg[u]++] = v;
        col_idx[deg[v]++] = u;
    }
    /* sort and deduplicate each row, compacting in place */
    int64_t out = 0;
    row_ptr[0] = 0;
    for (int32_t v = 0; v < n; ++v) {
        const int64_t a = start[v], b = start[v + 1];
        qsort(col_idx + a, (size_t)(b - a), sizeof(int32_t), gg_cmp_i32);
        for (int64_t e = a; e < b; ++e)
            if (e == a || col_idx[e] != col_idx[e - 1]) col_idx[out++] = col_idx[e];
        row_ptr[v + 1] = out;
    }
    free(start);
    free(deg);
    return out;
}
