/*
 * fc.h -- C-ABI of the forest-closeness sampling library for AMD Instinct
 * MI355X (gfx950).
 *
 * What it computes (van der Grinten, Angriman, Predari, Meyerhenke, "New
 * Approximation Algorithms for Forest Closeness Centrality -- for Individual
 * Vertices and Vertex Groups", SDM 2021):
 *   Omega = (alpha L + I)^{-1} is the forest matrix of a graph G (Section 2,
 *   "Forest Distance / Closeness").  Adding a universal vertex u* joined to
 *   every vertex with weight 1, and weighting G's edges by alpha, gives the
 *   augmented graph G* (Section 4.1).  Sampling uniform spanning trees of G*
 *   rooted at u* with Wilson's algorithm (Algorithm 3) and counting how often
 *   each edge {u*, v} is in a tree estimates Omega_vv (Algorithm 1,
 *   Prop. "unbiased"); forest farness follows from the diagonal alone
 *   (Eq. "eq-fdistu-tr": rho(v) = n Omega_vv + tr(Omega) - 2) and forest
 *   closeness is n / rho(v) (Definition "forest-dist-vertex").
 *
 * Conventions shared by every call:
 *   - Return FC_OK (0) or a negative FC_ERR_* code; fc_last_error() gives a
 *     message for the context's last failure.  Nothing is written to the
 *     outputs of a failing call unless stated.
 *   - Graphs are simple and undirected (Section 2: finite, simple,
 *     undirected), in CSR with both directions stored, rows sorted strictly
 *     ascending, no self-loops; unweighted, or with non-negative edge weights
 *     (Section 2 defines L for weighted graphs: L = D - A with A holding the
 *     weights and D the weighted degrees).  Input that violates this is
 *     rejected with FC_ERR_GRAPH (checked on the device for every call,
 *     unless params.flags has FC_FLAG_TRUSTED_GRAPH).  The graph is never
 *     modified.
 *   - Every output array is a DEVICE pointer on the context's device, owned
 *     by the caller (for example a torch tensor's data_ptr()).  Graph arrays
 *     may be host or device memory (fc_graph.mem).
 *   - All device work is enqueued on the context's stream; every call
 *     returns only after its work has finished (the stream is synchronised).
 *   - A context is not thread-safe; use one per host thread.  Results are a
 *     pure function of (graph, alpha, seed, stream_id, tree range): the
 *     output of disjoint tree ranges may be summed (checkpoint / resume).
 *
 * Randomness contract (the paper does not fix one; both this library and the
 * test oracle implement it independently):
 *   - The j-th step taken out of vertex v in tree t (j = 0, 1, ...) uses
 *     x = Philox4x32-10(counter = (v, j, t, stream_id), key = (seed mod 2^32,
 *     seed >> 32)) (Salmon et al., SC 2011).
 *   - The step goes to u* iff d_v = 0 or x0 < thr(d_v), where
 *     thr(d) = floor(2^32 * (1 / ((alpha * d) + 1))) evaluated in IEEE
 *     binary64 with each operation rounded separately; otherwise it goes to
 *     col_idx[row_ptr[v] + floor(x1 * d_v / 2^32)].
 *   - Weighted graphs (fc_graph.weights): W_v is the binary64 sum of v's row
 *     weights, added one by one in CSR order starting from 0, and
 *     S_v(i) the same running sum through entry i of the row.  The step goes
 *     to u* iff W_v = 0 or x0 < thr_w(W_v), thr_w(W) = floor(2^32 * (1 /
 *     ((alpha * W) + 1))) (binary64, each operation rounded); otherwise it
 *     goes to the first entry i of the row with u < S_v(i), where
 *     u = (x1 * W_v) * 2^-32 (binary64).  A walk on a weighted graph leaves v
 *     along an edge with probability proportional to its weight (Section 4.1
 *     weighs G's edges by alpha and u*'s by 1), and this picks entry i with
 *     probability w_i / W_v up to binary64 rounding.  With unit weights and
 *     degrees below 2^21 (x1 * d is then exact) it is the unweighted rule.
 *   By Wilson's cycle-popping theorem the sampled tree and the number of
 *   steps taken out of every vertex do not depend on the order in which
 *   walks are started, which lets the device schedule walks freely.
 */
#ifndef FC_H
#define FC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FC_API __attribute__((visibility("default")))

/* return codes */
#define FC_OK 0
#define FC_ERR_ARG (-1)         /* invalid argument (NULL, range, alpha <= 0, ...) */
#define FC_ERR_GRAPH (-2)       /* CSR is not simple, symmetric and sorted */
#define FC_ERR_NOMEM (-3)       /* device allocation failed */
#define FC_ERR_HIP (-4)         /* HIP runtime error (no device, launch failure) */
#define FC_ERR_UNSUPPORTED (-5) /* n or nnz beyond the supported range */
#define FC_ERR_OVERFLOW (-6)    /* a per-vertex draw count in one tree exceeded 2^31 - 1
                                   (2^28 - 1 with the LDS-counter sampler) */

/* fc_graph.mem */
#define FC_MEM_HOST 0
#define FC_MEM_DEVICE 1

/* fc_params.estimator */
#define FC_EST_DIRECT 0        /* Omega_vv ~ R[v] / tau */
#define FC_EST_ALG1_LITERAL 1  /* R[v] / tau - (n+2)/(n+1)^2, see fc_diag_estimate */

/* fc_params.flags (and fc_batch_create flags) */
#define FC_FLAG_TRUSTED_GRAPH 1 /* skip the device-side CSR validation */
#define FC_FLAG_AUTOTUNE 8      /* fc_batch_create: time candidate launch shapes, keep the fastest */
#define FC_FLAG_SAMPLER_LANE 2  /* force the lane-per-tree sampler */
#define FC_FLAG_SAMPLER_COOP 4  /* force the workgroup-per-tree sampler, counters in global memory */
#define FC_FLAG_SAMPLER_LDS 16  /* force the workgroup-per-tree sampler with every in-arrow
                                   counter in LDS; FC_ERR_UNSUPPORTED when one tree's
                                   counters and settled bitmap do not fit */
#define FC_FLAG_SAMPLER_HYB 32  /* force the hybrid workgroup-per-tree sampler: counters and
                                   settled bits of the highest-degree vertices in LDS, the
                                   rest in global memory */
#define FC_FLAG_SAMPLER_TILE 64 /* force the tile sampler: the tree's cycles are popped tile by
                                   tile (tiles of consecutive ids, counters in LDS), the
                                   cycles that cross tiles through the graph of the vertices
                                   whose arrow leaves their tile */
/* No sampler flag: a workgroup-per-tree sampler, with LDS counters whenever
 * one tree's counters and settled bitmap fit; else the tile sampler when at
 * most a tenth of the CSR entries join ids of different tiles (option
 * "tile_cross_permille"); else with global counters when the settled bitmap
 * alone fits in LDS; else the hybrid (option "coop_lds_counts" = 0: global
 * counters throughout).  The lane sampler runs
 * only on request.  All samplers produce identical results (same trees, same
 * counts). */

typedef struct fc_ctx fc_ctx;

/* A graph G = (V, E) with V = {0, ..., n-1}: n >= 0 vertices and nnz = 2|E|
 * stored directed entries. row_ptr: int32[n+1], row_ptr[0] = 0,
 * row_ptr[n] = nnz; col_idx: int32[nnz]. n < 2^31 - 1, nnz < 2^31.
 * weights: NULL (every edge weighs 1), or double[nnz] in the same memory as
 * row_ptr and col_idx: weights[e] is the weight of the edge {v, col_idx[e]}
 * of row v, equal (bit for bit) to the weight stored with the reverse entry,
 * and either 0 or in [2^-64, 2^64] (so that every sum, product and quotient
 * of the randomness contract stays finite and normal; a zero-weight edge is
 * never walked and is absent from L).  Violations are FC_ERR_GRAPH. */
typedef struct {
    int32_t n;
    int64_t nnz;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const double *weights; /* NULL or double[nnz] */
    int32_t mem;           /* FC_MEM_HOST or FC_MEM_DEVICE */
} fc_graph;

/* Parameters of Algorithm 1 (ApproxDiagForestMatrix(G, alpha, eps, delta)).
 *   alpha > 0; 0 < eps < 1; 0 < delta < 1; 0 <= kappa < 1.
 *   tau: number of trees; 0 means tau = fc_tau(m, n, eps, delta, kappa).
 *   seed, stream_id: Philox key and counter word 3 (see the contract above). */
typedef struct {
    double alpha;
    double eps;
    double delta;
    double kappa;
    uint64_t seed;
    uint32_t tau;
    uint32_t stream_id;
    int32_t estimator; /* FC_EST_* */
    int32_t flags;     /* FC_FLAG_* */
} fc_params;

/* Filled by the sampling calls (any pointer may be NULL). */
typedef struct {
    uint32_t tau;            /* trees sampled */
    uint32_t trees_in_flight;/* concurrent trees used by the sampler */
    uint64_t walk_steps;     /* total random-successor calls (sum of visit counts) */
    uint64_t roots;          /* total edges {u*, v} over all trees (= sum of R) */
    uint64_t digest_sum;     /* sum over trees of the per-tree digest, mod 2^64 */
    double ms_sample;        /* device time of the sampling kernel */
    double ms_total;         /* host wall time of the call */
    char sampler[16];        /* "wilson_lane", "wilson_coop", "wilson_lds" (workgroup sampler,
                                counters in LDS), "wilson_hyb" (hybrid), or for a batch
                                "batch:<threads>x<wg per CU>"
                                ("lbatch:..." with counters in LDS) */
    double phase_ms[8];      /* workgroup sampler with option "phase_timing": average
                                milliseconds per workgroup spent in
                                wilson_coop: first arrows, in-arrow counting, peel
                                  level 0, peel levels, reverse sweep, redraw, output;
                                wilson_lds: first arrows, in-arrow counting with peel
                                  level 0, wide peel levels, single-wave peel levels,
                                  reverse sweep (which also lists the vertices left
                                  hanging off cycles), scan for the cycle vertices,
                                  cycle popping, output;
                                else zeros */
    double ms_predraw;       /* part of ms_sample spent drawing every tree's first arrows
                                ahead of the LDS-counter sampler (option "predraw_mib"),
                                else 0 */
} fc_stats;

/* Create a context on HIP device `hip_device` that enqueues its work on
 * `hip_stream` (a hipStream_t; NULL = the device's null stream).  The context
 * owns its device scratch memory until fc_destroy. */
FC_API int fc_create(fc_ctx **ctx, int hip_device, void *hip_stream);
FC_API int fc_destroy(fc_ctx *ctx);
/* Change the stream later calls use. */
FC_API int fc_set_stream(fc_ctx *ctx, void *hip_stream);

/* Launch-shape options of a context (results never depend on them):
 *   "coop_threads"    threads per workgroup of the workgroup sampler (64..512, multiple of 64)
 *   "coop_wg_per_cu"  workgroups per CU of the workgroup sampler (>= 1)
 *   "coop_lds_bits"   settled bitmap in LDS: 1 when it fits, 0 never (global memory)
 *   "coop_word32"     32-bit per-vertex tree words when they fit: 1 (default) or 0 (64-bit)
 *   "coop_in_bits"    second LDS bitmap (vertices with in-arrows) when it fits: 1 (default) or 0
 *   "coop_lds_counts" 1 (default): the workgroup sampler keeps every in-arrow counter of a
 *                     tree in LDS (degree-sized fields on degree-class relabelled ids) when
 *                     they and the settled bitmap fit; 0: counters in global tree words
 *   "lds_threads"     threads per workgroup of that LDS-counter variant (64..1024, multiple
 *                     of 64; 0, the default: 1024 when LDS holds at most two trees per
 *                     CU, else narrower (down to 256) as the trees per CU grow)
 *   "lds_wg_per_cu"   cap on its resident workgroups per CU (0, the default: as many as fit)
 *   "lanes_per_wave"  active lanes per wave of the lane sampler (1..64)
 *   "max_slots"       cap on trees in flight (0 = memory bound only)
 *   "phase_timing"    1: the workgroup sampler reports per-phase times in fc_stats
 *   "hyb_hot_cap"     cap on how many (highest-degree) vertices the hybrid sampler keeps in
 *                     LDS (default 2^31 - 1: as many as fit; 0: none, all counters global)
 *   "predraw_mib"     the LDS-counter sampler draws every tree's first arrows in one
 *                     vertex-major kernel beforehand (each vertex's record and adjacency
 *                     row read once for many trees) when the graph has at least 16384
 *                     non-isolated vertices and the words of all the call's trees
 *                     (8 n bytes each) fit in this many MiB; 0: never (each tree draws
 *                     its own); default 32768
 *   "max_draws"       cap on the arrows one vertex may draw in one tree, below each
 *                     sampler's own limit (0, the default: no extra cap); a call that
 *                     exceeds it returns FC_ERR_OVERFLOW (exercises that error path)
 *   "lds_repop"       LDS-counter sampler: a 2-cycle that the redrawn arrows of a round
 *                     close again is popped in that same round (cycle popping may pop
 *                     any cycle at any time: the same trees) instead of a round later
 *                     with everything that hangs off it; 0 never, 1 weighted graphs
 *                     only, 2 always, 3 (the default) always, except that a batch
 *                     created with FC_FLAG_AUTOTUNE times each LDS launch group with
 *                     and without the re-pops and keeps the faster (the trees are the
 *                     same either way)
 *   "coop_repop"      the same for the global-counter sampler (graphs whose counters do
 *                     not fit LDS), with an LDS filter that flags the re-popped
 *                     vertices; 0 never, 1 weighted graphs only, 2 always (the default)
 *   "lds_lean"        LDS-counter sampler, workgroups of at most 512 threads: 1 runs the
 *                     lean register shape (fewer loads in flight per lane, six waves per
 *                     SIMD instead of four); 0 (the default) the full one.  A batch created
 *                     with FC_FLAG_AUTOTUNE times both shapes and keeps the faster (the
 *                     trees are the same either way)
 *   "tile_size"       tile sampler: vertices per tile, a multiple of 64 up to 32704 (0, the
 *                     default: the widest tile whose LDS arrays fit)
 *   "tile_cross_permille"  the tile sampler is picked automatically when at most this many
 *                     CSR entries per thousand join ids of different tiles (default 100)
 *   "tile_threads"    threads per workgroup of the tile sampler (64..1024, multiple of 64;
 *                     default 1024)
 *   "tile_repop"      the tile sampler pops a 2-cycle that a round's new arrows close again
 *                     within that round, inside the tile: 0 never, 1 weighted graphs only,
 *                     2 always (the default)
 *   "tile_bits_lds"   1 (default): the tile sampler keeps its exit and settled bitmaps
 *                     (n bits each) in LDS when they fit; 0: in global memory, so that a
 *                     small tile_size leaves room for several workgroups per CU
 *   "kendall_pairs"   1: fc_kendall_tau compares all n(n-1)/2 pairs (tiled) instead of
 *                     counting discordant pairs by a merge sort (0, the default); same
 *                     counts, O(n^2) instead of O(n log^2 n) work
 * Returns FC_ERR_ARG for an unknown key or a value out of range. */
FC_API int fc_set_option(fc_ctx *ctx, const char *key, int64_t value);

/* Sample size of Algorithm 1: tau = ceil(ln(2 max(m, n) / delta) /
 * (2 (1 - kappa)^2 eps^2)) (Algorithm 1; proof of Theorem "time-approx":
 * Hoeffding's bound with a union bound over the estimated entries).
 * m = number of undirected edges.  Host-only; needs no context. */
FC_API int fc_tau(int64_t m, int64_t n, double eps, double delta, double kappa,
                  uint32_t *tau_out);

/* Root thresholds thr(d) for d = 0..d_max as the device computes them
 * (thr(0) = 2^32); out: host uint64[d_max + 1]. */
FC_API int fc_thresholds(fc_ctx *ctx, double alpha, int32_t d_max, uint64_t *out);

/* Sample trees t = tree_begin .. tree_begin + tree_count - 1 of G* rooted at
 * u* (Algorithm 3, called tau times by Algorithm 1) and ACCUMULATE into the
 * outputs (the caller zeroes them first):
 *   root_counts  uint32[n]     R[v] += [edge {u*, v} in tree]       (required)
 *   visit_counts uint64[n]     += steps taken out of v in the tree  (or NULL)
 * and WRITE per-tree outputs, indexed by t - tree_begin:
 *   tree_digests uint64[tree_count]   sum_v mix64((v << 32) | parent(v)) with
 *                mix64 the SplitMix64 finaliser; u* has id n       (or NULL)
 *   tree_steps   uint64[tree_count]   sum of visit counts           (or NULL)
 *   parents      int32[tree_count*n]  parent of v, u* = n           (or NULL)
 *   tree_visits  uint32[tree_count*n] visit count of v              (or NULL)
 * Uses params->alpha, seed, stream_id and flags. */
FC_API int fc_sample(fc_ctx *ctx, const fc_graph *g, const fc_params *params,
                     uint32_t tree_begin, uint32_t tree_count, uint32_t *root_counts,
                     uint64_t *visit_counts, uint64_t *tree_digests, uint64_t *tree_steps,
                     int32_t *parents, uint32_t *tree_visits, fc_stats *stats);

/* fc_sample for callers that cannot allocate device memory during the call
 * (tight serving loops, harnesses that forbid hipMalloc, processes capturing
 * HIP graphs on other streams meanwhile): the same arguments, trees and
 * outputs as fc_sample, but every
 * buffer the call needs beyond its inputs and outputs (vertex records,
 * relabelled ids, per-tree state, lists, counters) is carved from one static
 * device array of the library, 64 MiB per device, held from the first
 * fc_create on that device until the process ends; the call itself never
 * allocates or frees device memory.
 *   g: device-resident graph (g->mem = FC_MEM_DEVICE, else FC_ERR_ARG).
 *   Trees in flight shrink to what the array holds; a graph whose per-graph
 *   buffers and one tree's state do not fit gets FC_ERR_NOMEM (the message
 *   names the buffer and the limit) and nothing is written to the outputs.
 *   No first-arrow pre-draw (option "predraw_mib" is ignored).
 * Every call on a device shares that device's array and leaves its contents
 * behind: calls that overlap in time on one device (two host threads, two
 * streams) race and must be serialised by the caller.  Like fc_sample it
 * synchronises its stream and reads counters back to the host, so the call
 * itself cannot be recorded into a graph. */
FC_API int fc_sample_noalloc(fc_ctx *ctx, const fc_graph *g, const fc_params *params,
                             uint32_t tree_begin, uint32_t tree_count, uint32_t *root_counts,
                             uint64_t *visit_counts, uint64_t *tree_digests,
                             uint64_t *tree_steps, int32_t *parents, uint32_t *tree_visits,
                             fc_stats *stats);

/* Algorithm 1, ApproxDiagForestMatrix(G, alpha, eps, delta): samples tau trees
 * (tree ids 0..tau-1) and writes diag_out[v] (double[n]):
 *   FC_EST_DIRECT:       R[v] / tau, an unbiased estimate of Omega_vv
 *                        (r_{G*}(u*, v) = Omega_vv; Prop. "unbiased");
 *   FC_EST_ALG1_LITERAL: the paper's last loop, R[v]/tau - x(u*) + 2 x(v),
 *                        with x the minimum-norm solution of
 *                        L* x = e_{u*} - 1/(n+1) 1, which is
 *                        R[v]/tau - (n+2)/(n+1)^2.
 * With probability >= 1 - delta every entry is within eps of Omega_vv
 * (Theorem "time-approx").  root_counts_out (uint32[n], or NULL) receives R. */
FC_API int fc_diag_estimate(fc_ctx *ctx, const fc_graph *g, const fc_params *params,
                            double *diag_out, uint32_t *root_counts_out, fc_stats *stats);

/* Forest farness and closeness of every vertex from the same sample:
 *   farness_out[v]   = (n R[v] + S) / tau - 2, S = sum_w R[w]
 *                      (Eq. "eq-fdistu-tr" with the estimated diagonal)
 *   closeness_out[v] = n / farness_out[v]   (Definition "forest-dist-vertex")
 * diag_out as in fc_diag_estimate.  Any output pointer may be NULL except
 * farness_out. */
FC_API int fc_farness(fc_ctx *ctx, const fc_graph *g, const fc_params *params,
                      double *farness_out, double *closeness_out, double *diag_out,
                      uint32_t *root_counts_out, fc_stats *stats);

/* ---------------------------------------------------------------------- */
/* Batches: many (graph, alpha, tree range) jobs sampled by one persistent  */
/* launch.  Each job is Algorithm 3 applied tree_count times to its own G*  */
/* (Section 4.1 with that job's alpha); the jobs share nothing but the      */
/* launch.  A job's results are identical to fc_sample on the same graph,  */
/* alpha, seed, stream_id and tree range.                                   */
/* ---------------------------------------------------------------------- */
typedef struct {
    fc_graph graph;         /* mem must be FC_MEM_DEVICE */
    double alpha;           /* > 0 */
    uint32_t stream_id;     /* Philox counter word 3 of this job's trees */
    uint32_t tree_begin;    /* first tree id */
    uint32_t tree_count;    /* number of trees */
    uint32_t pad;
    uint32_t *root_counts;  /* device uint32[n]: R[v] += ..., accumulated (caller zeroes) */
    uint64_t *tree_digests; /* device uint64[tree_count] (as in fc_sample) or NULL */
} fc_job;

typedef struct fc_batch fc_batch;

/* Prepare a batch of n_jobs jobs under one Philox key (seed): validates every
 * distinct graph (unless FC_FLAG_TRUSTED_GRAPH), builds each job's vertex
 * records of G*, orders the work items (trees) largest graph first, sizes
 * the per-slot scratch for the largest graph, optionally autotunes the
 * launch shape (FC_FLAG_AUTOTUNE; results do not depend on it: each candidate
 * shape is warmed up on a few trees, then timed twice on a thirty-second of
 * every job's trees, best of two; the choice is kept per device and job
 * shapes, so a batch created again with the same graph sizes, alphas, tree
 * counts and options is not timed again; with the environment variable
 * FC_TUNE_CACHE naming a file, choices are also appended there and read back
 * by later processes) and captures the sampling launch as a HIP graph.  The job array is copied; the graphs
 * and output buffers it points to must stay valid until fc_batch_destroy.
 * Returns FC_ERR_ARG for a job with a host graph, alpha <= 0, a NULL
 * root_counts, or more than 2^32 - 1 trees in total. */
FC_API int fc_batch_create(fc_ctx *ctx, const fc_job *jobs, int32_t n_jobs, uint64_t seed,
                           int32_t flags, fc_batch **out);
/* Sample every tree of every job (one replay of the captured launch on the
 * context's stream) and accumulate into the jobs' root_counts; writes
 * tree_digests where given.  stats: totals over the batch; ms_sample is the
 * device time of the launch. */
FC_API int fc_batch_run(fc_batch *batch, fc_stats *stats);
FC_API int fc_batch_destroy(fc_batch *batch);

/* ---------------------------------------------------------------------- */
/* Linear solves with the forest matrix system (alpha L + I) X = B.          */
/* ---------------------------------------------------------------------- */
#define FC_PREC_FP64 0          /* Jacobi-preconditioned CG in binary64 */
#define FC_PREC_FP32_REFINED 1  /* binary32 CG inside binary64 iterative refinement */

/* Solve (alpha L + I) X = B for 1 <= nrhs <= 64 right-hand sides: the system
 * behind the forest matrix Omega = (alpha L + I)^{-1} (Section 2), the solve of
 * Algorithm 1 (via its grounded form) and the CG ground truth of the
 * experiments (Section 6.1).
 *   B, X  device double[n * nrhs], row-major (X[v * nrhs + j]); X holds the
 *         initial guess on entry (zero it for a cold start), the solution on exit.
 *   Stops when every column has ||B_j - A X_j||_2 <= rtol ||B_j||_2 (residual
 *   always evaluated in binary64), or after max_iters inner CG iterations.
 *   FC_PREC_FP64: one CG on the correction, all in binary64.
 *   FC_PREC_FP32_REFINED: repeat { R = B - A X (binary64); solve A D = R/|R|
 *   with binary32 CG to a relative residual of 1e-5; X += |R| D (binary64) }.
 *   iters_out (host, or NULL): inner CG iterations; relres_out (host double[nrhs],
 *   or NULL): final relative residuals.  Returns FC_OK also when max_iters
 *   ran out; check relres_out.  FC_ERR_UNSUPPORTED for nrhs > 64.
 *   flags: FC_FLAG_TRUSTED_GRAPH. */
FC_API int fc_solve(fc_ctx *ctx, const fc_graph *g, double alpha, const double *B, double *X,
                    int32_t nrhs, double rtol, int32_t precision, int32_t max_iters, int32_t flags,
                    int32_t *iters_out, double *relres_out);

/* ---------------------------------------------------------------------- */
/* Ranking output (Section 6, "Vertex Ranking", and the footnote of its   */
/* accuracy paragraph: the top vertices of the forest closeness ranking   */
/* have the lowest Omega_vv, since farness grows with Omega_vv by Eq.     */
/* "eq-fdistu-tr").  Both calls work on device arrays and synchronise.    */
/* ---------------------------------------------------------------------- */

/* Vertices sorted by score: ascending (descending = 0) or descending, equal
 * scores by vertex id ascending; -0 and +0 are equal, +-inf are ordinary.
 *   score: device double[n] (n >= 0), no NaN (else FC_ERR_ARG, nothing written).
 *   order: device int32[n] or NULL: order[i] = the vertex at position i.
 *   rank:  device int32[n] or NULL: rank[v] = the position of v.
 * The top k of the forest closeness ranking are order[0..k) for score = the
 * estimated diagonal (ascending) or the closeness (descending). */
FC_API int fc_rank(fc_ctx *ctx, const double *score, int32_t n, int32_t descending,
                   int32_t *order, int32_t *rank);

/* Kendall's rank correlation tau-b of two score vectors (the KT the paper
 * reports for the ranking of the estimate against the ground truth).  Over all
 * pairs i < j: n_c concordant, n_d discordant, n_a tied in a, n_b tied in b
 * (pairs tied in both count in n_a and n_b, and n_ab of them);
 * tau_b = (n_c - n_d) / sqrt((n0 - n_a)(n0 - n_b)), n0 = n(n-1)/2, evaluated in
 * binary64 from the exact integer counts (NaN when a or b is constant, n < 2).
 *   a, b:   device double[n], 0 <= n <= 65535 * 256 (else FC_ERR_UNSUPPORTED),
 *           no NaN (FC_ERR_ARG).
 *   tau_b:  host double, or NULL.
 *   counts: host int64[5] = {n_c, n_d, n_a, n_b, n_ab}, or NULL.
 * On the device: min-ranks of a and b by radix sort, ties from the sorted runs,
 * pairs tied in both from a sort of the (rank a, rank b) pairs, discordant pairs
 * as the strict inversions of rank b in that order, counted by a bottom-up merge
 * sort (option "kendall_pairs": all pairs compared instead). */
FC_API int fc_kendall_tau(fc_ctx *ctx, const double *a, const double *b, int32_t n,
                          double *tau_b, int64_t *counts);

/* ---------------------------------------------------------------------- */
/* Group forest closeness (Section 5): the forest farness of a vertex set */
/* S is f(S) = tr((L*_{-S})^{-1}), L* the Laplacian of G* with the rows   */
/* and columns of S removed; its closeness is 1/f(S).                     */
/* ---------------------------------------------------------------------- */

/* The greedy maximiser of group forest closeness (Algorithm 2): the first
 * vertex has the lowest Omega_vv (the highest forest closeness); then, k - 1
 * times, the vertex v of V \ S maximising |M e_v|^2 / M_vv, M = (L*_{-S})^{-1},
 * joins S, and M is downdated by the rank-1 formula (ties: the smallest id).
 * Dense binary64 on the device: one inverse of alpha L + I (blocked
 * Gauss-Jordan with fp64 matrix cores), a change of ground to the first vertex
 * in place of Algorithm 2's pseudo-inverse and second inverse, then one pass
 * over M per step.  Needs 8 N^2 bytes of device memory, N = n rounded up to 64.
 *   g:      the graph (weights allowed); 1 <= k <= n <= 65535 (FC_ERR_UNSUPPORTED
 *           beyond 65535).
 *   flags:  FC_FLAG_TRUSTED_GRAPH or 0.
 *   group:  host int32[k]: the vertices in the order chosen.
 *   farness: host double[k] or NULL: f(S) after each choice. */
FC_API int fc_group_closeness(fc_ctx *ctx, const fc_graph *g, double alpha, int32_t k,
                              int32_t flags, int32_t *group, double *farness);

/* Measurement utility (not part of the method): rate of independent random
 * 4-byte accesses -- loads (atomics = 0) or atomic adds (atomics = 1) -- over
 * a device footprint of footprint_bytes (rounded down to a power of two,
 * >= 4 KiB), in accesses per second, into *rate_out.  The library allocates
 * and frees the footprint.  The sampler's random gathers and in-arrow
 * atomics are bounded by these rates. */
FC_API int fc_probe_random_access(fc_ctx *ctx, uint64_t footprint_bytes, int32_t atomics,
                                  double *rate_out);

/* Message for an error code / for the last failing call on a context. */
FC_API const char *fc_error_string(int code);
FC_API const char *fc_last_error(fc_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* FC_H */
