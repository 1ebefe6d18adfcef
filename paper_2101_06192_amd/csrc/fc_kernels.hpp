// Host-side launch wrappers of the device kernels (one translation unit per
// kernel family).  Every wrapper enqueues on `stream` and returns the launch
// status; none synchronises.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fc_device.hpp"

namespace fc {

// CSR checks (input contract: simple, undirected, sorted rows).  Pass 1
// checks row_ptr (monotone, bounds); pass 2, run only if pass 1 found
// nothing, checks columns, self-loops, ordering and symmetry.
hipError_t launch_validate_rows(const int32_t *row_ptr, int32_t n, int64_t nnz,
                                unsigned int *err, hipStream_t stream);
// With weights (not null) it also checks every weight's range and that it
// equals the weight of the reverse entry.
hipError_t launch_validate_cols(const int32_t *row_ptr, const int32_t *col_idx,
                                const double *weights, int32_t n, int64_t nnz, unsigned int *err,
                                hipStream_t stream);

// Running weight sums of every row: S[e] = binary64 sum of weights[row_ptr[v] .. e],
// added one by one in CSR order from 0 (one thread per row).
hipError_t launch_row_wsum(const int32_t *row_ptr, const double *weights, int32_t n, double *S,
                           hipStream_t stream);
// Step thresholds of a weighted graph from its running sums S: T[e] = the
// smallest x in [0, 2^32] with (x * W_v) * 2^-32 >= S[e] (W_v the last running
// sum of e's row), clamped to [1, 2^32 - 1] (one thread per kColChunk entries).
// T has room for nnz + kWeightedScan entries (the padding is never counted).
hipError_t launch_step_thresholds(const int32_t *row_ptr, const double *S, int32_t n,
                                  int64_t nnz, uint32_t *T, hipStream_t stream);
// Weighted degrees: W[v] = the last running sum of row v (0 for an empty row).
hipError_t launch_row_wdeg(const int32_t *row_ptr, const double *weights, int32_t n, double *W,
                           hipStream_t stream);

// Per-vertex records of G* for one alpha; atomically maxes the degree into *dmax
// and, when iso is not null, writes the bitmap of isolated vertices
// (ceil(n / 32) words).  With running sums S (not null) the root threshold is
// that of the weighted degree W_v = S[row_ptr[v + 1] - 1] (0 for an empty row),
// and the W_v are added into *wtotal (when not null; any order).
hipError_t launch_build_vrec(const int32_t *row_ptr, const double *S, int32_t n, double alpha,
                             VRec *vrec, unsigned int *dmax, uint32_t *iso, double *wtotal,
                             hipStream_t stream);

// thr(d), d = 0..d_max, as the device computes it (uint64, 2^32 for "always").
hipError_t launch_thresholds(double alpha, int32_t d_max, unsigned long long *out,
                             hipStream_t stream);

// Lane-per-tree Wilson sampler.
struct LaneArgs {
    const VRec *vrec;
    const int32_t *col_idx;
    const double *wsum;       // running weight sums per CSR entry (weighted graph), or null
    const uint32_t *wthr;     // step thresholds per CSR entry (with wsum)
    uint64_t *state;          // slots * n words
    uint32_t n;
    uint32_t slots;
    uint32_t lanes_per_wave;  // active lanes in each 64-lane wave
    uint32_t tree_begin;
    uint32_t tree_count;
    uint32_t stream_id;
    uint32_t key0, key1;
    unsigned long long step_cap;  // per-tree bound on steps; exceeding it is an error
    uint32_t k_limit;         // largest per-vertex draw count in one tree; beyond it is an error
    unsigned int *queue;      // next tree index (relative to tree_begin)
    uint32_t *root_counts;
    unsigned long long *visit_counts;
    unsigned long long *tree_digests;
    unsigned long long *tree_steps;
    int32_t *parents;
    uint32_t *tree_visits;
    Totals *totals;
};
hipError_t launch_wilson_lane(const LaneArgs &a, hipStream_t stream);

// Workgroup-per-tree sampler (round-synchronous cycle popping).  A job is
// one (graph, alpha, stream) with a range of trees and its own outputs.
// The LDS-counter variant reads the degree-class relabelled graph instead:
// vrec and adj on internal ids (vrec.always_root = original id | flag << 31),
// orig maps internal ids back, and [0, n0), [n0, n1), [n1, n2), [n2, n3) are
// the internal ids of the 4-, 8-, 16- and 32-bit counter classes, [n3, n) the
// isolated vertices.
struct CoopJob {
    const VRec *vrec;
    const int32_t *col_idx;
    const double *wsum;             // running weight sums per CSR entry (weighted graph), or null
    const uint32_t *wthr;           // step thresholds per CSR entry (with wsum)
    const unsigned long long *adj;  // LDS variant: internal | original << 18 per CSR entry
    const uint32_t *orig;           // LDS variant: original id of each internal id
    uint32_t n;
    uint32_t n0, n1, n2, n3;        // LDS variant: class boundaries
    uint32_t tree_count;            // trees of the job (isolated vertices' totals)
    uint32_t hot;                   // hybrid variant: ids [0, hot) keep their counter in LDS
    const uint32_t *iso;            // global-counter variant: bitmap of isolated vertices, or null
    uint32_t tshift;          // bits of the target field in a tree word
    uint32_t stream_id;
    uint32_t tree_begin;
    uint32_t first_item;      // work item of the job's first tree
    uint32_t pad;
    unsigned long long step_cap;  // per-tree bound on draws; exceeding it is an error
    uint32_t *root_counts;
    unsigned long long *visit_counts;
    unsigned long long *tree_digests;
    unsigned long long *tree_steps;
    int32_t *parents;
    uint32_t *tree_visits;
};

struct CoopArgs {
    void *word;               // slots * n_max words (u32 or u64): target | in-arrow count << tshift
    uint64_t *kk;             // slots * n_max: (epoch << 32) | arrows drawn, for redrawn vertices
    uint64_t *lists;          // slots * 3 n_max: (vertex, target) pairs: two unsettled lists, peel order
    uint32_t *levels;         // slots * (n_max + 2): peel level boundaries
    uint32_t *bits;           // slots * ceil(n_max/32): settled bitmap when it is not kept in LDS
    uint32_t *origt;          // hybrid variant: slots * n_max original target ids
    uint64_t *pre;            // LDS variant, single job: item_count * n_max tree words whose
                              // first arrows are drawn already (launch_lds_predraw), used in
                              // place of the slot's word array; or null
    uint32_t n_max;           // largest n of any job (per-slot stride)
    uint32_t slots;           // workgroups (trees in flight)
    uint32_t item_count;      // trees over all jobs
    uint32_t key0, key1;
    uint32_t max_rounds;      // bound on popping rounds per tree; exceeding it is an error
    uint32_t k_limit;         // largest per-vertex draw count in one tree; beyond it is an error
    unsigned int *queue;
    Totals *totals;
    unsigned long long *phase_ticks;  // 7 wall-clock tick sums per phase, or null
    CoopJob single;           // the job of a single-graph launch (jobs == null)
    const CoopJob *jobs;      // batch: device job table
    const uint32_t *item_job; // batch: job index of each work item
};
// lds_bits: settled bitmap in LDS; in_bits (needs lds_bits): second LDS bitmap of
// vertices with in-arrows.
// weighted: some job carries running weight sums (the weighted instantiation
// checks each job's pointer).
// repop_words: 0, or a power of two: re-formed 2-cycles are popped within the
// round that re-forms them, with an LDS filter of that many 32-bit words.
hipError_t launch_wilson_coop(const CoopArgs &a, uint32_t threads, bool lds_bits, bool in_bits,
                              bool word32, bool weighted, uint32_t repop_words, hipStream_t stream);
// Allow up to `bytes` of dynamic LDS per workgroup for every variant (set once
// per device to the device limit; launches pass what they need).
hipError_t coop_set_lds_limit(size_t bytes);
// Workgroups of the chosen variant that fit on one CU at once (0 if unknown).
int coop_max_active(uint32_t threads, bool lds_bits, bool in_bits, bool word32, uint32_t n_max,
                    bool weighted, uint32_t repop_words);
size_t coop_lds_bytes(uint32_t n);  // dynamic LDS of the settled bitmap

// LDS-counter variant (n < 2^kRelabelIdBits): the per-tree arrays are word
// (u64: internal target | original target << 18 | draw count << 36), lists
// and levels as above (no kk); the settled bitmap and all in-arrow counters
// live in LDS.
// weighted: some job carries running weight sums (the weighted instantiation
// checks each job's pointer); repop: re-formed 2-cycles are popped within the
// round that re-forms them; lean (workgroups of at most 512 threads, ignored
// above): the shape with fewer items in flight per lane and fewer registers,
// six waves per SIMD instead of four.
hipError_t launch_wilson_lds(const CoopArgs &a, uint32_t threads, uint32_t lds_words,
                             bool weighted, bool repop, bool lean, hipStream_t stream);
hipError_t lds_set_limit(size_t bytes);  // as coop_set_lds_limit, for the LDS-counter kernel
// First arrow of every non-isolated vertex in every tree of a single-job LDS
// launch (a.single, items [0, a.item_count)): a.pre[item * a.n_max + v] = the
// tree word the LDS kernel's first round would write.  Vertex-major, so the
// relabelled records and adjacency are read once per vertex tile for many trees.
hipError_t launch_lds_predraw(const CoopArgs &a, hipStream_t stream);
int lds_max_active(uint32_t threads, uint32_t lds_words, bool weighted, bool repop, bool lean);

// Hybrid variant (ids widest class first: 32-bit fields end at e3, 16-bit at
// e2, 8-bit at e1, then 4-bit): LDS fields and settled bits of ids [0, hot).
hipError_t launch_wilson_hyb(const CoopArgs &a, uint32_t threads, uint32_t lds_words,
                             hipStream_t stream);
hipError_t hyb_set_limit(size_t bytes);
int hyb_max_active(uint32_t threads, uint32_t lds_words, bool weighted);
struct HotLayout {
    uint32_t o2, o1, o0, ob, words;
};
__host__ __device__ inline HotLayout hot_layout(uint32_t hot, uint32_t e3, uint32_t e2, uint32_t e1) {
    const uint32_t h3 = hot < e3 ? hot : e3, h2 = hot < e2 ? hot : e2, h1 = hot < e1 ? hot : e1;
    HotLayout L;
    L.o2 = h3;
    L.o1 = L.o2 + ((h2 - h3 + 1u) >> 1);
    L.o0 = L.o1 + ((h1 - h2 + 3u) >> 2);
    L.ob = L.o0 + ((hot - h1 + 7u) >> 3);
    L.words = L.ob + ((hot + 31u) >> 5);
    return L;
}

// LDS word offsets of one tree's counter classes and settled bitmap.
struct CountLayout {
    uint32_t o1, o2, o3, ob, words;
};
__host__ __device__ inline CountLayout count_layout(uint32_t n, uint32_t n0, uint32_t n1,
                                                    uint32_t n2) {
    CountLayout L;
    L.o1 = (n0 + 7u) >> 3;
    L.o2 = L.o1 + ((n1 - n0 + 3u) >> 2);
    L.o3 = L.o2 + ((n2 - n1 + 1u) >> 1);
    L.ob = L.o3 + (n - n2);
    L.words = L.ob + ((n + 31u) >> 5);
    return L;
}

// Id width of the relabelled adjacency entries (internal | original << bits)
// and of the LDS-counter sampler's packed words: graphs need n < 2^bits.
constexpr uint32_t kRelabelIdBits = 18;

// Degree-class relabelling (blocks of 1024 vertices): per-block class counts
// into blk (kRelabelClasses per block), first internal id per block and class
// into base, and bounds[0..3] = n0, n1, n2, n3.
constexpr uint32_t kRelabelClasses = 5;
uint32_t relabel_blocks(uint32_t n);
// widest_first orders the classes 32-, 16-, 8-, 4-bit (hybrid sampler) instead
// of 4-, 8-, 16-, 32-bit; isolated vertices come last either way.
hipError_t launch_class_bounds(const int32_t *row_ptr, uint32_t n, bool widest_first, uint32_t *blk,
                               uint32_t *base, uint32_t *bounds, hipStream_t stream);
// inv/orig permutations and relabelled adjacency of one graph (base from
// launch_class_bounds).
hipError_t launch_relabel_graph(const int32_t *row_ptr, const int32_t *col_idx, uint32_t n,
                                int64_t nnz, const uint32_t *base, uint32_t orig_shift,
                                uint32_t *inv, uint32_t *orig, unsigned long long *adj,
                                hipStream_t stream);
// Relabelled records of one G* (from the original-id records vrec).
hipError_t launch_relabel_vrec(const VRec *vrec, const uint32_t *inv, uint32_t n, VRec *vrec_r,
                               hipStream_t stream);

// Tile sampler (graphs whose ids are local): one workgroup per tree pops the
// cycles inside each tile of B consecutive ids with LDS counters, finds the
// cycles that cross tiles on the functional graph of the exit vertices, and
// finishes the few vertices whose exit does not reach u* with global counters.
constexpr uint32_t kTileMax = 32704;  // largest tile: local ids and codes fit 15 bits
struct TileArgs {
    const VRec *vrec;          // records of G* (original ids)
    const int32_t *col_idx;
    const double *wsum;        // running weight sums per CSR entry (weighted graph), or null
    const uint32_t *wthr;      // step thresholds per CSR entry (with wsum)
    uint32_t n;
    uint32_t B;                // tile size (vertices), 1..kTileMax
    uint32_t Bp;               // B rounded up to a multiple of 64
    uint32_t ntiles;           // ceil(n / B)
    uint32_t tree_begin, tree_count, stream_id, key0, key1;
    uint32_t slots;            // workgroups (trees in flight)
    uint32_t k_limit;          // largest per-vertex draw count in one tree
    uint32_t max_rounds;       // bound on popping rounds per tile and in the residual
    unsigned long long step_cap;  // per-tree bound on draws
    uint32_t *pre;             // tree_count * n first-arrow targets drawn ahead, or null
    uint32_t *tw;              // slots * n targets (when pre is null)
    uint64_t *kk;              // slots * n (epoch << 32) | draws; zeroed per launch
    uint16_t *ex;              // slots * n tile-local exit, or 0x7FFF (reaches u* in the tile)
    uint32_t *exl;             // slots * n per-tile exit lists (tile * B offsets)
    uint32_t *ecnt;            // slots * ntiles exits per tile
    uint32_t *pc;              // slots * n in-counts; zeroed per launch
    uint32_t *sc;              // slots * n exit-graph successors
    uint32_t *bl;              // slots * 3 n lists
    uint32_t *lv;              // slots * (n + 2) peel level bounds
    uint32_t *bits;            // slots * ceil(n / 32) settled bitmap (residual rounds)
    uint32_t *xb;              // slots * ceil(n / 32) exits that reach u*, or null: in LDS
    uint32_t bits_lds;         // 1: the residual rounds use a copy of bits in LDS
    uint32_t repop;            // 1: pop re-formed 2-cycles within the tile round that re-forms them
    unsigned int *queue;
    Totals *totals;
    unsigned long long *phase_ticks;  // 8 tick sums: tile loads, counts, peels, pops, exits,
                                      // exit graph, residual, output
    uint32_t *root_counts;
    unsigned long long *visit_counts;
    unsigned long long *tree_digests;
    unsigned long long *tree_steps;
    int32_t *parents;
    uint32_t *tree_visits;
};
// lds: dynamic LDS bytes, at least tile_lds_bytes(B) and, with xb null or
// bits_lds set, a bitmap of n bits (4 ceil(n / 32)).
hipError_t launch_wilson_tile(const TileArgs &a, uint32_t threads, size_t lds, hipStream_t stream);
// First arrow of every vertex in every tree of the call: a.pre[item * n + v].
hipError_t launch_tile_predraw(const TileArgs &a, hipStream_t stream);
hipError_t tile_set_limit(size_t bytes);
int tile_max_active(uint32_t threads, size_t lds, bool weighted);
size_t tile_lds_bytes(uint32_t B);  // LDS of one tile's arrays
// *out += CSR entries whose ends lie in different tiles of B ids.
hipError_t launch_count_cross(const int32_t *row_ptr, const int32_t *col_idx, uint32_t n,
                              uint32_t B, unsigned long long *out, hipStream_t stream);

// p[0..count) = value (a kernel, so that it can sit in a captured HIP graph).
hipError_t launch_fill_u64(unsigned long long *p, size_t count, unsigned long long value,
                           hipStream_t stream);

// Memory probe: blocks x 256 threads, each issuing iters x 8 random 4-byte
// loads (or atomic adds) into data[0 .. words_pow2), words_pow2 a power of two.
hipError_t launch_random_access(uint32_t *data, uint32_t words_pow2, uint32_t iters, bool atomics,
                                uint32_t blocks, uint32_t *sink, hipStream_t stream);

// S = sum of R (exact, uint64) into *sum (caller zeroes it).
hipError_t launch_sum_u32(const uint32_t *x, int32_t n, unsigned long long *sum,
                          hipStream_t stream);

// diag / farness / closeness from R and S (any output may be null).
hipError_t launch_estimate(const uint32_t *R, int32_t n, uint32_t tau, int literal,
                           const unsigned long long *sum, double *diag, double *farness,
                           double *closeness, hipStream_t stream);

// Block CG on (alpha L + I) X = B, row-major n x k, k <= 64.
struct CgWork {
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const double *weights;  // edge weights (weighted Laplacian), or null
    const double *wdeg;     // weighted degrees (with weights), or null
    uint32_t n, k;
    double alpha;
    uint32_t max_blocks;
    const double *B;        // n x k right-hand sides
    double *X;              // n x k solution (binary64)
    double *R64;            // n x k binary64 residual B - A X
    void *r, *z, *p, *q, *d;  // n x k inner vectors in the inner precision
    double *partial_a, *partial_b;  // max_blocks x 64 partial sums
    double *scalars;        // 8 x 64: rz, rz_new, pq, rr, tol2, step, beta, active
    double *scale;          // 64: residual norms the inner solve is scaled by
    double *res_rr, *res_bb;  // 64: |R_j|^2 and |B_j|^2
    unsigned int *any;      // device flag: some column still active
};
// Inner Jacobi-preconditioned CG on A d = R64 / scale (per column), then
// X += scale * d.  Stops a column when |r_j|^2 <= tol2_j (scalars[256 + j]).
template <typename T>
hipError_t cg_inner(const CgWork &w, uint32_t max_iters, uint32_t poll, uint32_t *iters,
                    hipStream_t stream);
// R64 = B - A X and |R_j|^2 into res_rr (and |B_j|^2 into res_bb).
hipError_t cg_residual(const CgWork &w, bool with_b, hipStream_t stream);

}  // namespace fc
