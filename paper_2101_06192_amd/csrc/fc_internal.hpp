// Host-side internals shared by the C-ABI translation units: the context,
// device buffers and the graph preparation helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "fc.h"
#include "fc_kernels.hpp"

struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct Small {  // device-side counters of one call
    fc::Totals totals;
    unsigned int queue;
    unsigned int graph_err;
    unsigned long long sum;
    unsigned int dmax;
    unsigned int pad;
    unsigned long long phase_ticks[8];
    unsigned int class_bounds[4];  // n0, n1, n2, n3 of the degree-class relabelling
    double wtotal;                 // sum of the weighted degrees (weighted graphs)
};

struct fc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string last_error;
    DevBuf state, vrec, row_ptr, col_idx, small, rtmp, thr, cword, ckk, clists, clevels, cbits;
    DevBuf s_r64, s_r, s_z, s_p, s_q, s_d, s_pa, s_pb, s_small, s_wdeg;  // solver workspace
    DevBuf rl_blk, rl_base, rl_inv, rl_orig, rl_vrec, rl_adj;     // degree-class relabelling
    DevBuf iso;                                                   // isolated-vertex bitmap
    DevBuf corigt;                                                // hybrid: target ids per slot
    DevBuf cpre;                                                  // LDS: pre-drawn tree words
    DevBuf weights, wsum, wthr;  // staged edge weights (host graphs), running row weight sums,
                                 // step thresholds
    DevBuf rk_key0, rk_key1, rk_val0, rk_val1, rk_hist, rk_thist, rk_ra, rk_rb, rk_s;  // ranking
    DevBuf g_mat, g_vec, g_part, g_taken, g_scr;  // group closeness: matrix, vectors, sums, flags, scratch
    DevBuf t_ex, t_exl, t_ecnt, t_pc, t_sc, t_bl, t_xb;  // tile sampler (exits, counts, lists)
    hipEvent_t ev0 = nullptr, ev1 = nullptr, evm = nullptr;
    size_t state_budget = 0;      // bytes of per-tree state the sampler may use
    uint32_t lanes_per_wave = 64; // active lanes per wave in the lane sampler
    uint32_t max_slots = 0;       // 0 = as many trees in flight as memory allows
    uint32_t cu_count = 256;
    size_t max_lds = 65536;       // dynamic LDS a workgroup may use
    uint32_t coop_threads = 512;  // threads per workgroup in the workgroup sampler
    uint32_t coop_wg_per_cu = 3;  // resident workgroups per CU in the workgroup sampler
    uint32_t force_sampler = 0;   // 0 auto, 1 lane, 2 coop, 3 lds, 4 hyb (environment override)
    bool coop_lds_bits = true;    // settled bitmap in LDS when it fits
    bool coop_word32 = true;      // 32-bit tree words when target and count fit
    bool coop_in_bits = true;     // in-arrow bitmap in LDS when both bitmaps fit
    bool phase_timing = false;    // per-phase wall-clock ticks of the workgroup sampler
    uint32_t max_draws = 0;       // per-vertex draw limit in one tree (0: each sampler's own)
    uint32_t hyb_hot_cap = 0x7FFFFFFF;  // hybrid sampler: cap on the LDS-resident id prefix
    bool coop_lds_counts = true;  // in-arrow counters in LDS when the tree's fields fit
    uint32_t lds_threads = 0;     // threads per workgroup of the LDS-counter sampler (0: by n)
    uint32_t lds_wg_per_cu = 0;   // its resident workgroups per CU (0: as many as fit)
    uint32_t predraw_mib = 32768;  // budget of pre-drawn first arrows (0: off)
    bool kendall_pairs = false;   // Kendall's tau by all pairs instead of merge-sort counts
    uint32_t lds_repop = 3;       // re-formed 2-cycle pops: 0 never, 1 weighted graphs, 2 always,
                                  // 3 always, and timed both ways by batch autotuning
    uint32_t coop_repop = 2;      // the same for the global-counter sampler
    uint32_t lds_lean = 0;        // LDS-counter sampler: the lean register shape for workgroups
                                  // of at most 512 threads (batch autotuning times both)
    uint32_t tile_size = 0;       // tile sampler: vertices per tile (0: the widest that fits LDS)
    uint32_t tile_cross_permille = 100;  // picked automatically when at most this share (per
                                         // mille) of the CSR entries cross tiles
    uint32_t tile_threads = 1024; // threads per workgroup of the tile sampler
    uint32_t tile_repop = 2;      // tile sampler's re-formed 2-cycle pops: 0 never, 1 weighted, 2 always
    uint32_t tile_bits_lds = 1;   // tile sampler's exit and settled bitmaps in LDS when they fit (0: global)
    double wall_khz = 100000.0;   // device wall clock rate
    // Arena mode (fc_sample_noalloc): every buffer of one call is carved from
    // this device range instead of being allocated; null in ordinary contexts.
    char *arena = nullptr;
    size_t arena_size = 0, arena_off = 0;
};


#define FC_HIP(ctx, expr, what)                          \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
    } while (0)


namespace fc_host {

// static LDS of the LDS-counter kernel (item, tails, totals, phase clocks) with margin
constexpr size_t kLdsStaticBytes = 1024;
// fewest non-isolated vertices for which the LDS sampler draws first arrows ahead
constexpr uint32_t kPredrawMinVertices = 16384;

int set_err(fc_ctx *ctx, int code, const std::string &msg);
int hip_fail(fc_ctx *ctx, hipError_t e, const char *what);
// Grow-only device buffer: (re)allocates when `bytes` exceeds its size; in
// arena mode carves it from the context's arena instead (never allocates).
int ensure(fc_ctx *ctx, DevBuf &b, size_t bytes, const char *what);
// Bytes of per-tree state the sampler may use now: the context's budget, or
// in arena mode what is left of the arena.
size_t state_budget_now(const fc_ctx *ctx);
uint32_t env_u32(const char *name, uint32_t dflt);
bool valid_alpha(double a);

// Resolved device view of a graph for one call.
struct GraphView {
    int32_t n = 0;
    int64_t nnz = 0;
    const int32_t *row_ptr = nullptr;
    const int32_t *col_idx = nullptr;
    const double *weights = nullptr;  // device edge weights, or null (unit weights)
};

int check_graph_args(fc_ctx *ctx, const fc_graph *g);
// Stage (if on the host) and validate the CSR (and weights) on the device.
int prepare_graph(fc_ctx *ctx, const fc_graph *g, bool trusted, GraphView *out);
// Running row weight sums and step thresholds of a weighted graph into the two
// buffers (both null for an unweighted graph).
int weight_tables(fc_ctx *ctx, const GraphView &g, DevBuf &sbuf, DevBuf &tbuf, const double **S,
                  const uint32_t **T);
double now_ms();
int begin(fc_ctx *ctx);
// Threads per workgroup of the LDS-counter sampler for `trees` trees whose
// counters and bitmap take lds_words words of LDS.
uint32_t lds_threads_for(const fc_ctx *ctx, uint64_t trees, uint32_t lds_words);
// Bits of the target field so that n < 2^tshift, and whether a 32-bit tree
// word also holds an in-arrow count up to dmax.
void word_layout(uint32_t n, uint32_t dmax, bool allow32, uint32_t *tshift, bool *word32);
// Global-counter sampler: LDS words of the re-pop filter for a launch of
// `threads` x `per_cu` workgroups (0 when the option is off or nothing fits).
uint32_t coop_repop_words(const fc_ctx *ctx, uint32_t threads, uint32_t per_cu, bool lds_bits,
                          bool in_bits, bool word32, uint32_t n, bool weighted);

}  // namespace fc_host
