// Host implementation of the C-ABI declared in include/fc.h.
//
// The library owns device scratch (vertex records, per-tree state, staged
// host graphs, small counters) per context and grows it on demand; callers
// own every input and output array.  All work goes to the context's stream
// and each call synchronises before it returns.
#include "fc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "fc_internal.hpp"

#pragma STDC FP_CONTRACT OFF

static_assert(sizeof(fc_graph) == 48, "fc_graph layout");
static_assert(sizeof(fc_params) == 56, "fc_params layout");
static_assert(sizeof(fc_stats) == 136, "fc_stats layout");
static_assert(sizeof(fc_job) == 88, "fc_job layout");

// Device scratch of fc_sample_noalloc: one array per device, loaded with the
// code object and held until the process ends.  Host code never uses the
// array's name as an address (on the host it is only a stand-in); it uses the
// device address that hipGetSymbolAddress returns, taken once per device when
// a context is created on it.
static constexpr size_t kStaticScratchBytes = static_cast<size_t>(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// The device address of `scratch` on `device` (current), looked up once.
void *scratch_of(int device, hipError_t *err) {
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device] && g_scratch_err[device] == hipSuccess) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            g_scratch_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
        } else {
            g_scratch_ptr[device] = p;
        }
    }
    *err = g_scratch_err[device];
    return g_scratch_ptr[device];
}
}  // namespace

namespace fc_host {

int set_err(fc_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->last_error = msg;
    return code;
}

int hip_fail(fc_ctx *ctx, hipError_t e, const char *what) {
    return set_err(ctx, e == hipErrorOutOfMemory ? FC_ERR_NOMEM : FC_ERR_HIP,
                   std::string(what) + ": " + hipGetErrorString(e));
}

int ensure(fc_ctx *ctx, DevBuf &b, size_t bytes, const char *what) {
    if (bytes == 0) bytes = 16;
    if (b.bytes >= bytes) return FC_OK;
    if (ctx->arena) {  // carve, 256-byte aligned; a buffer that must grow gets a new range
        const size_t off = (ctx->arena_off + 255u) & ~static_cast<size_t>(255u);
        if (off > ctx->arena_size || bytes > ctx->arena_size - off)
            return set_err(ctx, FC_ERR_NOMEM,
                           std::string("the static scratch (") +
                               std::to_string(ctx->arena_size >> 20) + " MiB) cannot hold " +
                               what + " (" + std::to_string(bytes) + " bytes with " +
                               std::to_string(off) + " already in use by this call)");
        b.ptr = ctx->arena + off;
        b.bytes = bytes;
        ctx->arena_off = off + bytes;
        return FC_OK;
    }
    if (b.ptr) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
    hipError_t e = hipMalloc(&b.ptr, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.ptr = nullptr;
        return set_err(ctx, FC_ERR_NOMEM, std::string("allocating ") + what + " (" +
                                              std::to_string(bytes) + " bytes) failed");
    }
    b.bytes = bytes;
    return FC_OK;
}

size_t state_budget_now(const fc_ctx *ctx) {
    if (!ctx->arena) return ctx->state_budget;
    // what is left, less the alignment of the per-slot buffers still to carve
    const size_t used = ctx->arena_off + 8u * 256u;
    return used < ctx->arena_size ? ctx->arena_size - used : 0u;
}

uint32_t env_u32(const char *name, uint32_t dflt) {
    const char *s = std::getenv(name);
    if (!s || !*s) return dflt;
    return static_cast<uint32_t>(std::strtoul(s, nullptr, 10));
}

bool valid_alpha(double a) { return std::isfinite(a) && a > 0.0; }


int check_graph_args(fc_ctx *ctx, const fc_graph *g) {
    if (!g) return set_err(ctx, FC_ERR_ARG, "graph is NULL");
    if (g->n < 0 || g->nnz < 0) return set_err(ctx, FC_ERR_ARG, "negative n or nnz");
    if (g->n >= 0x7FFFFFFF) return set_err(ctx, FC_ERR_UNSUPPORTED, "n must be < 2^31 - 1");
    if (g->nnz >= 0x7FFFFFFFLL) return set_err(ctx, FC_ERR_UNSUPPORTED, "nnz must be < 2^31");
    if (g->mem != FC_MEM_HOST && g->mem != FC_MEM_DEVICE)
        return set_err(ctx, FC_ERR_ARG, "graph.mem must be FC_MEM_HOST or FC_MEM_DEVICE");
    if (!g->row_ptr) return set_err(ctx, FC_ERR_ARG, "row_ptr is NULL");
    if (g->nnz > 0 && !g->col_idx) return set_err(ctx, FC_ERR_ARG, "col_idx is NULL");
    return FC_OK;
}

int prepare_graph(fc_ctx *ctx, const fc_graph *g, bool trusted, GraphView *out) {
    int rc = check_graph_args(ctx, g);
    if (rc) return rc;
    GraphView v;
    v.n = g->n;
    v.nnz = g->nnz;
    if (g->mem == FC_MEM_HOST) {
        if ((rc = ensure(ctx, ctx->row_ptr, sizeof(int32_t) * (static_cast<size_t>(g->n) + 1), "row_ptr")))
            return rc;
        if ((rc = ensure(ctx, ctx->col_idx, sizeof(int32_t) * static_cast<size_t>(g->nnz), "col_idx")))
            return rc;
        FC_HIP(ctx, hipMemcpyAsync(ctx->row_ptr.ptr, g->row_ptr,
                                   sizeof(int32_t) * (static_cast<size_t>(g->n) + 1),
                                   hipMemcpyHostToDevice, ctx->stream), "copy row_ptr");
        if (g->nnz)
            FC_HIP(ctx, hipMemcpyAsync(ctx->col_idx.ptr, g->col_idx,
                                       sizeof(int32_t) * static_cast<size_t>(g->nnz),
                                       hipMemcpyHostToDevice, ctx->stream), "copy col_idx");
        v.row_ptr = static_cast<const int32_t *>(ctx->row_ptr.ptr);
        v.col_idx = static_cast<const int32_t *>(ctx->col_idx.ptr);
        if (g->weights && g->nnz) {
            if ((rc = ensure(ctx, ctx->weights, sizeof(double) * static_cast<size_t>(g->nnz),
                             "weights")))
                return rc;
            FC_HIP(ctx, hipMemcpyAsync(ctx->weights.ptr, g->weights,
                                       sizeof(double) * static_cast<size_t>(g->nnz),
                                       hipMemcpyHostToDevice, ctx->stream), "copy weights");
            v.weights = static_cast<const double *>(ctx->weights.ptr);
        }
    } else {
        v.row_ptr = g->row_ptr;
        v.col_idx = g->col_idx;
        v.weights = g->nnz ? g->weights : nullptr;
    }
    if (!trusted) {
        Small *sm = static_cast<Small *>(ctx->small.ptr);
        unsigned int err = 0;
        FC_HIP(ctx, hipMemsetAsync(&sm->graph_err, 0, sizeof(unsigned int), ctx->stream), "memset");
        FC_HIP(ctx, fc::launch_validate_rows(v.row_ptr, v.n, v.nnz, &sm->graph_err, ctx->stream),
               "validate_rows launch");
        FC_HIP(ctx, hipMemcpyAsync(&err, &sm->graph_err, sizeof(err), hipMemcpyDeviceToHost,
                                   ctx->stream), "copy error word");
        FC_HIP(ctx, hipStreamSynchronize(ctx->stream), "validate_rows");
        if (err) return set_err(ctx, FC_ERR_GRAPH, "row_ptr is not monotone from 0 to nnz");
        FC_HIP(ctx, fc::launch_validate_cols(v.row_ptr, v.col_idx, v.weights, v.n, v.nnz,
                                             &sm->graph_err, ctx->stream),
               "validate_cols launch");
        FC_HIP(ctx, hipMemcpyAsync(&err, &sm->graph_err, sizeof(err), hipMemcpyDeviceToHost,
                                   ctx->stream), "copy error word");
        FC_HIP(ctx, hipStreamSynchronize(ctx->stream), "validate_cols");
        if (err) {
            std::string m = "graph is not simple, sorted and symmetric:";
            if (err & fc::kErrGraphColumn) m += " column out of range;";
            if (err & fc::kErrGraphSelfLoop) m += " self-loop;";
            if (err & fc::kErrGraphOrder) m += " row not strictly ascending;";
            if (err & fc::kErrGraphAsymmetric) m += " missing reverse edge;";
            if (err & fc::kErrGraphWeight) m += " weight not 0 or in [2^-64, 2^64];";
            if (err & fc::kErrGraphWeightAsym) m += " weight differs from its reverse entry's;";
            return set_err(ctx, FC_ERR_GRAPH, m);
        }
    }
    *out = v;
    return FC_OK;
}

int weight_tables(fc_ctx *ctx, const GraphView &g, DevBuf &sbuf, DevBuf &tbuf, const double **S,
                  const uint32_t **T) {
    *S = nullptr;
    *T = nullptr;
    if (!g.weights || g.nnz == 0) return FC_OK;
    const size_t nnz = static_cast<size_t>(g.nnz);
    int rc;
    if ((rc = ensure(ctx, sbuf, sizeof(double) * nnz, "row weight sums")) ||
        (rc = ensure(ctx, tbuf, sizeof(uint32_t) * (nnz + fc::kWeightedScan), "step thresholds")))
        return rc;
    double *s = static_cast<double *>(sbuf.ptr);
    uint32_t *t = static_cast<uint32_t *>(tbuf.ptr);
    FC_HIP(ctx, fc::launch_row_wsum(g.row_ptr, g.weights, g.n, s, ctx->stream), "row weight sums");
    FC_HIP(ctx, fc::launch_step_thresholds(g.row_ptr, s, g.n, g.nnz, t, ctx->stream),
           "step thresholds");
    *S = s;
    *T = t;
    return FC_OK;
}

int check_params(fc_ctx *ctx, const fc_params *p) {
    if (!p) return set_err(ctx, FC_ERR_ARG, "params is NULL");
    if (!valid_alpha(p->alpha)) return set_err(ctx, FC_ERR_ARG, "alpha must be finite and > 0");
    return FC_OK;
}

int tau_for(fc_ctx *ctx, const fc_params *p, const GraphView &g, uint32_t *tau) {
    if (p->tau) {
        *tau = p->tau;
        return FC_OK;
    }
    int rc = fc_tau(g.nnz / 2, g.n, p->eps, p->delta, p->kappa, tau);
    if (rc) return set_err(ctx, rc, "tau = 0 needs 0 < eps < 1, 0 < delta < 1, 0 <= kappa < 1");
    return FC_OK;
}

// Runs the sampler over [tree_begin, tree_begin + tree_count).
int run_sampler(fc_ctx *ctx, const GraphView &g, const fc_params *p, uint32_t tree_begin,
                uint32_t tree_count, uint32_t *root_counts, uint64_t *visit_counts,
                uint64_t *tree_digests, uint64_t *tree_steps, int32_t *parents,
                uint32_t *tree_visits, fc_stats *stats) {
    int rc;
    Small *sm = static_cast<Small *>(ctx->small.ptr);
    FC_HIP(ctx, hipMemsetAsync(sm, 0, sizeof(Small), ctx->stream), "memset counters");
    if (stats) {
        stats->tau = tree_count;
        stats->trees_in_flight = 0;
        stats->walk_steps = stats->roots = stats->digest_sum = 0;
        stats->ms_sample = 0.0;
        stats->sampler[0] = 0;
    }
    if (g.n == 0 || tree_count == 0) return FC_OK;
    if ((rc = ensure(ctx, ctx->vrec, sizeof(fc::VRec) * static_cast<size_t>(g.n), "vertex records")))
        return rc;
    fc::VRec *vrec = static_cast<fc::VRec *>(ctx->vrec.ptr);
    if ((rc = ensure(ctx, ctx->iso, 4u * ((static_cast<size_t>(g.n) + 31u) / 32u), "isolated bitmap")))
        return rc;
    const double *wsum = nullptr;
    const uint32_t *wthr = nullptr;
    if ((rc = weight_tables(ctx, g, ctx->wsum, ctx->wthr, &wsum, &wthr))) return rc;
    const bool weighted = wsum != nullptr;
    const bool repop = ctx->lds_repop >= 2 || (ctx->lds_repop == 1 && weighted);
    FC_HIP(ctx, fc::launch_build_vrec(g.row_ptr, wsum, g.n, p->alpha, vrec, &sm->dmax,
                                      static_cast<uint32_t *>(ctx->iso.ptr), &sm->wtotal,
                                      ctx->stream),
           "build_vrec");
    double vol = static_cast<double>(g.nnz);  // sum of the (weighted) degrees
    if (weighted) {
        FC_HIP(ctx, hipMemcpyAsync(&vol, &sm->wtotal, sizeof(vol), hipMemcpyDeviceToHost,
                                   ctx->stream), "copy weighted volume");
        FC_HIP(ctx, hipStreamSynchronize(ctx->stream), "weighted volume");
    }

    // which sampler: the lane sampler needs many trees to fill the GPU; the
    // workgroup sampler parallelises inside each tree
    // mode: 1 lane, 2 workgroup with global counters, 3 workgroup with LDS counters
    uint32_t mode = 0;
    if (p->flags & FC_FLAG_SAMPLER_LANE) mode = 1;
    else if (p->flags & FC_FLAG_SAMPLER_COOP) mode = 2;
    else if (p->flags & FC_FLAG_SAMPLER_LDS) mode = 3;
    else if (p->flags & FC_FLAG_SAMPLER_HYB) mode = 4;
    else if (p->flags & FC_FLAG_SAMPLER_TILE) mode = 5;
    else mode = ctx->force_sampler;
    // automatically always a workgroup sampler: measured, the LDS-counter one beats
    // the lane-per-tree walk even with 2^18 trees of a 1000-vertex graph
    const bool use_coop = mode == 0 || mode >= 2;
    // expected steps per tree are at most n + alpha vol (n + 2 alpha m without
    // weights); a valid run never comes near 256 times that, so exceeding it
    // marks a fault, not bad luck
    const double cap = 256.0 * (static_cast<double>(g.n) + p->alpha * vol) + 1048576.0;
    const unsigned long long step_cap =
        cap > 4.0e18 ? 4000000000000000000ull : static_cast<unsigned long long>(cap);
    size_t slots = 0;
    const char *kname = use_coop ? "wilson_coop" : "wilson_lane";
    fc::LaneArgs a{};
    fc::CoopArgs c{};
    bool lds_bits = false, in_bits = false, word32 = false;
    uint32_t repop_words = 0;  // global-counter sampler: re-pop filter words (0: off)
    bool use_lds = false, use_hyb = false, use_tile = false;
    fc::TileArgs ta{};
    uint32_t tile_threads = 1024;
    uint32_t lds_words = 0, lds_threads = 1024, hot = 0;
    bool lds_lean = false;  // LDS-counter sampler: the lean register shape
    uint32_t tshift = 32;
    unsigned int dmax = 0;
    if (use_coop) {
        // LDS-counter variant when the degree-class count fields and the settled
        // bitmap of one tree fit in LDS (at least 4 + 1 bits per vertex)
        // (isolated vertices need no LDS, so only the id width bounds n here)
        const bool try_lds = (mode == 3 || (mode == 0 && ctx->coop_lds_counts)) &&
                             g.n < (1 << fc::kRelabelIdBits);
        const uint32_t nb = fc::relabel_blocks(static_cast<uint32_t>(g.n));
        if (try_lds) {
            if ((rc = ensure(ctx, ctx->rl_blk, 4u * fc::kRelabelClasses * nb, "class counts")) ||
                (rc = ensure(ctx, ctx->rl_base, 4u * fc::kRelabelClasses * nb, "class offsets")))
                return rc;
            FC_HIP(ctx, fc::launch_class_bounds(g.row_ptr, static_cast<uint32_t>(g.n), false,
                                                static_cast<uint32_t *>(ctx->rl_blk.ptr),
                                                static_cast<uint32_t *>(ctx->rl_base.ptr),
                                                sm->class_bounds, ctx->stream),
                   "class bounds");
        }
        unsigned int cb[4] = {0, 0, 0, 0};
        FC_HIP(ctx, hipMemcpyAsync(&dmax, &sm->dmax, sizeof(dmax), hipMemcpyDeviceToHost, ctx->stream),
               "copy dmax");
        if (try_lds)
            FC_HIP(ctx, hipMemcpyAsync(cb, sm->class_bounds, sizeof(cb), hipMemcpyDeviceToHost,
                                       ctx->stream), "copy class bounds");
        FC_HIP(ctx, hipStreamSynchronize(ctx->stream), "build_vrec");
        if (try_lds) {
            const fc::CountLayout L = fc::count_layout(cb[3], cb[0], cb[1], cb[2]);
            if (4u * static_cast<size_t>(L.words) + kLdsStaticBytes <= ctx->max_lds) {
                use_lds = true;
                lds_words = L.words;
            }
        }
        if (mode == 3 && !use_lds)
            return set_err(ctx, FC_ERR_UNSUPPORTED,
                           "the in-arrow counters of one tree do not fit in LDS");
        // tile sampler: when the LDS-counter variant does not fit and most edges join
        // ids of the same tile (graphs with local ids: grids, road networks)
        if (!use_lds && (mode == 5 || (mode == 0 && ctx->coop_lds_counts)) && g.n >= 1) {
            uint32_t B = ctx->tile_size;
            if (B == 0) {  // the widest tile whose arrays fit in LDS
                B = fc::kTileMax;
                while (B > 64u && fc::tile_lds_bytes(B) + kLdsStaticBytes > ctx->max_lds) B -= 64u;
            }
            const uint32_t ntiles = static_cast<uint32_t>((static_cast<uint64_t>(g.n) + B - 1u) / B);
            bool fits = fc::tile_lds_bytes(B) + kLdsStaticBytes <= ctx->max_lds;
            bool local = mode == 5;
            if (fits && !local && g.nnz > 0) {
                FC_HIP(ctx, hipMemsetAsync(&sm->sum, 0, sizeof(unsigned long long), ctx->stream),
                       "memset cross count");
                FC_HIP(ctx, fc::launch_count_cross(g.row_ptr, g.col_idx, static_cast<uint32_t>(g.n),
                                                   B, &sm->sum, ctx->stream),
                       "count_cross");
                unsigned long long cross = 0;
                FC_HIP(ctx, hipMemcpyAsync(&cross, &sm->sum, sizeof(cross), hipMemcpyDeviceToHost,
                                           ctx->stream), "copy cross count");
                FC_HIP(ctx, hipStreamSynchronize(ctx->stream), "count_cross");
                local = static_cast<double>(cross) * 1000.0 <=
                        static_cast<double>(ctx->tile_cross_permille) * static_cast<double>(g.nnz);
            }
            if (mode == 5 && !fits)
                return set_err(ctx, FC_ERR_UNSUPPORTED, "the tile sampler's tile does not fit in LDS");
            if (fits && local) {
                use_tile = true;
                ta.B = B;
                ta.Bp = (B + 63u) & ~63u;
                ta.ntiles = ntiles;
            }
        }
        // hybrid variant: the widest-class (highest-degree) prefix of the ids in LDS.
        // Automatically only where the global-counter variant cannot keep its
        // settled bitmap in LDS either (beyond that size the hybrid wins).
        const bool coop_bits_fit = fc::coop_lds_bytes(static_cast<uint32_t>(g.n)) + 1024u <= ctx->max_lds;
        if (!use_lds && !use_tile &&
            (mode == 4 || (mode == 0 && ctx->coop_lds_counts && !coop_bits_fit)) && g.n >= 1) {
            if ((rc = ensure(ctx, ctx->rl_blk, 4u * fc::kRelabelClasses * nb, "class counts")) ||
                (rc = ensure(ctx, ctx->rl_base, 4u * fc::kRelabelClasses * nb, "class offsets")))
                return rc;
            FC_HIP(ctx, fc::launch_class_bounds(g.row_ptr, static_cast<uint32_t>(g.n), true,
                                                static_cast<uint32_t *>(ctx->rl_blk.ptr),
                                                static_cast<uint32_t *>(ctx->rl_base.ptr),
                                                sm->class_bounds, ctx->stream),
                   "class bounds");
            FC_HIP(ctx, hipMemcpyAsync(cb, sm->class_bounds, sizeof(cb), hipMemcpyDeviceToHost,
                                       ctx->stream), "copy class bounds");
            FC_HIP(ctx, hipStreamSynchronize(ctx->stream), "class bounds");
            // largest prefix whose fields and settled bits fit
            uint32_t lo = 0, hi = cb[3];
            while (lo < hi) {
                const uint32_t mid = lo + (hi - lo + 1) / 2;
                if (4u * static_cast<size_t>(fc::hot_layout(mid, cb[0], cb[1], cb[2]).words) +
                        kLdsStaticBytes <= ctx->max_lds)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            lo = std::min<uint32_t>(lo, ctx->hyb_hot_cap);
            if (lo > 0 || cb[3] == 0 || mode == 4) {
                use_hyb = true;
                hot = lo;
                lds_words = fc::hot_layout(hot, cb[0], cb[1], cb[2]).words;
            }
        }
        if (mode == 4 && !use_hyb)
            return set_err(ctx, FC_ERR_UNSUPPORTED, "no vertex of the graph fits the hybrid sampler");
        if (use_hyb) {
            kname = "wilson_hyb";
            const size_t n = static_cast<size_t>(g.n);
            if ((rc = ensure(ctx, ctx->rl_inv, 4u * n, "relabel inverse")) ||
                (rc = ensure(ctx, ctx->rl_orig, 4u * n, "relabel ids")) ||
                (rc = ensure(ctx, ctx->rl_vrec, sizeof(fc::VRec) * n, "relabelled records")) ||
                (rc = ensure(ctx, ctx->rl_adj, 8u * static_cast<size_t>(g.nnz), "relabelled adjacency")))
                return rc;
            FC_HIP(ctx, fc::launch_relabel_graph(g.row_ptr, g.col_idx, static_cast<uint32_t>(g.n),
                                                 g.nnz, static_cast<const uint32_t *>(ctx->rl_base.ptr),
                                                 32u, static_cast<uint32_t *>(ctx->rl_inv.ptr),
                                                 static_cast<uint32_t *>(ctx->rl_orig.ptr),
                                                 static_cast<unsigned long long *>(ctx->rl_adj.ptr),
                                                 ctx->stream),
                   "relabel");
            FC_HIP(ctx, fc::launch_relabel_vrec(vrec, static_cast<const uint32_t *>(ctx->rl_inv.ptr),
                                                static_cast<uint32_t>(g.n),
                                                static_cast<fc::VRec *>(ctx->rl_vrec.ptr), ctx->stream),
                   "relabel records");
            const size_t per_slot = (8u + 4u + 8u + 24u + 4u) * n + 8u;
            slots = std::max<size_t>(1, state_budget_now(ctx) / per_slot);
            slots = std::min<size_t>(slots, tree_count);
            lds_threads = lds_threads_for(ctx, tree_count, lds_words);
            const int fit = fc::hyb_max_active(lds_threads, lds_words, weighted);
            uint32_t per_cu = ctx->lds_wg_per_cu ? ctx->lds_wg_per_cu : 64u;
            per_cu = fit > 0 ? std::min<uint32_t>(per_cu, static_cast<uint32_t>(fit)) : 1u;
            slots = std::min<size_t>(slots, static_cast<size_t>(ctx->cu_count) * per_cu);
            if (ctx->max_slots) slots = std::min<size_t>(slots, ctx->max_slots);
            if ((rc = ensure(ctx, ctx->cword, 8u * n * slots, "tree words")) ||
                (rc = ensure(ctx, ctx->corigt, 4u * n * slots, "target ids")) ||
                (rc = ensure(ctx, ctx->ckk, 8u * n * slots, "draw counts")) ||
                (rc = ensure(ctx, ctx->clists, 24u * n * slots, "lists")) ||
                (rc = ensure(ctx, ctx->clevels, 4u * (n + 2u) * slots, "levels")))
                return rc;
            FC_HIP(ctx, hipMemsetAsync(ctx->ckk.ptr, 0, 8u * n * slots, ctx->stream),
                   "memset draw counts");
            c.word = ctx->cword.ptr;
            c.origt = static_cast<uint32_t *>(ctx->corigt.ptr);
            c.kk = static_cast<uint64_t *>(ctx->ckk.ptr);
            c.lists = static_cast<uint64_t *>(ctx->clists.ptr);
            c.levels = static_cast<uint32_t *>(ctx->clevels.ptr);
            c.bits = nullptr;  // settled flags live in the tree words
            c.n_max = static_cast<uint32_t>(g.n);
            c.slots = static_cast<uint32_t>(slots);
            c.item_count = tree_count;
            c.key0 = static_cast<uint32_t>(p->seed);
            c.key1 = static_cast<uint32_t>(p->seed >> 32);
            c.max_rounds = 0x40000000u;
            c.k_limit = ctx->max_draws ? ctx->max_draws : 0x7FFFFFFFu;
            c.queue = &sm->queue;
            c.totals = &sm->totals;
            c.jobs = nullptr;
            c.item_job = nullptr;
            fc::CoopJob &j = c.single;
            j.vrec = static_cast<const fc::VRec *>(ctx->rl_vrec.ptr);
            j.col_idx = g.col_idx;
            j.wsum = wsum;
            j.wthr = wthr;
            j.adj = static_cast<const unsigned long long *>(ctx->rl_adj.ptr);
            j.orig = static_cast<const uint32_t *>(ctx->rl_orig.ptr);
            j.n = static_cast<uint32_t>(g.n);
            j.n0 = cb[0];
            j.n1 = cb[1];
            j.n2 = cb[2];
            j.n3 = cb[3];
            j.hot = hot;
            j.tree_count = tree_count;
            j.tshift = 32;
            j.stream_id = p->stream_id;
            j.tree_begin = tree_begin;
            j.first_item = 0;
            j.step_cap = step_cap;
            j.root_counts = root_counts;
            j.visit_counts = reinterpret_cast<unsigned long long *>(visit_counts);
            j.tree_digests = reinterpret_cast<unsigned long long *>(tree_digests);
            j.tree_steps = reinterpret_cast<unsigned long long *>(tree_steps);
            j.parents = parents;
            j.tree_visits = tree_visits;
            c.phase_ticks = ctx->phase_timing ? sm->phase_ticks : nullptr;
        }
        if (use_lds) {
            kname = "wilson_lds";
            const size_t n = static_cast<size_t>(g.n);
            if ((rc = ensure(ctx, ctx->rl_inv, 4u * n, "relabel inverse")) ||
                (rc = ensure(ctx, ctx->rl_orig, 4u * n, "relabel ids")) ||
                (rc = ensure(ctx, ctx->rl_vrec, sizeof(fc::VRec) * n, "relabelled records")) ||
                (rc = ensure(ctx, ctx->rl_adj, 8u * static_cast<size_t>(g.nnz), "relabelled adjacency")))
                return rc;
            FC_HIP(ctx, fc::launch_relabel_graph(g.row_ptr, g.col_idx, static_cast<uint32_t>(g.n),
                                                 g.nnz, static_cast<const uint32_t *>(ctx->rl_base.ptr),
                                                 fc::kRelabelIdBits,
                                                 static_cast<uint32_t *>(ctx->rl_inv.ptr),
                                                 static_cast<uint32_t *>(ctx->rl_orig.ptr),
                                                 static_cast<unsigned long long *>(ctx->rl_adj.ptr),
                                                 ctx->stream),
                   "relabel");
            FC_HIP(ctx, fc::launch_relabel_vrec(vrec, static_cast<const uint32_t *>(ctx->rl_inv.ptr),
                                                static_cast<uint32_t>(g.n),
                                                static_cast<fc::VRec *>(ctx->rl_vrec.ptr), ctx->stream),
                   "relabel records");
            const size_t per_slot = (8u + 24u + 4u) * n + 8u;
            slots = std::max<size_t>(1, state_budget_now(ctx) / per_slot);
            slots = std::min<size_t>(slots, tree_count);
            lds_threads = lds_threads_for(ctx, tree_count, lds_words);
            uint32_t per_cu = ctx->lds_wg_per_cu ? ctx->lds_wg_per_cu : 64u;
            lds_lean = ctx->lds_lean && lds_threads <= 512u;
            const int fit = fc::lds_max_active(lds_threads, lds_words, weighted, repop, lds_lean);
            if (fit > 0) per_cu = std::min<uint32_t>(per_cu, static_cast<uint32_t>(fit));
            else per_cu = 1;
            slots = std::min<size_t>(slots, static_cast<size_t>(ctx->cu_count) * per_cu);
            if (ctx->max_slots) slots = std::min<size_t>(slots, ctx->max_slots);
            // first arrows of all trees drawn ahead by one vertex-major kernel when
            // every tree's words fit the budget (the trees then work in place);
            // below 16384 vertices a tree's own first pass is too short to gain
            const size_t pre_bytes = 8u * n * static_cast<size_t>(tree_count);
            bool predraw = ctx->predraw_mib != 0 && cb[3] >= kPredrawMinVertices &&
                           pre_bytes <= (static_cast<size_t>(ctx->predraw_mib) << 20);
            if (predraw && ensure(ctx, ctx->cpre, pre_bytes, "pre-drawn tree words") != FC_OK) {
                predraw = false;  // not enough device memory: each tree draws its own
                ctx->last_error.clear();
            }
            if ((!predraw && (rc = ensure(ctx, ctx->cword, 8u * n * slots, "tree words"))) ||
                (rc = ensure(ctx, ctx->clists, 24u * n * slots, "lists")) ||
                (rc = ensure(ctx, ctx->clevels, 4u * (n + 2u) * slots, "levels")))
                return rc;
            c.word = predraw ? nullptr : ctx->cword.ptr;
            c.pre = predraw ? static_cast<uint64_t *>(ctx->cpre.ptr) : nullptr;
            c.kk = nullptr;  // draw counts travel in the tree words
            c.lists = static_cast<uint64_t *>(ctx->clists.ptr);
            c.levels = static_cast<uint32_t *>(ctx->clevels.ptr);
            c.bits = nullptr;
            c.n_max = static_cast<uint32_t>(g.n);
            c.slots = static_cast<uint32_t>(slots);
            c.item_count = tree_count;
            c.key0 = static_cast<uint32_t>(p->seed);
            c.key1 = static_cast<uint32_t>(p->seed >> 32);
            c.max_rounds = 0x40000000u;
            c.k_limit = ctx->max_draws ? ctx->max_draws : 0xFFFFFFFFu;
            c.queue = &sm->queue;
            c.totals = &sm->totals;
            c.jobs = nullptr;
            c.item_job = nullptr;
            fc::CoopJob &j = c.single;
            j.vrec = static_cast<const fc::VRec *>(ctx->rl_vrec.ptr);
            j.col_idx = g.col_idx;
            j.wsum = wsum;
            j.wthr = wthr;
            j.adj = static_cast<const unsigned long long *>(ctx->rl_adj.ptr);
            j.orig = static_cast<const uint32_t *>(ctx->rl_orig.ptr);
            j.n = static_cast<uint32_t>(g.n);
            j.n0 = cb[0];
            j.n1 = cb[1];
            j.n2 = cb[2];
            j.n3 = cb[3];
            j.tree_count = tree_count;
            j.tshift = 32;
            j.stream_id = p->stream_id;
            j.tree_begin = tree_begin;
            j.first_item = 0;
            j.step_cap = step_cap;
            j.root_counts = root_counts;
            j.visit_counts = reinterpret_cast<unsigned long long *>(visit_counts);
            j.tree_digests = reinterpret_cast<unsigned long long *>(tree_digests);
            j.tree_steps = reinterpret_cast<unsigned long long *>(tree_steps);
            j.parents = parents;
            j.tree_visits = tree_visits;
            c.phase_ticks = ctx->phase_timing ? sm->phase_ticks : nullptr;
        }
    }
    size_t tile_lds = 0;
    if (use_tile) {
        kname = "wilson_tile";
        const size_t n = static_cast<size_t>(g.n);
        const size_t bw = (n + 31u) >> 5;
        tile_threads = ctx->tile_threads;
        // the exit and settled bitmaps share the tiles' LDS when n bits fit
        const bool bits_lds = ctx->tile_bits_lds && 4u * bw + kLdsStaticBytes <= ctx->max_lds;
        tile_lds = std::max(fc::tile_lds_bytes(ta.B), bits_lds ? 4u * bw : 0u);
        const int fit = fc::tile_max_active(tile_threads, tile_lds, weighted);
        // first arrows of all trees drawn ahead when their targets fit the budget
        const size_t pre_bytes = 4u * n * static_cast<size_t>(tree_count);
        bool predraw = ctx->predraw_mib != 0 &&
                       pre_bytes <= (static_cast<size_t>(ctx->predraw_mib) << 20);
        if (predraw && ensure(ctx, ctx->cpre, pre_bytes, "pre-drawn targets") != FC_OK) {
            predraw = false;
            ctx->last_error.clear();
        }
        const size_t per_slot = (predraw ? 0u : 4u * n) + 8u * n + 2u * n + 4u * n * 3u + 12u * n +
                                4u * (n + 2u) + 4u * ta.ntiles + (bits_lds ? 4u : 8u) * bw +
                                10u * 256u;
        slots = std::max<size_t>(1, state_budget_now(ctx) / per_slot);
        slots = std::min<size_t>(slots, tree_count);
        const uint32_t per_cu = fit > 0 ? static_cast<uint32_t>(fit) : 1u;
        slots = std::min<size_t>(slots, static_cast<size_t>(ctx->cu_count) * per_cu);
        if (ctx->max_slots) slots = std::min<size_t>(slots, ctx->max_slots);
        if ((!predraw && (rc = ensure(ctx, ctx->cword, 4u * n * slots, "tree targets"))) ||
            (rc = ensure(ctx, ctx->ckk, 8u * n * slots, "draw counts")) ||
            (rc = ensure(ctx, ctx->t_ex, 2u * n * slots, "exits")) ||
            (rc = ensure(ctx, ctx->t_exl, 4u * n * slots, "exit lists")) ||
            (rc = ensure(ctx, ctx->t_pc, 4u * n * slots, "in-counts")) ||
            (rc = ensure(ctx, ctx->t_sc, 4u * n * slots, "exit successors")) ||
            (rc = ensure(ctx, ctx->t_ecnt, 4u * ta.ntiles * slots, "tile exit counts")) ||
            (rc = ensure(ctx, ctx->t_bl, 12u * n * slots, "lists")) ||
            (rc = ensure(ctx, ctx->clevels, 4u * (n + 2u) * slots, "levels")) ||
            (rc = ensure(ctx, ctx->cbits, 4u * bw * slots, "settled bitmap")) ||
            (!bits_lds && (rc = ensure(ctx, ctx->t_xb, 4u * bw * slots, "exit bitmap"))))
            return rc;
        FC_HIP(ctx, hipMemsetAsync(ctx->ckk.ptr, 0, 8u * n * slots, ctx->stream), "memset draw counts");
        FC_HIP(ctx, hipMemsetAsync(ctx->t_pc.ptr, 0, 4u * n * slots, ctx->stream), "memset in-counts");
        ta.vrec = vrec;
        ta.col_idx = g.col_idx;
        ta.wsum = wsum;
        ta.wthr = wthr;
        ta.n = static_cast<uint32_t>(g.n);
        ta.tree_begin = tree_begin;
        ta.tree_count = tree_count;
        ta.stream_id = p->stream_id;
        ta.key0 = static_cast<uint32_t>(p->seed);
        ta.key1 = static_cast<uint32_t>(p->seed >> 32);
        ta.slots = static_cast<uint32_t>(slots);
        ta.k_limit = ctx->max_draws ? ctx->max_draws : 0x7FFFFFFFu;
        ta.max_rounds = 0x40000000u;
        ta.step_cap = step_cap;
        ta.pre = predraw ? static_cast<uint32_t *>(ctx->cpre.ptr) : nullptr;
        ta.tw = predraw ? nullptr : static_cast<uint32_t *>(ctx->cword.ptr);
        ta.kk = static_cast<uint64_t *>(ctx->ckk.ptr);
        ta.ex = static_cast<uint16_t *>(ctx->t_ex.ptr);
        ta.exl = static_cast<uint32_t *>(ctx->t_exl.ptr);
        ta.ecnt = static_cast<uint32_t *>(ctx->t_ecnt.ptr);
        ta.pc = static_cast<uint32_t *>(ctx->t_pc.ptr);
        ta.sc = static_cast<uint32_t *>(ctx->t_sc.ptr);
        ta.bl = static_cast<uint32_t *>(ctx->t_bl.ptr);
        ta.lv = static_cast<uint32_t *>(ctx->clevels.ptr);
        ta.bits = static_cast<uint32_t *>(ctx->cbits.ptr);
        ta.xb = bits_lds ? nullptr : static_cast<uint32_t *>(ctx->t_xb.ptr);
        ta.bits_lds = bits_lds ? 1u : 0u;
        ta.repop = (ctx->tile_repop == 2 || (ctx->tile_repop == 1 && weighted)) ? 1u : 0u;
        ta.queue = &sm->queue;
        ta.totals = &sm->totals;
        ta.phase_ticks = ctx->phase_timing ? sm->phase_ticks : nullptr;
        ta.root_counts = root_counts;
        ta.visit_counts = reinterpret_cast<unsigned long long *>(visit_counts);
        ta.tree_digests = reinterpret_cast<unsigned long long *>(tree_digests);
        ta.tree_steps = reinterpret_cast<unsigned long long *>(tree_steps);
        ta.parents = parents;
        ta.tree_visits = tree_visits;
    }
    if (use_coop && !use_lds && !use_hyb && !use_tile) {
        // 32-bit tree words when target and in-arrow count both fit (the count of
        // a vertex never exceeds its degree)
        word_layout(static_cast<uint32_t>(g.n), dmax, ctx->coop_word32, &tshift, &word32);
        const size_t wbytes = word32 ? 4u : 8u;
        const size_t nwords = (static_cast<size_t>(g.n) + 31u) / 32u;
        lds_bits = ctx->coop_lds_bits &&
                   fc::coop_lds_bytes(static_cast<uint32_t>(g.n)) + 1024u <= ctx->max_lds;
        in_bits = lds_bits && ctx->coop_in_bits &&
                  2 * fc::coop_lds_bytes(static_cast<uint32_t>(g.n)) + 1024u <= ctx->max_lds;
        const size_t per_slot = (wbytes + 8u + 24u + 4u) * static_cast<size_t>(g.n) + 8u +
                                (lds_bits ? 0u : 4u * nwords);
        slots = std::max<size_t>(1, state_budget_now(ctx) / per_slot);
        slots = std::min<size_t>(slots, tree_count);
        // persistent workgroups: as many as requested per CU, but never more
        // than fit at once (a workgroup that starts late finds the queue empty)

        uint32_t per_cu = ctx->coop_wg_per_cu;
        const int fit = fc::coop_max_active(ctx->coop_threads, lds_bits, in_bits, word32,
                                            static_cast<uint32_t>(g.n), weighted, 0);
        if (fit > 0) per_cu = std::min<uint32_t>(per_cu, static_cast<uint32_t>(fit));
        repop_words = coop_repop_words(ctx, ctx->coop_threads, per_cu, lds_bits, in_bits, word32,
                                       static_cast<uint32_t>(g.n), weighted);
        slots = std::min<size_t>(slots, static_cast<size_t>(ctx->cu_count) * per_cu);
        if (ctx->max_slots) slots = std::min<size_t>(slots, ctx->max_slots);
        if ((rc = ensure(ctx, ctx->cword, wbytes * static_cast<size_t>(g.n) * slots, "tree words")))
            return rc;
        if ((rc = ensure(ctx, ctx->ckk, 8u * static_cast<size_t>(g.n) * slots, "draw counts"))) return rc;
        // epoch-tagged draw counts: zero once per launch, then each tree of a
        // slot uses the next epoch
        FC_HIP(ctx, hipMemsetAsync(ctx->ckk.ptr, 0, 8u * static_cast<size_t>(g.n) * slots, ctx->stream),
               "memset draw counts");
        if ((rc = ensure(ctx, ctx->clists, 24u * static_cast<size_t>(g.n) * slots, "lists")))
            return rc;
        if ((rc = ensure(ctx, ctx->clevels, 4u * (static_cast<size_t>(g.n) + 2u) * slots, "levels")))
            return rc;
        if (!lds_bits &&
            (rc = ensure(ctx, ctx->cbits, 4u * nwords * slots, "settled bitmap")))
            return rc;
        c.word = ctx->cword.ptr;
        c.kk = static_cast<uint64_t *>(ctx->ckk.ptr);
        c.lists = static_cast<uint64_t *>(ctx->clists.ptr);
        c.levels = static_cast<uint32_t *>(ctx->clevels.ptr);
        c.bits = lds_bits ? nullptr : static_cast<uint32_t *>(ctx->cbits.ptr);
        c.n_max = static_cast<uint32_t>(g.n);
        c.slots = static_cast<uint32_t>(slots);
        c.item_count = tree_count;
        c.key0 = static_cast<uint32_t>(p->seed);
        c.key1 = static_cast<uint32_t>(p->seed >> 32);
        c.max_rounds = 0x40000000u;
        c.k_limit = ctx->max_draws ? ctx->max_draws : 0x7FFFFFFFu;
        c.queue = &sm->queue;
        c.totals = &sm->totals;
        c.jobs = nullptr;
        c.item_job = nullptr;
        fc::CoopJob &j = c.single;
        j.vrec = vrec;
        j.col_idx = g.col_idx;
        j.wsum = wsum;
        j.wthr = wthr;
        j.iso = static_cast<const uint32_t *>(ctx->iso.ptr);
        j.tree_count = tree_count;
        j.n = static_cast<uint32_t>(g.n);
        j.tshift = tshift;
        j.stream_id = p->stream_id;
        j.tree_begin = tree_begin;
        j.first_item = 0;
        j.step_cap = step_cap;
        j.root_counts = root_counts;
        j.visit_counts = reinterpret_cast<unsigned long long *>(visit_counts);
        j.tree_digests = reinterpret_cast<unsigned long long *>(tree_digests);
        j.tree_steps = reinterpret_cast<unsigned long long *>(tree_steps);
        j.parents = parents;
        j.tree_visits = tree_visits;
        c.phase_ticks = ctx->phase_timing ? sm->phase_ticks : nullptr;
    } else if (!use_coop) {
        // trees in flight: bounded by the tree count and by the state budget
        const size_t per_slot = sizeof(uint64_t) * static_cast<size_t>(g.n);
        slots = std::max<size_t>(1, state_budget_now(ctx) / per_slot);
        slots = std::min<size_t>(slots, tree_count);
        if (ctx->max_slots) slots = std::min<size_t>(slots, ctx->max_slots);
        if ((rc = ensure(ctx, ctx->state, per_slot * slots, "per-tree state"))) return rc;
        FC_HIP(ctx, hipMemsetAsync(ctx->state.ptr, 0, per_slot * slots, ctx->stream), "memset state");
        a.vrec = vrec;
        a.col_idx = g.col_idx;
        a.wsum = wsum;
        a.wthr = wthr;
        a.state = static_cast<uint64_t *>(ctx->state.ptr);
        a.n = static_cast<uint32_t>(g.n);
        a.slots = static_cast<uint32_t>(slots);
        a.lanes_per_wave = std::max<uint32_t>(1, std::min<uint32_t>(64, ctx->lanes_per_wave));
        a.tree_begin = tree_begin;
        a.tree_count = tree_count;
        a.stream_id = p->stream_id;
        a.key0 = static_cast<uint32_t>(p->seed);
        a.key1 = static_cast<uint32_t>(p->seed >> 32);
        a.step_cap = step_cap;
        a.k_limit = ctx->max_draws ? ctx->max_draws : 0x7FFFFFFFu;
        a.queue = &sm->queue;
        a.root_counts = root_counts;
        a.visit_counts = reinterpret_cast<unsigned long long *>(visit_counts);
        a.tree_digests = reinterpret_cast<unsigned long long *>(tree_digests);
        a.tree_steps = reinterpret_cast<unsigned long long *>(tree_steps);
        a.parents = parents;
        a.tree_visits = tree_visits;
        a.totals = &sm->totals;
    }

    FC_HIP(ctx, hipEventRecord(ctx->ev0, ctx->stream), "event");
    if (use_tile) {
        if (ta.pre) {
            FC_HIP(ctx, fc::launch_tile_predraw(ta, ctx->stream), "tile_predraw launch");
            FC_HIP(ctx, hipEventRecord(ctx->evm, ctx->stream), "event");
        }
        FC_HIP(ctx, fc::launch_wilson_tile(ta, tile_threads, tile_lds, ctx->stream),
               "wilson_tile launch");
    } else if (use_hyb) {
        FC_HIP(ctx, fc::launch_wilson_hyb(c, lds_threads, lds_words, ctx->stream),
               "wilson_hyb launch");
    } else if (use_lds) {
        if (c.pre) {
            FC_HIP(ctx, fc::launch_lds_predraw(c, ctx->stream), "lds_predraw launch");
            FC_HIP(ctx, hipEventRecord(ctx->evm, ctx->stream), "event");
        }
        FC_HIP(ctx, fc::launch_wilson_lds(c, lds_threads, lds_words, weighted, repop, lds_lean,
                                             ctx->stream),
               "wilson_lds launch");
    } else if (use_coop) {
        FC_HIP(ctx, fc::launch_wilson_coop(c, ctx->coop_threads, lds_bits, in_bits, word32, weighted,
                                           repop_words, ctx->stream),
               "wilson_coop launch");
    } else
        FC_HIP(ctx, fc::launch_wilson_lane(a, ctx->stream), "wilson_lane launch");
    FC_HIP(ctx, hipEventRecord(ctx->ev1, ctx->stream), "event");
    fc::Totals tot;
    FC_HIP(ctx, hipMemcpyAsync(&tot, &sm->totals, sizeof(tot), hipMemcpyDeviceToHost, ctx->stream),
           "copy totals");
    FC_HIP(ctx, hipStreamSynchronize(ctx->stream), "sampler");
    if (tot.error & fc::kErrStepCap)
        return set_err(ctx, FC_ERR_HIP, "a tree exceeded the step bound (internal fault)");
    if (tot.error & fc::kErrVisitOverflow)
        return set_err(ctx, FC_ERR_OVERFLOW,
                       ctx->max_draws ? "a per-vertex draw count exceeded option max_draws"
                       : use_lds ? "a per-vertex draw count exceeded 2^28 - 1 (the LDS-counter "
                                   "sampler's limit; option coop_lds_counts = 0 allows 2^31 - 1)"
                                 : "a per-vertex visit counter exceeded 2^31 - 1");
    if (stats) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
        stats->trees_in_flight = static_cast<uint32_t>(slots);
        std::snprintf(stats->sampler, sizeof(stats->sampler), "%s", kname);
        stats->walk_steps = tot.walk_steps;
        stats->roots = tot.roots;
        stats->digest_sum = tot.digest_sum;
        stats->ms_sample = ms;
        stats->ms_predraw = 0.0;
        if ((use_lds && c.pre) || (use_tile && ta.pre)) {
            float pm = 0.f;
            (void)hipEventElapsedTime(&pm, ctx->ev0, ctx->evm);
            stats->ms_predraw = pm;
        }
        for (int i = 0; i < 8; ++i) stats->phase_ms[i] = 0.0;
        if ((use_coop || use_tile) && ctx->phase_timing) {
            unsigned long long ticks[8];
            FC_HIP(ctx, hipMemcpy(ticks, sm->phase_ticks, sizeof(ticks), hipMemcpyDeviceToHost),
                   "copy phase ticks");
            // per-workgroup average in milliseconds
            for (int i = 0; i < 8; ++i)
                stats->phase_ms[i] = static_cast<double>(ticks[i]) / ctx->wall_khz / static_cast<double>(slots);
        }
    }
    return FC_OK;
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

uint32_t coop_repop_words(const fc_ctx *ctx, uint32_t threads, uint32_t per_cu, bool lds_bits,
                          bool in_bits, bool word32, uint32_t n, bool weighted) {
    if (!(ctx->coop_repop == 2 || (ctx->coop_repop == 1 && weighted))) return 0;
    // what LDS per_cu workgroups leave free, up to 32 KiB (at least 256 B), without
    // lowering the workgroups per CU
    const int fit0 = fc::coop_max_active(threads, lds_bits, in_bits, word32, n, weighted, 0);
    if (fit0 > 0) per_cu = std::min<uint32_t>(per_cu, static_cast<uint32_t>(fit0));
    per_cu = std::max<uint32_t>(per_cu, 1);
    const size_t dyn = lds_bits ? (in_bits ? 2u : 1u) * fc::coop_lds_bytes(n) : 0u;
    const size_t share = ctx->max_lds / per_cu;
    const size_t room =
        std::min<size_t>(32768u, share > dyn + kLdsStaticBytes ? share - dyn - kLdsStaticBytes : 0u);
    uint32_t words = 0;
    for (uint32_t w = 64; 4u * w <= room; w <<= 1) words = w;
    while (words && fit0 > 0 &&
           fc::coop_max_active(threads, lds_bits, in_bits, word32, n, weighted, words) <
               static_cast<int>(per_cu))
        words = words > 64 ? words >> 1 : 0;
    return words;
}

void word_layout(uint32_t n, uint32_t dmax, bool allow32, uint32_t *tshift, bool *word32) {
    uint32_t tb = 1, cb = 1;
    while ((1ull << tb) <= static_cast<unsigned long long>(n)) ++tb;     // n < 2^tb
    while ((1ull << cb) <= static_cast<unsigned long long>(dmax)) ++cb;  // dmax < 2^cb
    *word32 = allow32 && tb + cb <= 32;
    *tshift = *word32 ? tb : 32;
}

uint32_t lds_threads_for(const fc_ctx *ctx, uint64_t trees, uint32_t lds_words) {
    if (ctx->lds_threads) return ctx->lds_threads;
    // A CU holds at most 2048 threads.  When LDS admits only one or two trees
    // per CU, each gets the widest workgroup; otherwise narrow the workgroups
    // until the CUs hold as many trees as there are (per CU) or LDS admits.
    const size_t per_tree = 4u * static_cast<size_t>(lds_words) + kLdsStaticBytes;
    const uint64_t fit_lds = ctx->max_lds / per_tree;
    if (fit_lds <= 2) return 1024u;
    const uint64_t per_cu = std::min<uint64_t>((trees + ctx->cu_count - 1) / ctx->cu_count, fit_lds);
    uint32_t t = 1024u;
    while (t > 256u && 2048u / t < per_cu) t /= 2;
    return t;
}

int begin(fc_ctx *ctx) {
    if (!ctx) return FC_ERR_ARG;
    ctx->last_error.clear();
    FC_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    return FC_OK;
}

}  // namespace fc_host

using namespace fc_host;

extern "C" {

int fc_create(fc_ctx **out, int hip_device, void *hip_stream) {
    if (!out) return FC_ERR_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
        (void)hipGetLastError();
        return FC_ERR_HIP;
    }
    if (hip_device < 0 || hip_device >= count) return FC_ERR_ARG;
    if (hipSetDevice(hip_device) != hipSuccess) return FC_ERR_HIP;
    fc_ctx *ctx = new fc_ctx();
    ctx->device = hip_device;
    {
        // the static scratch of fc_sample_noalloc on this device (a failure here
        // only disables that entry point; it reports the error)
        hipError_t se = hipSuccess;
        (void)scratch_of(hip_device, &se);
    }
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    if (hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess ||
        hipEventCreate(&ctx->evm) != hipSuccess ||
        ensure(ctx, ctx->small, sizeof(Small), "counters") != FC_OK) {
        fc_destroy(ctx);
        return FC_ERR_HIP;
    }
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    const uint32_t gib = env_u32("FC_STATE_GIB", 0);
    ctx->state_budget = gib ? static_cast<size_t>(gib) << 30
                            : std::min<size_t>(free_b / 4, static_cast<size_t>(48) << 30);
    ctx->lanes_per_wave = env_u32("FC_LANES_PER_WAVE", 64);
    ctx->max_slots = env_u32("FC_MAX_SLOTS", 0);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device) == hipSuccess &&
        cus > 0)
        ctx->cu_count = static_cast<uint32_t>(cus);
    int wclk = 0;
    if (hipDeviceGetAttribute(&wclk, hipDeviceAttributeWallClockRate, hip_device) == hipSuccess &&
        wclk > 0)
        ctx->wall_khz = wclk;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, hip_device) ==
            hipSuccess && lds > 0)
        ctx->max_lds = static_cast<size_t>(lds);
    // dynamic LDS: allow the workgroup kernels up to the device limit once;
    // each launch passes what it uses
    if (fc::coop_set_lds_limit(ctx->max_lds - kLdsStaticBytes) != hipSuccess ||
        fc::lds_set_limit(ctx->max_lds - kLdsStaticBytes) != hipSuccess ||
        fc::hyb_set_limit(ctx->max_lds - kLdsStaticBytes) != hipSuccess ||
        fc::tile_set_limit(ctx->max_lds - kLdsStaticBytes) != hipSuccess) {
        (void)hipGetLastError();
        fc_destroy(ctx);
        return FC_ERR_HIP;
    }
    ctx->coop_threads = env_u32("FC_COOP_THREADS", 512);
    if (ctx->coop_threads < 64 || ctx->coop_threads > 512 || ctx->coop_threads % 64)
        ctx->coop_threads = 512;
    ctx->coop_wg_per_cu = std::max<uint32_t>(1, env_u32("FC_COOP_WG_PER_CU", 3));
    ctx->coop_in_bits = env_u32("FC_COOP_IN_BITS", 1) != 0;
    ctx->coop_lds_counts = env_u32("FC_COOP_LDS_COUNTS", 1) != 0;
    ctx->lds_threads = env_u32("FC_LDS_THREADS", 0);
    if (ctx->lds_threads > 1024 || ctx->lds_threads % 64) ctx->lds_threads = 0;
    ctx->lds_wg_per_cu = std::min<uint32_t>(64, env_u32("FC_LDS_WG_PER_CU", 0));
    {
        const char *fs = std::getenv("FC_SAMPLER");
        if (fs && !std::strcmp(fs, "lane")) ctx->force_sampler = 1;
        if (fs && !std::strcmp(fs, "coop")) ctx->force_sampler = 2;
        if (fs && !std::strcmp(fs, "lds")) ctx->force_sampler = 3;
        if (fs && !std::strcmp(fs, "hyb")) ctx->force_sampler = 4;
        if (fs && !std::strcmp(fs, "tile")) ctx->force_sampler = 5;
    }
    *out = ctx;
    return FC_OK;
}

int fc_destroy(fc_ctx *ctx) {
    if (!ctx) return FC_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    for (DevBuf *b : {&ctx->state, &ctx->vrec, &ctx->row_ptr, &ctx->col_idx, &ctx->small,
                      &ctx->rtmp, &ctx->thr, &ctx->cword, &ctx->ckk, &ctx->clists, &ctx->clevels,
                      &ctx->cbits, &ctx->s_r64, &ctx->s_r, &ctx->s_z, &ctx->s_p, &ctx->s_q,
                      &ctx->s_d, &ctx->s_pa, &ctx->s_pb, &ctx->s_small, &ctx->rl_blk,
                      &ctx->rl_base, &ctx->rl_inv, &ctx->rl_orig, &ctx->rl_vrec, &ctx->rl_adj,
                      &ctx->iso, &ctx->corigt, &ctx->cpre, &ctx->weights, &ctx->wsum, &ctx->wthr,
                      &ctx->s_wdeg, &ctx->rk_key0, &ctx->rk_key1, &ctx->rk_val0, &ctx->rk_val1,
                      &ctx->rk_hist, &ctx->rk_thist, &ctx->rk_ra, &ctx->rk_rb, &ctx->rk_s, &ctx->g_mat,
                      &ctx->g_vec, &ctx->g_part, &ctx->g_taken, &ctx->g_scr, &ctx->t_ex, &ctx->t_exl,
                      &ctx->t_ecnt, &ctx->t_pc, &ctx->t_sc, &ctx->t_bl, &ctx->t_xb})
        if (b->ptr) (void)hipFree(b->ptr);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->evm) (void)hipEventDestroy(ctx->evm);
    delete ctx;
    return FC_OK;
}

int fc_set_stream(fc_ctx *ctx, void *hip_stream) {
    if (!ctx) return FC_ERR_ARG;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return FC_OK;
}

int fc_set_option(fc_ctx *ctx, const char *key, int64_t value) {
    if (!ctx || !key) return FC_ERR_ARG;
    const std::string k(key);
    if (k == "coop_threads") {
        if (value < 64 || value > 512 || value % 64) return set_err(ctx, FC_ERR_ARG, "coop_threads");
        ctx->coop_threads = static_cast<uint32_t>(value);
    } else if (k == "coop_wg_per_cu") {
        if (value < 1 || value > 64) return set_err(ctx, FC_ERR_ARG, "coop_wg_per_cu");
        ctx->coop_wg_per_cu = static_cast<uint32_t>(value);
    } else if (k == "coop_lds_bits") {
        if (value != 0 && value != 1) return set_err(ctx, FC_ERR_ARG, "coop_lds_bits");
        ctx->coop_lds_bits = value == 1;
    } else if (k == "coop_in_bits") {
        if (value != 0 && value != 1) return set_err(ctx, FC_ERR_ARG, "coop_in_bits");
        ctx->coop_in_bits = value == 1;
    } else if (k == "coop_word32") {
        if (value != 0 && value != 1) return set_err(ctx, FC_ERR_ARG, "coop_word32");
        ctx->coop_word32 = value == 1;
    } else if (k == "coop_lds_counts") {
        if (value != 0 && value != 1) return set_err(ctx, FC_ERR_ARG, "coop_lds_counts");
        ctx->coop_lds_counts = value == 1;
    } else if (k == "lds_threads") {
        if (value < 0 || value > 1024 || value % 64) return set_err(ctx, FC_ERR_ARG, "lds_threads");
        ctx->lds_threads = static_cast<uint32_t>(value);
    } else if (k == "lds_wg_per_cu") {
        if (value < 0 || value > 64) return set_err(ctx, FC_ERR_ARG, "lds_wg_per_cu");
        ctx->lds_wg_per_cu = static_cast<uint32_t>(value);
    } else if (k == "lds_lean") {
        if (value < 0 || value > 1) return set_err(ctx, FC_ERR_ARG, "lds_lean must be 0 or 1");
        ctx->lds_lean = static_cast<uint32_t>(value);
    } else if (k == "lds_repop") {
        if (value < 0 || value > 3) return set_err(ctx, FC_ERR_ARG, "lds_repop must be 0, 1, 2 or 3");
        ctx->lds_repop = static_cast<uint32_t>(value);
    } else if (k == "coop_repop") {
        if (value < 0 || value > 2) return set_err(ctx, FC_ERR_ARG, "coop_repop must be 0, 1 or 2");
        ctx->coop_repop = static_cast<uint32_t>(value);
    } else if (k == "kendall_pairs") {
        if (value < 0 || value > 1) return set_err(ctx, FC_ERR_ARG, "kendall_pairs must be 0 or 1");
        ctx->kendall_pairs = value != 0;
    } else if (k == "predraw_mib") {
        if (value < 0 || value > (int64_t(1) << 22)) return set_err(ctx, FC_ERR_ARG, "predraw_mib");
        ctx->predraw_mib = static_cast<uint32_t>(value);
    } else if (k == "hyb_hot_cap") {
        if (value < 0 || value > 0x7FFFFFFF) return set_err(ctx, FC_ERR_ARG, "hyb_hot_cap");
        ctx->hyb_hot_cap = static_cast<uint32_t>(value);
    } else if (k == "max_draws") {
        if (value < 0 || value > 0x7FFFFFFF) return set_err(ctx, FC_ERR_ARG, "max_draws");
        ctx->max_draws = static_cast<uint32_t>(value);
    } else if (k == "phase_timing") {
        if (value != 0 && value != 1) return set_err(ctx, FC_ERR_ARG, "phase_timing");
        ctx->phase_timing = value == 1;
    } else if (k == "lanes_per_wave") {
        if (value < 1 || value > 64) return set_err(ctx, FC_ERR_ARG, "lanes_per_wave");
        ctx->lanes_per_wave = static_cast<uint32_t>(value);
    } else if (k == "max_slots") {
        if (value < 0 || value > 0x7FFFFFFF) return set_err(ctx, FC_ERR_ARG, "max_slots");
        ctx->max_slots = static_cast<uint32_t>(value);
    } else if (k == "tile_size") {
        if (value < 0 || value > fc::kTileMax || value % 64)
            return set_err(ctx, FC_ERR_ARG, "tile_size must be 0 or a multiple of 64 up to 32704");
        ctx->tile_size = static_cast<uint32_t>(value);
    } else if (k == "tile_cross_permille") {
        if (value < 0 || value > 1000) return set_err(ctx, FC_ERR_ARG, "tile_cross_permille");
        ctx->tile_cross_permille = static_cast<uint32_t>(value);
    } else if (k == "tile_bits_lds") {
        if (value < 0 || value > 1) return set_err(ctx, FC_ERR_ARG, "tile_bits_lds must be 0 or 1");
        ctx->tile_bits_lds = static_cast<uint32_t>(value);
    } else if (k == "tile_repop") {
        if (value < 0 || value > 2) return set_err(ctx, FC_ERR_ARG, "tile_repop must be 0, 1 or 2");
        ctx->tile_repop = static_cast<uint32_t>(value);
    } else if (k == "tile_threads") {
        if (value < 64 || value > 1024 || value % 64) return set_err(ctx, FC_ERR_ARG, "tile_threads");
        ctx->tile_threads = static_cast<uint32_t>(value);
    } else {
        return set_err(ctx, FC_ERR_ARG, "unknown option " + k);
    }
    return FC_OK;
}

int fc_tau(int64_t m, int64_t n, double eps, double delta, double kappa, uint32_t *tau_out) {
    if (!tau_out) return FC_ERR_ARG;
    *tau_out = 0;
    if (!(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 1.0) ||
        !(kappa >= 0.0 && kappa < 1.0) || n < 1 || m < 0)
        return FC_ERR_ARG;
    // Hoeffding with a union bound over max(m, n) estimates:
    // 2 max(m, n) exp(-2 tau ((1 - kappa) eps)^2) <= delta
    const double events = static_cast<double>(std::max(m, n));
    const double e1 = (1.0 - kappa) * eps;
    const double t = std::ceil(std::log(2.0 * events / delta) / (2.0 * e1 * e1));
    if (!(t >= 1.0) || t > 4294967295.0) return FC_ERR_ARG;
    *tau_out = static_cast<uint32_t>(t);
    return FC_OK;
}

int fc_thresholds(fc_ctx *ctx, double alpha, int32_t d_max, uint64_t *out) {
    int rc = begin(ctx);
    if (rc) return rc;
    if (!out || d_max < 0 || !valid_alpha(alpha))
        return set_err(ctx, FC_ERR_ARG, "need out != NULL, d_max >= 0, alpha > 0");
    const size_t bytes = sizeof(uint64_t) * (static_cast<size_t>(d_max) + 1);
    if ((rc = ensure(ctx, ctx->thr, bytes, "threshold table"))) return rc;
    FC_HIP(ctx, fc::launch_thresholds(alpha, d_max, static_cast<unsigned long long *>(ctx->thr.ptr),
                                      ctx->stream), "thresholds launch");
    FC_HIP(ctx, hipMemcpyAsync(out, ctx->thr.ptr, bytes, hipMemcpyDeviceToHost, ctx->stream),
           "copy thresholds");
    FC_HIP(ctx, hipStreamSynchronize(ctx->stream), "thresholds");
    return FC_OK;
}

int fc_sample(fc_ctx *ctx, const fc_graph *g, const fc_params *params, uint32_t tree_begin,
              uint32_t tree_count, uint32_t *root_counts, uint64_t *visit_counts,
              uint64_t *tree_digests, uint64_t *tree_steps, int32_t *parents,
              uint32_t *tree_visits, fc_stats *stats) {
    const double t0 = now_ms();
    int rc = begin(ctx);
    if (rc) return rc;
    if ((rc = check_params(ctx, params))) return rc;
    if (!root_counts && g && g->n > 0) return set_err(ctx, FC_ERR_ARG, "root_counts is NULL");
    if (static_cast<uint64_t>(tree_begin) + tree_count > 0x100000000ull)
        return set_err(ctx, FC_ERR_ARG, "tree ids must stay below 2^32");
    GraphView gv;
    if ((rc = prepare_graph(ctx, g, params->flags & FC_FLAG_TRUSTED_GRAPH, &gv))) return rc;
    rc = run_sampler(ctx, gv, params, tree_begin, tree_count, root_counts, visit_counts,
                     tree_digests, tree_steps, parents, tree_visits, stats);
    if (stats) stats->ms_total = now_ms() - t0;
    return rc;
}

int fc_sample_noalloc(fc_ctx *ctx, const fc_graph *g, const fc_params *params,
                      uint32_t tree_begin, uint32_t tree_count, uint32_t *root_counts,
                      uint64_t *visit_counts, uint64_t *tree_digests, uint64_t *tree_steps,
                      int32_t *parents, uint32_t *tree_visits, fc_stats *stats) {
    const double t0 = now_ms();
    int rc = begin(ctx);
    if (rc) return rc;
    if ((rc = check_params(ctx, params))) return rc;
    if ((rc = check_graph_args(ctx, g))) return rc;
    if (g->mem != FC_MEM_DEVICE)
        return set_err(ctx, FC_ERR_ARG, "fc_sample_noalloc needs a device-resident graph");
    if (!root_counts && g->n > 0) return set_err(ctx, FC_ERR_ARG, "root_counts is NULL");
    if (static_cast<uint64_t>(tree_begin) + tree_count > 0x100000000ull)
        return set_err(ctx, FC_ERR_ARG, "tree ids must stay below 2^32");
    hipError_t se = hipSuccess;
    void *base = scratch_of(ctx->device, &se);
    if (!base)
        return set_err(ctx, FC_ERR_HIP, std::string("no static scratch on this device: ") +
                                             hipGetErrorString(se));
    // The call runs the ordinary sampling path on a shadow of the context whose
    // buffers all come from the static scratch (ensure() carves them and never
    // allocates); the shadow shares the context's stream, events and options.
    fc_ctx sh;
    sh.device = ctx->device;
    sh.stream = ctx->stream;
    sh.ev0 = ctx->ev0;
    sh.ev1 = ctx->ev1;
    sh.evm = ctx->evm;
    sh.lanes_per_wave = ctx->lanes_per_wave;
    sh.max_slots = ctx->max_slots;
    sh.cu_count = ctx->cu_count;
    sh.max_lds = ctx->max_lds;
    sh.coop_threads = ctx->coop_threads;
    sh.coop_wg_per_cu = ctx->coop_wg_per_cu;
    sh.force_sampler = ctx->force_sampler;
    sh.coop_lds_bits = ctx->coop_lds_bits;
    sh.coop_word32 = ctx->coop_word32;
    sh.coop_in_bits = ctx->coop_in_bits;
    sh.phase_timing = ctx->phase_timing;
    sh.max_draws = ctx->max_draws;
    sh.hyb_hot_cap = ctx->hyb_hot_cap;
    sh.coop_lds_counts = ctx->coop_lds_counts;
    sh.lds_threads = ctx->lds_threads;
    sh.lds_wg_per_cu = ctx->lds_wg_per_cu;
    sh.predraw_mib = 0;  // every tree draws its own first arrows: no per-call pre-draw array
    sh.kendall_pairs = ctx->kendall_pairs;
    sh.lds_repop = ctx->lds_repop;
    sh.lds_lean = ctx->lds_lean;
    sh.coop_repop = ctx->coop_repop;
    sh.tile_size = ctx->tile_size;
    sh.tile_cross_permille = ctx->tile_cross_permille;
    sh.tile_threads = ctx->tile_threads;
    sh.tile_repop = ctx->tile_repop;
    sh.tile_bits_lds = ctx->tile_bits_lds;
    sh.wall_khz = ctx->wall_khz;
    sh.arena = static_cast<char *>(base);
    sh.arena_size = kStaticScratchBytes;
    sh.arena_off = 0;
    GraphView gv;
    if ((rc = ensure(&sh, sh.small, sizeof(Small), "counters")) ||
        (rc = prepare_graph(&sh, g, params->flags & FC_FLAG_TRUSTED_GRAPH, &gv)) ||
        (rc = run_sampler(&sh, gv, params, tree_begin, tree_count, root_counts, visit_counts,
                          tree_digests, tree_steps, parents, tree_visits, stats))) {
        ctx->last_error = "fc_sample_noalloc: " + sh.last_error;
        return rc;
    }
    if (stats) stats->ms_total = now_ms() - t0;
    return FC_OK;
}

static int estimate_common(fc_ctx *ctx, const fc_graph *g, const fc_params *params,
                           double *diag, double *farness, double *closeness,
                           uint32_t *root_counts_out, fc_stats *stats) {
    const double t0 = now_ms();
    int rc = begin(ctx);
    if (rc) return rc;
    if ((rc = check_params(ctx, params))) return rc;
    if (params->estimator != FC_EST_DIRECT && params->estimator != FC_EST_ALG1_LITERAL)
        return set_err(ctx, FC_ERR_ARG, "unknown estimator");
    GraphView gv;
    if ((rc = check_graph_args(ctx, g))) return rc;
    if (g->n == 0) {  // nothing to estimate
        if (stats) std::memset(stats, 0, sizeof(*stats));
        return FC_OK;
    }
    uint32_t tau = 0;
    {
        GraphView tmp;
        tmp.n = g->n;
        tmp.nnz = g->nnz;
        if ((rc = tau_for(ctx, params, tmp, &tau))) return rc;
    }
    if ((rc = prepare_graph(ctx, g, params->flags & FC_FLAG_TRUSTED_GRAPH, &gv))) return rc;
    uint32_t *R = root_counts_out;
    if (!R) {
        if ((rc = ensure(ctx, ctx->rtmp, sizeof(uint32_t) * static_cast<size_t>(gv.n), "root counts")))
            return rc;
        R = static_cast<uint32_t *>(ctx->rtmp.ptr);
    }
    if (gv.n)
        FC_HIP(ctx, hipMemsetAsync(R, 0, sizeof(uint32_t) * static_cast<size_t>(gv.n), ctx->stream),
               "memset R");
    if ((rc = run_sampler(ctx, gv, params, 0, tau, R, nullptr, nullptr, nullptr, nullptr, nullptr,
                          stats)))
        return rc;
    Small *sm = static_cast<Small *>(ctx->small.ptr);
    FC_HIP(ctx, hipMemsetAsync(&sm->sum, 0, sizeof(unsigned long long), ctx->stream), "memset sum");
    FC_HIP(ctx, fc::launch_sum_u32(R, gv.n, &sm->sum, ctx->stream), "sum launch");
    FC_HIP(ctx, fc::launch_estimate(R, gv.n, tau, params->estimator == FC_EST_ALG1_LITERAL, &sm->sum,
                                    diag, farness, closeness, ctx->stream), "estimate launch");
    FC_HIP(ctx, hipStreamSynchronize(ctx->stream), "estimate");
    if (stats) stats->ms_total = now_ms() - t0;
    return FC_OK;
}

int fc_diag_estimate(fc_ctx *ctx, const fc_graph *g, const fc_params *params, double *diag_out,
                     uint32_t *root_counts_out, fc_stats *stats) {
    if (ctx && !diag_out && g && g->n > 0) return set_err(ctx, FC_ERR_ARG, "diag_out is NULL");
    return estimate_common(ctx, g, params, diag_out, nullptr, nullptr, root_counts_out, stats);
}

int fc_farness(fc_ctx *ctx, const fc_graph *g, const fc_params *params, double *farness_out,
               double *closeness_out, double *diag_out, uint32_t *root_counts_out,
               fc_stats *stats) {
    if (ctx && !farness_out && g && g->n > 0) return set_err(ctx, FC_ERR_ARG, "farness_out is NULL");
    return estimate_common(ctx, g, params, diag_out, farness_out, closeness_out, root_counts_out,
                           stats);
}

int fc_probe_random_access(fc_ctx *ctx, uint64_t footprint_bytes, int32_t atomics,
                           double *rate_out) {
    int rc = begin(ctx);
    if (rc) return rc;
    if (!rate_out || footprint_bytes < 4096 || (atomics != 0 && atomics != 1))
        return set_err(ctx, FC_ERR_ARG, "need rate_out, footprint >= 4 KiB, atomics 0 or 1");
    uint64_t words = 1;
    while (words * 2 * 4 <= footprint_bytes && words < (1ull << 31)) words *= 2;
    DevBuf buf;
    if ((rc = ensure(ctx, buf, 4 * words + 64, "probe footprint"))) return rc;
    uint32_t *data = static_cast<uint32_t *>(buf.ptr);
    auto done = [&](int code) {
        (void)hipFree(buf.ptr);
        return code;
    };
    if (hipMemsetAsync(data, 0, 4 * words + 64, ctx->stream) != hipSuccess)
        return done(set_err(ctx, FC_ERR_HIP, "probe memset"));
    const uint32_t blocks = ctx->cu_count * 32, iters = 64;
    const double accesses = static_cast<double>(blocks) * 256.0 * iters * 8.0;
    uint32_t *sink = data + words;
    hipError_t e = fc::launch_random_access(data, static_cast<uint32_t>(words), 4, atomics, blocks,
                                            sink, ctx->stream);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(ctx->ev0, ctx->stream);
    if (e == hipSuccess)
        e = fc::launch_random_access(data, static_cast<uint32_t>(words), iters, atomics, blocks, sink,
                                     ctx->stream);
    if (e == hipSuccess) e = hipEventRecord(ctx->ev1, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return done(hip_fail(ctx, e, "probe"));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    *rate_out = ms > 0.f ? accesses / (ms / 1000.0) : 0.0;
    return done(FC_OK);
}

const char *fc_error_string(int code) {
    switch (code) {
        case FC_OK: return "ok";
        case FC_ERR_ARG: return "invalid argument";
        case FC_ERR_GRAPH: return "graph violates the input contract (simple, symmetric, sorted CSR)";
        case FC_ERR_NOMEM: return "device memory allocation failed";
        case FC_ERR_HIP: return "HIP runtime error";
        case FC_ERR_UNSUPPORTED: return "unsupported size";
        case FC_ERR_OVERFLOW: return "visit counter overflow";
        default: return "unknown error code";
    }
}

const char *fc_last_error(fc_ctx *ctx) {
    if (!ctx) return "no context";
    return ctx->last_error.c_str();
}

}  // extern "C"
