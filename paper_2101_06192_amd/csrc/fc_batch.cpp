// Batches of sampling jobs (fc_batch_create / fc_batch_run / fc_batch_destroy).
//
// A batch turns many (graph, alpha, tree range) jobs into one list of work
// items (trees), ordered largest graph first so that the longest trees start
// early, and samples them with the workgroup-per-tree kernel in a single
// persistent launch whose workgroups pull items from a device queue.  The
// per-slot scratch is sized for the largest graph.  Everything that does not
// change between runs (validation, vertex records, item order, scratch,
// launch shape) happens once in fc_batch_create; a run replays a captured
// HIP graph made of two fill kernels (counters, epoch-tagged draw counts)
// and the sampling kernel.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "fc_internal.hpp"

using namespace fc_host;

struct fc_batch {
    fc_ctx *ctx = nullptr;
    std::vector<fc_job> jobs;
    uint64_t seed = 0;
    int32_t flags = 0;
    DevBuf vrec, jobtab, item_job, word, kk, lists, levels, bits, small, dmax, scratch_r;
    DevBuf rl_blk, rl_base, rl_bounds, rl_inv, rl_orig, rl_adj, rl_vrec;  // degree-class relabelling
    uint32_t n_max = 0, item_count = 0, slots = 0, threads = 512, wg_per_cu = 4;
    size_t ntab = 0;  // entries of the device job table (jobs that have trees)
    bool lds_bits = false, in_bits = false, word32 = true;
    bool use_lds = false;     // LDS-counter kernel
    uint32_t lds_words = 0;   // its dynamic LDS (largest graph of the batch)
    size_t kk_words = 0;
    fc::CoopArgs args{};
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev_in = nullptr, ev0 = nullptr, ev1 = nullptr;
};

namespace {

int free_batch(fc_batch *b) {
    if (!b) return FC_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (DevBuf *d : {&b->vrec, &b->jobtab, &b->item_job, &b->word, &b->kk, &b->lists, &b->levels,
                      &b->bits, &b->small, &b->dmax, &b->scratch_r, &b->rl_blk, &b->rl_base,
                      &b->rl_bounds, &b->rl_inv, &b->rl_orig, &b->rl_adj, &b->rl_vrec})
        if (d->ptr) (void)hipFree(d->ptr);
    for (hipEvent_t e : {b->ev_in, b->ev0, b->ev1})
        if (e) (void)hipEventDestroy(e);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return FC_OK;
}

// Enqueue one run on `stream`: reset counters and draw-count epochs, then sample.
hipError_t enqueue_run(fc_batch *b, const fc::CoopArgs &a, uint32_t threads, hipStream_t stream) {
    hipError_t e = fc::launch_fill_u64(static_cast<unsigned long long *>(b->small.ptr),
                                       sizeof(Small) / 8, 0ull, stream);
    if (e != hipSuccess) return e;
    if (b->use_lds) return fc::launch_wilson_lds(a, threads, b->lds_words, stream);
    e = fc::launch_fill_u64(static_cast<unsigned long long *>(b->kk.ptr), b->kk_words, 0ull, stream);
    if (e != hipSuccess) return e;
    return fc::launch_wilson_coop(a, threads, b->lds_bits, b->in_bits, b->word32, stream);
}

// Size the scratch for `slots` workgroups and point the launch arguments at it.
int size_scratch(fc_batch *b, uint32_t slots) {
    fc_ctx *ctx = b->ctx;
    int rc;
    const size_t n = b->n_max, nwords = (n + 31) / 32;
    const size_t wbytes = b->word32 && !b->use_lds ? 4 : 8;
    if ((rc = ensure(ctx, b->word, wbytes * n * slots, "batch tree words"))) return rc;
    if (!b->use_lds && (rc = ensure(ctx, b->kk, 8 * n * slots, "batch draw counts"))) return rc;
    if ((rc = ensure(ctx, b->lists, 24 * n * slots, "batch lists"))) return rc;
    if ((rc = ensure(ctx, b->levels, 4 * (n + 2) * slots, "batch levels"))) return rc;
    if (!b->use_lds && !b->lds_bits &&
        (rc = ensure(ctx, b->bits, 4 * nwords * slots, "batch bitmap")))
        return rc;
    b->kk_words = n * slots;
    b->slots = slots;
    fc::CoopArgs &a = b->args;
    a.word = b->word.ptr;
    a.kk = b->use_lds ? nullptr : static_cast<uint64_t *>(b->kk.ptr);
    a.lists = static_cast<uint64_t *>(b->lists.ptr);
    a.levels = static_cast<uint32_t *>(b->levels.ptr);
    a.bits = b->lds_bits || b->use_lds ? nullptr : static_cast<uint32_t *>(b->bits.ptr);
    a.slots = slots;
    return FC_OK;
}

uint32_t slots_for(fc_batch *b, uint32_t threads, uint32_t wg_per_cu) {
    const size_t n = b->n_max;
    const int fit = b->use_lds ? fc::lds_max_active(threads, b->lds_words)
                               : fc::coop_max_active(threads, b->lds_bits, b->in_bits, b->word32,
                                                     b->n_max);
    if (fit > 0) wg_per_cu = std::min<uint32_t>(wg_per_cu, static_cast<uint32_t>(fit));
    const size_t per_slot = b->use_lds ? (8 + 24 + 4) * n + 8
                                       : ((b->word32 ? 4 : 8) + 8 + 24 + 4) * n + 8 +
                                             (b->lds_bits ? 0 : 4 * ((n + 31) / 32));
    size_t slots = std::max<size_t>(1, b->ctx->state_budget / per_slot);
    slots = std::min<size_t>(slots, static_cast<size_t>(b->ctx->cu_count) * wg_per_cu);
    slots = std::min<size_t>(slots, b->item_count);
    return static_cast<uint32_t>(std::max<size_t>(slots, 1));
}

// Launch-shape autotuning on a prefix of the work items with throw-away
// outputs: results never depend on the shape, only the time does.
int autotune(fc_batch *b) {
    fc_ctx *ctx = b->ctx;
    int rc;
    static const uint32_t cand_coop[][2] = {{256, 3}, {256, 6}, {512, 2}, {512, 3}, {128, 12}};
    static const uint32_t cand_lds[][2] = {{256, 64}, {512, 64}, {1024, 64}, {256, 4}, {512, 2}};
    std::vector<std::array<uint32_t, 2>> cand;
    if (b->use_lds)
        for (const auto &c : cand_lds) cand.push_back({c[0], c[1]});
    else
        for (const auto &c : cand_coop) cand.push_back({c[0], c[1]});
    // throw-away job table: same graphs and records, outputs into one scratch R
    std::vector<fc::CoopJob> tab(b->ntab);
    FC_HIP(ctx, hipMemcpy(tab.data(), b->jobtab.ptr, sizeof(fc::CoopJob) * tab.size(),
                          hipMemcpyDeviceToHost), "read job table");
    if ((rc = ensure(ctx, b->scratch_r, 4 * static_cast<size_t>(b->n_max), "tuning outputs"))) return rc;
    DevBuf tmp_tab;
    for (auto &j : tab) {
        j.root_counts = static_cast<uint32_t *>(b->scratch_r.ptr);
        j.visit_counts = nullptr;
        j.tree_digests = nullptr;
        j.tree_steps = nullptr;
        j.parents = nullptr;
        j.tree_visits = nullptr;
    }
    if ((rc = ensure(ctx, tmp_tab, sizeof(fc::CoopJob) * tab.size(), "tuning job table"))) return rc;
    FC_HIP(ctx, hipMemcpy(tmp_tab.ptr, tab.data(), sizeof(fc::CoopJob) * tab.size(),
                          hipMemcpyHostToDevice), "write tuning table");
    const uint32_t prefix = std::min<uint32_t>(b->item_count,
                                               std::max<uint32_t>(b->item_count / 16, 4096));
    float best = 1e30f;
    uint32_t best_t = b->threads, best_w = b->wg_per_cu;
    for (const auto &c : cand) {
        const uint32_t slots = slots_for(b, c[0], c[1]);
        if ((rc = size_scratch(b, slots))) break;
        fc::CoopArgs a = b->args;
        a.jobs = static_cast<const fc::CoopJob *>(tmp_tab.ptr);
        a.item_count = prefix;
        FC_HIP(ctx, hipEventRecord(b->ev0, b->stream), "event");
        FC_HIP(ctx, enqueue_run(b, a, c[0], b->stream), "tuning launch");
        FC_HIP(ctx, hipEventRecord(b->ev1, b->stream), "event");
        FC_HIP(ctx, hipStreamSynchronize(b->stream), "tuning run");
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, b->ev0, b->ev1);
        Small sm;
        FC_HIP(ctx, hipMemcpy(&sm, b->small.ptr, sizeof(sm), hipMemcpyDeviceToHost), "read counters");
        if (sm.totals.error) {
            rc = set_err(ctx, FC_ERR_HIP, "autotuning run reported a kernel error");
            break;
        }
        if (ms < best) {
            best = ms;
            best_t = c[0];
            best_w = c[1];
        }
    }
    if (tmp_tab.ptr) (void)hipFree(tmp_tab.ptr);
    if (rc) return rc;
    b->threads = best_t;
    b->wg_per_cu = best_w;
    return FC_OK;
}

}  // namespace

extern "C" {

int fc_batch_create(fc_ctx *ctx, const fc_job *jobs, int32_t n_jobs, uint64_t seed, int32_t flags,
                    fc_batch **out) {
    int rc = begin(ctx);
    if (rc) return rc;
    if (!out || n_jobs < 0 || (n_jobs > 0 && !jobs))
        return set_err(ctx, FC_ERR_ARG, "need out != NULL and a job array");
    *out = nullptr;
    uint64_t items = 0;
    uint32_t n_max = 0;
    for (int32_t i = 0; i < n_jobs; ++i) {
        const fc_job &j = jobs[i];
        if ((rc = check_graph_args(ctx, &j.graph))) return rc;
        if (j.graph.mem != FC_MEM_DEVICE)
            return set_err(ctx, FC_ERR_ARG, "batch jobs need device graphs (FC_MEM_DEVICE)");
        if (!valid_alpha(j.alpha)) return set_err(ctx, FC_ERR_ARG, "job alpha must be finite and > 0");
        if (j.graph.n > 0 && j.tree_count > 0 && !j.root_counts)
            return set_err(ctx, FC_ERR_ARG, "job root_counts is NULL");
        if (static_cast<uint64_t>(j.tree_begin) + j.tree_count > 0x100000000ull)
            return set_err(ctx, FC_ERR_ARG, "job tree ids must stay below 2^32");
        if (j.graph.n > 0) {
            items += j.tree_count;
            n_max = std::max<uint32_t>(n_max, static_cast<uint32_t>(j.graph.n));
        }
    }
    if (items >= 0xFFFFFFFFull) return set_err(ctx, FC_ERR_ARG, "more than 2^32 - 1 trees in a batch");

    fc_batch *b = new fc_batch();
    b->ctx = ctx;
    b->jobs.assign(jobs, jobs + n_jobs);
    b->seed = seed;
    b->flags = flags;
    b->n_max = n_max;
    b->item_count = static_cast<uint32_t>(items);
    b->threads = ctx->coop_threads;
    b->wg_per_cu = ctx->coop_wg_per_cu;
    auto fail = [&](int code) {
        free_batch(b);
        return code;
    };
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&b->ev_in) != hipSuccess || hipEventCreate(&b->ev0) != hipSuccess ||
        hipEventCreate(&b->ev1) != hipSuccess)
        return fail(set_err(ctx, FC_ERR_HIP, "creating the batch stream and events failed"));
    if ((rc = ensure(ctx, b->small, sizeof(Small), "batch counters"))) return fail(rc);
    if (items == 0) {
        *out = b;
        return FC_OK;
    }

    // validate each distinct graph once
    if (!(flags & FC_FLAG_TRUSTED_GRAPH)) {
        std::vector<const int32_t *> seen;
        for (const fc_job &j : b->jobs) {
            if (std::find(seen.begin(), seen.end(), j.graph.row_ptr) != seen.end()) continue;
            seen.push_back(j.graph.row_ptr);
            GraphView gv;
            if ((rc = prepare_graph(ctx, &j.graph, false, &gv))) return fail(rc);
        }
    }

    // work order: jobs with trees, largest graph first (stable)
    std::vector<int32_t> order;
    for (int32_t i = 0; i < n_jobs; ++i)
        if (b->jobs[i].graph.n > 0 && b->jobs[i].tree_count > 0) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return b->jobs[x].graph.n > b->jobs[y].graph.n;
    });

    // vertex records of every job's G* and each graph's maximum degree
    std::vector<size_t> voff(order.size());
    size_t vtotal = 0;
    for (size_t k = 0; k < order.size(); ++k) {
        voff[k] = vtotal;
        vtotal += static_cast<size_t>(b->jobs[order[k]].graph.n);
    }
    if ((rc = ensure(ctx, b->vrec, sizeof(fc::VRec) * vtotal, "batch vertex records"))) return fail(rc);
    if ((rc = ensure(ctx, b->dmax, 4 * order.size(), "batch degrees"))) return fail(rc);
    FC_HIP(ctx, hipMemsetAsync(b->dmax.ptr, 0, 4 * order.size(), b->stream), "memset degrees");
    fc::VRec *vrec = static_cast<fc::VRec *>(b->vrec.ptr);
    unsigned int *dmax_d = static_cast<unsigned int *>(b->dmax.ptr);
    for (size_t k = 0; k < order.size(); ++k) {
        const fc_job &j = b->jobs[order[k]];
        FC_HIP(ctx, fc::launch_build_vrec(j.graph.row_ptr, j.graph.n, j.alpha, vrec + voff[k],
                                          dmax_d + k, b->stream), "build_vrec");
    }
    // degree classes of each distinct graph, for the LDS-counter kernel
    struct GInfo {
        const int32_t *rp, *ci;
        uint32_t n;
        int64_t nnz;
        size_t off_n, off_e, off_b;
    };
    std::vector<GInfo> gs;
    std::vector<uint32_t> gof(order.size());
    size_t tn = 0, te = 0, tb = 0;
    for (size_t k = 0; k < order.size(); ++k) {
        const fc_graph &gr = b->jobs[order[k]].graph;
        size_t f = 0;
        while (f < gs.size() && !(gs[f].rp == gr.row_ptr && gs[f].ci == gr.col_idx &&
                                  gs[f].n == static_cast<uint32_t>(gr.n)))
            ++f;
        if (f == gs.size()) {
            gs.push_back({gr.row_ptr, gr.col_idx, static_cast<uint32_t>(gr.n), gr.nnz, tn, te, tb});
            tn += static_cast<size_t>(gr.n);
            te += static_cast<size_t>(gr.nnz);
            tb += fc::relabel_blocks(static_cast<uint32_t>(gr.n));
        }
        gof[k] = static_cast<uint32_t>(f);
    }
    const bool try_lds = ctx->coop_lds_counts && !order.empty() &&
                         n_max < (1u << fc::kRelabelIdBits) &&
                         static_cast<size_t>(n_max) * 5u <= 8u * ctx->max_lds;
    std::vector<unsigned int> bounds(4 * gs.size(), 0u);
    if (try_lds) {
        if ((rc = ensure(ctx, b->rl_blk, 16 * tb, "class counts")) ||
            (rc = ensure(ctx, b->rl_base, 16 * tb, "class offsets")) ||
            (rc = ensure(ctx, b->rl_bounds, 16 * gs.size(), "class bounds")))
            return fail(rc);
        uint32_t *blk = static_cast<uint32_t *>(b->rl_blk.ptr);
        uint32_t *base = static_cast<uint32_t *>(b->rl_base.ptr);
        uint32_t *bnd = static_cast<uint32_t *>(b->rl_bounds.ptr);
        for (size_t f = 0; f < gs.size(); ++f)
            FC_HIP(ctx, fc::launch_class_bounds(gs[f].rp, gs[f].n, blk + 4 * gs[f].off_b,
                                                base + 4 * gs[f].off_b, bnd + 4 * f, b->stream),
                   "class bounds");
        FC_HIP(ctx, hipMemcpyAsync(bounds.data(), bnd, 16 * gs.size(), hipMemcpyDeviceToHost,
                                   b->stream), "copy class bounds");
    }
    std::vector<unsigned int> dmax(order.size());
    FC_HIP(ctx, hipMemcpyAsync(dmax.data(), dmax_d, 4 * order.size(), hipMemcpyDeviceToHost, b->stream),
           "copy degrees");
    FC_HIP(ctx, hipStreamSynchronize(b->stream), "batch preparation");
    if (try_lds) {
        uint32_t words = 0;
        for (size_t f = 0; f < gs.size(); ++f)
            words = std::max(words, fc::count_layout(gs[f].n, bounds[4 * f], bounds[4 * f + 1],
                                                     bounds[4 * f + 2]).words);
        b->use_lds = 4u * static_cast<size_t>(words) + kLdsStaticBytes <= ctx->max_lds;
        b->lds_words = words;
    }
    if (b->use_lds) {
        if ((rc = ensure(ctx, b->rl_inv, 4 * tn, "relabel inverse")) ||
            (rc = ensure(ctx, b->rl_orig, 4 * tn, "relabel ids")) ||
            (rc = ensure(ctx, b->rl_adj, 8 * te, "relabelled adjacency")) ||
            (rc = ensure(ctx, b->rl_vrec, sizeof(fc::VRec) * vtotal, "relabelled records")))
            return fail(rc);
        const uint32_t *base = static_cast<const uint32_t *>(b->rl_base.ptr);
        uint32_t *inv = static_cast<uint32_t *>(b->rl_inv.ptr);
        uint32_t *orig = static_cast<uint32_t *>(b->rl_orig.ptr);
        unsigned long long *adj = static_cast<unsigned long long *>(b->rl_adj.ptr);
        for (const GInfo &gi : gs)
            FC_HIP(ctx, fc::launch_relabel_graph(gi.rp, gi.ci, gi.n, gi.nnz, base + 4 * gi.off_b,
                                                 inv + gi.off_n, orig + gi.off_n, adj + gi.off_e,
                                                 b->stream), "relabel");
        fc::VRec *vr = static_cast<fc::VRec *>(b->rl_vrec.ptr);
        for (size_t k = 0; k < order.size(); ++k)
            FC_HIP(ctx, fc::launch_relabel_vrec(vrec + voff[k], inv + gs[gof[k]].off_n,
                                                static_cast<uint32_t>(b->jobs[order[k]].graph.n),
                                                vr + voff[k], b->stream), "relabel records");
        b->threads = lds_threads_for(ctx, b->item_count, b->lds_words);
        b->wg_per_cu = ctx->lds_wg_per_cu ? ctx->lds_wg_per_cu : 64u;
    }

    // one word width for the whole launch
    b->word32 = ctx->coop_word32;
    for (size_t k = 0; k < order.size(); ++k) {
        uint32_t ts;
        bool w32;
        word_layout(static_cast<uint32_t>(b->jobs[order[k]].graph.n), dmax[k], true, &ts, &w32);
        b->word32 = b->word32 && w32;
    }
    b->lds_bits = ctx->coop_lds_bits && fc::coop_lds_bytes(n_max) + 1024u <= ctx->max_lds;
    b->in_bits = b->lds_bits && ctx->coop_in_bits &&
                 2 * fc::coop_lds_bytes(n_max) + 1024u <= ctx->max_lds;

    // job table and item -> job map
    std::vector<fc::CoopJob> tab(order.size());
    std::vector<uint32_t> item_job(b->item_count);
    uint32_t first = 0;
    for (size_t k = 0; k < order.size(); ++k) {
        const fc_job &j = b->jobs[order[k]];
        fc::CoopJob &c = tab[k];
        std::memset(&c, 0, sizeof(c));
        c.vrec = vrec + voff[k];
        c.col_idx = j.graph.col_idx;
        c.n = static_cast<uint32_t>(j.graph.n);
        if (b->use_lds) {
            const GInfo &gi = gs[gof[k]];
            c.vrec = static_cast<const fc::VRec *>(b->rl_vrec.ptr) + voff[k];
            c.adj = static_cast<const unsigned long long *>(b->rl_adj.ptr) + gi.off_e;
            c.orig = static_cast<const uint32_t *>(b->rl_orig.ptr) + gi.off_n;
            c.n0 = bounds[4 * gof[k]];
            c.n1 = bounds[4 * gof[k] + 1];
            c.n2 = bounds[4 * gof[k] + 2];
        }
        bool w32;
        word_layout(c.n, dmax[k], b->word32, &c.tshift, &w32);
        c.stream_id = j.stream_id;
        c.tree_begin = j.tree_begin;
        c.first_item = first;
        const double cap = 256.0 * (static_cast<double>(j.graph.n) +
                                    j.alpha * static_cast<double>(j.graph.nnz)) + 1048576.0;
        c.step_cap = cap > 4.0e18 ? 4000000000000000000ull : static_cast<unsigned long long>(cap);
        c.root_counts = j.root_counts;
        c.tree_digests = reinterpret_cast<unsigned long long *>(j.tree_digests);
        std::fill(item_job.begin() + first, item_job.begin() + first + j.tree_count,
                  static_cast<uint32_t>(k));
        first += j.tree_count;
    }
    b->ntab = tab.size();
    if ((rc = ensure(ctx, b->jobtab, sizeof(fc::CoopJob) * tab.size(), "job table"))) return fail(rc);
    if ((rc = ensure(ctx, b->item_job, 4 * item_job.size(), "item map"))) return fail(rc);
    FC_HIP(ctx, hipMemcpyAsync(b->jobtab.ptr, tab.data(), sizeof(fc::CoopJob) * tab.size(),
                               hipMemcpyHostToDevice, b->stream), "copy job table");
    FC_HIP(ctx, hipMemcpyAsync(b->item_job.ptr, item_job.data(), 4 * item_job.size(),
                               hipMemcpyHostToDevice, b->stream), "copy item map");
    FC_HIP(ctx, hipStreamSynchronize(b->stream), "batch tables");

    fc::CoopArgs &a = b->args;
    std::memset(&a, 0, sizeof(a));
    a.n_max = n_max;
    a.item_count = b->item_count;
    a.key0 = static_cast<uint32_t>(seed);
    a.key1 = static_cast<uint32_t>(seed >> 32);
    a.max_rounds = 0x40000000u;
    a.k_limit = ctx->max_draws ? ctx->max_draws : b->use_lds ? 0xFFFFFFFFu : 0x7FFFFFFFu;
    Small *sm = static_cast<Small *>(b->small.ptr);
    a.queue = &sm->queue;
    a.totals = &sm->totals;
    a.phase_ticks = nullptr;
    a.jobs = static_cast<const fc::CoopJob *>(b->jobtab.ptr);
    a.item_job = static_cast<const uint32_t *>(b->item_job.ptr);
    if (b->use_lds) FC_HIP(ctx, fc::lds_set_limit(b->lds_words), "LDS limit");
    else FC_HIP(ctx, fc::coop_set_lds_limit(b->lds_bits, b->in_bits, b->word32, n_max), "coop LDS limit");

    if ((flags & FC_FLAG_AUTOTUNE) && (rc = autotune(b))) return fail(rc);
    if ((rc = size_scratch(b, slots_for(b, b->threads, b->wg_per_cu)))) return fail(rc);

    // capture the run: counter reset, epoch reset, sampling kernel
    FC_HIP(ctx, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    hipError_t ce = enqueue_run(b, b->args, b->threads, b->stream);
    hipError_t ee = hipStreamEndCapture(b->stream, &b->graph);
    if (ce != hipSuccess) return fail(hip_fail(ctx, ce, "capturing the batch launch"));
    if (ee != hipSuccess) return fail(hip_fail(ctx, ee, "end capture"));
    FC_HIP(ctx, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "instantiate graph");
    *out = b;
    return FC_OK;
}

int fc_batch_run(fc_batch *b, fc_stats *stats) {
    if (!b) return FC_ERR_ARG;
    fc_ctx *ctx = b->ctx;
    const double t0 = now_ms();
    int rc = begin(ctx);
    if (rc) return rc;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->tau = b->item_count;
        std::snprintf(stats->sampler, sizeof(stats->sampler), "%s:%ux%u",
                      b->use_lds ? "lbatch" : "batch", b->threads, b->wg_per_cu);
    }
    if (b->item_count == 0) return FC_OK;
    // order after the caller's earlier work on the context stream, and make the
    // context stream wait for the batch
    FC_HIP(ctx, hipEventRecord(b->ev_in, ctx->stream), "event");
    FC_HIP(ctx, hipStreamWaitEvent(b->stream, b->ev_in, 0), "wait");
    FC_HIP(ctx, hipEventRecord(b->ev0, b->stream), "event");
    FC_HIP(ctx, hipGraphLaunch(b->exec, b->stream), "graph launch");
    FC_HIP(ctx, hipEventRecord(b->ev1, b->stream), "event");
    Small sm;
    FC_HIP(ctx, hipMemcpyAsync(&sm, b->small.ptr, sizeof(sm), hipMemcpyDeviceToHost, b->stream),
           "copy counters");
    FC_HIP(ctx, hipStreamSynchronize(b->stream), "batch run");
    FC_HIP(ctx, hipStreamWaitEvent(ctx->stream, b->ev1, 0), "wait");
    if (sm.totals.error & fc::kErrStepCap)
        return set_err(ctx, FC_ERR_HIP, "a tree exceeded the step bound (internal fault)");
    if (sm.totals.error & fc::kErrVisitOverflow)
        return set_err(ctx, FC_ERR_OVERFLOW,
                       b->use_lds ? "a per-vertex draw count exceeded 2^28 - 1 (LDS counters)"
                                  : "a per-vertex visit counter exceeded 2^31 - 1");
    if (stats) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, b->ev0, b->ev1);
        stats->trees_in_flight = b->slots;
        stats->walk_steps = sm.totals.walk_steps;
        stats->roots = sm.totals.roots;
        stats->digest_sum = sm.totals.digest_sum;
        stats->ms_sample = ms;
        stats->ms_total = now_ms() - t0;
    }
    return FC_OK;
}

int fc_batch_destroy(fc_batch *b) { return free_batch(b); }

}  // extern "C"
