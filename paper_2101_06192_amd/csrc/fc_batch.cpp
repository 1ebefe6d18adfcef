// Batches of sampling jobs (fc_batch_create / fc_batch_run / fc_batch_destroy).
//
// A batch turns many (graph, alpha, tree range) jobs into lists of work items
// (trees), ordered largest graph first so that the longest trees start early,
// and samples each list with a workgroup-per-tree kernel in one persistent
// launch whose workgroups pull items from a device queue.  With LDS counters
// the jobs fall into up to two launch groups: graphs whose counter fields take
// at most a quarter of a CU's LDS ("narrow": several trees per CU, narrower
// workgroups) and the rest ("wide": one or two trees per CU).  Each group's
// per-slot scratch is sized for its largest graph.  Everything that does not
// change between runs (validation, vertex records, relabelling, item order,
// scratch, launch shapes) happens once in fc_batch_create; a run replays one
// captured HIP graph: per group, fill kernels (counters, draw-count epochs)
// and the sampling kernel.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <mutex>
#include <numeric>
#include <utility>
#include <vector>

#include "fc_internal.hpp"

using namespace fc_host;

namespace {

// One persistent launch: its jobs (batch job indices, largest graph first),
// device job table and item map, scratch, counters and launch shape.
struct Group {
    std::vector<int32_t> jobs;
    DevBuf jobtab, item_job, word, kk, lists, levels, bits, small, scratch_r;
    fc::CoopArgs args{};
    uint32_t n_max = 0, item_count = 0, slots = 0, threads = 512, wg_per_cu = 4;
    size_t ntab = 0, kk_words = 0;
    bool use_lds = false, lds_bits = false, in_bits = false, word32 = true;
    bool weighted = false;   // some job's graph carries edge weights
    bool repop = false;      // re-formed 2-cycles popped within their round (LDS kernel)
    bool lean = false;       // LDS kernel: the lean register shape (at most 512 threads)
    uint32_t repop_words = 0;  // the same, global-counter kernel: its LDS filter (set with the shape)
    uint32_t lds_words = 0;  // dynamic LDS of the LDS-counter kernel (largest graph)
};

}  // namespace

struct fc_batch {
    fc_ctx *ctx = nullptr;
    std::vector<fc_job> jobs;
    uint64_t seed = 0;
    int32_t flags = 0;
    DevBuf vrec, dmax, iso, wsum, wthr, wtot;  // weighted graphs' running row sums and step
                                               // thresholds, each job's weighted volume
    DevBuf rl_blk, rl_base, rl_bounds, rl_inv, rl_orig, rl_adj, rl_vrec;  // degree-class relabelling
    Group grp[2];
    int ngroups = 0;
    uint32_t item_count = 0;
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
    for (DevBuf *d : {&b->vrec, &b->dmax, &b->iso, &b->wsum, &b->wthr, &b->wtot, &b->rl_blk, &b->rl_base, &b->rl_bounds, &b->rl_inv,
                      &b->rl_orig, &b->rl_adj, &b->rl_vrec})
        if (d->ptr) (void)hipFree(d->ptr);
    for (Group &g : b->grp)
        for (DevBuf *d : {&g.jobtab, &g.item_job, &g.word, &g.kk, &g.lists, &g.levels, &g.bits,
                          &g.small, &g.scratch_r})
            if (d->ptr) (void)hipFree(d->ptr);
    for (hipEvent_t e : {b->ev_in, b->ev0, b->ev1})
        if (e) (void)hipEventDestroy(e);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return FC_OK;
}

// Enqueue one run of a group on `stream`: reset its counters (and draw-count
// epochs for the global-counter kernel), then sample.
hipError_t enqueue_group(const Group &g, const fc::CoopArgs &a, uint32_t threads,
                         hipStream_t stream) {
    hipError_t e = fc::launch_fill_u64(static_cast<unsigned long long *>(g.small.ptr),
                                       sizeof(Small) / 8, 0ull, stream);
    if (e != hipSuccess) return e;
    if (g.use_lds)
        return fc::launch_wilson_lds(a, threads, g.lds_words, g.weighted, g.repop, g.lean, stream);
    e = fc::launch_fill_u64(static_cast<unsigned long long *>(g.kk.ptr), g.kk_words, 0ull, stream);
    if (e != hipSuccess) return e;
    return fc::launch_wilson_coop(a, threads, g.lds_bits, g.in_bits, g.word32, g.weighted,
                                  g.repop_words, stream);
}

// Size a group's scratch for `slots` workgroups and point its arguments at it.
int size_scratch(fc_ctx *ctx, Group &g, uint32_t slots) {
    int rc;
    const size_t n = g.n_max, nwords = (n + 31) / 32;
    const size_t wbytes = g.word32 && !g.use_lds ? 4 : 8;
    if ((rc = ensure(ctx, g.word, wbytes * n * slots, "batch tree words"))) return rc;
    if (!g.use_lds && (rc = ensure(ctx, g.kk, 8 * n * slots, "batch draw counts"))) return rc;
    if ((rc = ensure(ctx, g.lists, 24 * n * slots, "batch lists"))) return rc;
    if ((rc = ensure(ctx, g.levels, 4 * (n + 2) * slots, "batch levels"))) return rc;
    if (!g.use_lds && !g.lds_bits && (rc = ensure(ctx, g.bits, 4 * nwords * slots, "batch bitmap")))
        return rc;
    g.kk_words = n * slots;
    g.slots = slots;
    fc::CoopArgs &a = g.args;
    a.word = g.word.ptr;
    a.kk = g.use_lds ? nullptr : static_cast<uint64_t *>(g.kk.ptr);
    a.lists = static_cast<uint64_t *>(g.lists.ptr);
    a.levels = static_cast<uint32_t *>(g.levels.ptr);
    a.bits = g.lds_bits || g.use_lds ? nullptr : static_cast<uint32_t *>(g.bits.ptr);
    a.slots = slots;
    return FC_OK;
}

// (also picks the re-pop filter of a global-counter group for this shape)
uint32_t slots_for(const fc_ctx *ctx, Group &g, uint32_t threads, uint32_t wg_per_cu) {
    const size_t n = g.n_max;
    const int fit = g.use_lds ? fc::lds_max_active(threads, g.lds_words, g.weighted, g.repop, g.lean)
                              : fc::coop_max_active(threads, g.lds_bits, g.in_bits, g.word32,
                                                    g.n_max, g.weighted, 0u);
    if (fit > 0) wg_per_cu = std::min<uint32_t>(wg_per_cu, static_cast<uint32_t>(fit));
    g.repop_words = g.use_lds ? 0u
                              : coop_repop_words(ctx, threads, wg_per_cu, g.lds_bits, g.in_bits,
                                                 g.word32, g.n_max, g.weighted);
    const size_t per_slot = g.use_lds ? (8 + 24 + 4) * n + 8
                                      : ((g.word32 ? 4 : 8) + 8 + 24 + 4) * n + 8 +
                                            (g.lds_bits ? 0 : 4 * ((n + 31) / 32));
    size_t slots = std::max<size_t>(1, ctx->state_budget / per_slot);
    slots = std::min<size_t>(slots, static_cast<size_t>(ctx->cu_count) * wg_per_cu);
    slots = std::min<size_t>(slots, g.item_count);
    return static_cast<uint32_t>(std::max<size_t>(slots, 1));
}

// Launch shapes chosen by autotuning, per device and group shape: a batch
// created again with the same job shapes (graph sizes, alphas, tree counts,
// options) takes the earlier choice without timing anything.
using TuneKey = std::vector<uint64_t>;
std::mutex g_tune_mu;
std::map<TuneKey, std::array<uint32_t, 4>> g_tune_cache;

// The on-disk form of the cache (environment variable FC_TUNE_CACHE: a file
// of lines "key threads wg_per_cu repop lean", the key a comma-separated list of
// the device's CU count and LDS size and the group's shape words).  Read when
// a key is missing from the process's cache; a tuned choice is appended.
std::string key_text(const fc_ctx *ctx, const TuneKey &k) {
    std::ostringstream os;
    os << ctx->cu_count << ',' << ctx->max_lds;
    for (uint64_t x : k) os << ',' << std::hex << x << std::dec;
    return os.str();
}

bool disk_lookup(const fc_ctx *ctx, const TuneKey &k, std::array<uint32_t, 4> *out) {
    const char *path = std::getenv("FC_TUNE_CACHE");
    if (!path || !*path) return false;
    std::ifstream f(path);
    if (!f) return false;
    const std::string want = key_text(ctx, k);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {  // the last line for a key wins
        std::istringstream is(line);
        std::string key;
        uint32_t t = 0, w = 0, r = 0, l = 0;
        if ((is >> key >> t >> w >> r >> l) && key == want && t >= 64 && t <= 1024 && t % 64 == 0 &&
            w >= 1 && w <= 64 && r <= 1 && l <= 1 && (l == 0 || t <= 512)) {
            *out = {t, w, r, l};
            found = true;
        }
    }
    return found;
}

void disk_store(const fc_ctx *ctx, const TuneKey &k, const std::array<uint32_t, 4> &c) {
    const char *path = std::getenv("FC_TUNE_CACHE");
    if (!path || !*path) return;
    std::ofstream f(path, std::ios::app);
    if (f) f << key_text(ctx, k) << ' ' << c[0] << ' ' << c[1] << ' ' << c[2] << ' ' << c[3] << '\n';
}

TuneKey tune_key(const fc_batch *b, const Group &g) {
    const fc_ctx *ctx = b->ctx;
    TuneKey k = {static_cast<uint64_t>(ctx->device), g.use_lds, g.n_max, g.lds_words, g.weighted,
                 g.word32, g.lds_bits, g.in_bits, ctx->lds_repop, ctx->coop_repop,
                 ctx->state_budget, ctx->max_draws};
    for (int32_t j : g.jobs) {
        const fc_job &jb = b->jobs[j];
        uint64_t abits;
        std::memcpy(&abits, &jb.alpha, sizeof(abits));
        k.insert(k.end(), {static_cast<uint64_t>(jb.graph.n), static_cast<uint64_t>(jb.graph.nnz),
                           abits, jb.tree_count, jb.graph.weights != nullptr});
    }
    return k;
}

// Launch-shape autotuning of one group on a sample of its work items with
// throw-away outputs: results never depend on the shape, only the time does.
// Each candidate is launched once on a few items (code load, caches), then
// timed twice on the sample; the best of the two counts.
int autotune(fc_batch *b, Group &g) {
    fc_ctx *ctx = b->ctx;
    int rc = FC_OK;
    const TuneKey key = tune_key(b, g);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        std::array<uint32_t, 4> c{};
        const bool hit = it != g_tune_cache.end() || disk_lookup(ctx, key, &c);
        if (hit) {
            if (it != g_tune_cache.end()) c = it->second;
            else g_tune_cache[key] = c;
            g.threads = c[0];
            g.wg_per_cu = c[1];
            g.repop = c[2] != 0u;
            g.lean = c[3] != 0u;
            return FC_OK;
        }
    }
    static const uint32_t cand_coop[][2] = {{256, 3}, {256, 6}, {512, 2}, {512, 3}, {128, 12}};
    // (threads, workgroups per CU, lean register shape) for the LDS kernel: the
    // lean shape holds fewer loads in flight per lane but fits six waves per SIMD
    // instead of four, which pays where trees are latency-bound (small graphs,
    // large alpha)
    static const uint32_t cand_lds[][3] = {{256, 64, 0}, {512, 64, 0}, {1024, 64, 0}, {256, 4, 0},
                                           {512, 2, 0},  {256, 64, 1}, {512, 64, 1}};
    // (threads, workgroups per CU, re-pops, lean): with option lds_repop = 3 the
    // LDS groups are timed with and without popping re-formed 2-cycles within
    // their round (the same trees either way; it pays on BA and ER graphs, not on
    // R-MAT batches); 0, 1 and 2 keep the re-pops as the option says
    std::vector<std::array<uint32_t, 4>> cand;
    const bool tune_repop = g.use_lds && ctx->lds_repop == 3;
    if (g.use_lds) {
        for (const auto &c : cand_lds) {
            cand.push_back({c[0], c[1], g.repop ? 1u : 0u, c[2]});
            if (tune_repop) cand.push_back({c[0], c[1], g.repop ? 0u : 1u, c[2]});
        }
    } else {
        for (const auto &c : cand_coop) cand.push_back({c[0], c[1], g.repop ? 1u : 0u, 0u});
    }
    // throw-away job table: same graphs and records, outputs into one scratch R
    std::vector<fc::CoopJob> tab(g.ntab);
    FC_HIP(ctx, hipMemcpy(tab.data(), g.jobtab.ptr, sizeof(fc::CoopJob) * tab.size(),
                          hipMemcpyDeviceToHost), "read job table");
    if ((rc = ensure(ctx, g.scratch_r, 4 * static_cast<size_t>(g.n_max), "tuning outputs"))) return rc;
    // the tuning sample: a thirty-second of every job's trees (at least one), so
    // that every graph and alpha of the group is in it, not only the largest
    // first jobs
    std::vector<uint32_t> tmap;
    for (size_t t = 0; t < tab.size(); ++t) {
        fc::CoopJob &j = tab[t];
        j.root_counts = static_cast<uint32_t *>(g.scratch_r.ptr);
        j.visit_counts = nullptr;
        j.tree_digests = nullptr;
        j.tree_steps = nullptr;
        j.parents = nullptr;
        j.tree_visits = nullptr;
        const uint32_t c = j.tree_count ? std::max<uint32_t>(1, j.tree_count / 32) : 0u;
        j.first_item = static_cast<uint32_t>(tmap.size());
        j.tree_count = c;
        tmap.insert(tmap.end(), c, static_cast<uint32_t>(t));
    }
    if (tmap.empty()) return FC_OK;
    DevBuf tmp_tab, tmp_map;
    if ((rc = ensure(ctx, tmp_tab, sizeof(fc::CoopJob) * tab.size(), "tuning job table")) ||
        (rc = ensure(ctx, tmp_map, 4 * tmap.size(), "tuning item map"))) {
        if (tmp_tab.ptr) (void)hipFree(tmp_tab.ptr);
        return rc;
    }
    const uint32_t prefix = static_cast<uint32_t>(tmap.size());
    float best = 1e30f;
    uint32_t best_t = g.threads, best_w = g.wg_per_cu;
    bool best_r = g.repop, best_l = g.lean;
    hipError_t he = hipMemcpy(tmp_tab.ptr, tab.data(), sizeof(fc::CoopJob) * tab.size(),
                              hipMemcpyHostToDevice);
    if (he == hipSuccess)
        he = hipMemcpy(tmp_map.ptr, tmap.data(), 4 * tmap.size(), hipMemcpyHostToDevice);
    if (he != hipSuccess) rc = hip_fail(ctx, he, "write tuning table");
    for (size_t c = 0; rc == FC_OK && c < cand.size(); ++c) {
        g.repop = cand[c][2] != 0u;
        g.lean = cand[c][3] != 0u;
        const uint32_t slots = slots_for(ctx, g, cand[c][0], cand[c][1]);
        if ((rc = size_scratch(ctx, g, slots))) break;
        fc::CoopArgs a = g.args;
        a.jobs = static_cast<const fc::CoopJob *>(tmp_tab.ptr);
        a.item_job = static_cast<const uint32_t *>(tmp_map.ptr);
        float cbest = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            // rep 0 warms the variant up on the first few items; reps 1 and 2 are timed
            a.item_count = rep == 0 ? std::min<uint32_t>(prefix, slots) : prefix;
            if ((he = hipEventRecord(b->ev0, b->stream)) != hipSuccess ||
                (he = enqueue_group(g, a, cand[c][0], b->stream)) != hipSuccess ||
                (he = hipEventRecord(b->ev1, b->stream)) != hipSuccess ||
                (he = hipStreamSynchronize(b->stream)) != hipSuccess) {
                rc = hip_fail(ctx, he, "tuning run");
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, b->ev0, b->ev1);
            Small sm;
            if ((he = hipMemcpy(&sm, g.small.ptr, sizeof(sm), hipMemcpyDeviceToHost)) != hipSuccess) {
                rc = hip_fail(ctx, he, "read counters");
                break;
            }
            if (sm.totals.error) {
                rc = set_err(ctx, FC_ERR_HIP, "autotuning run reported a kernel error");
                break;
            }
            if (rep > 0) cbest = std::min(cbest, ms);
        }
        if (rc == FC_OK && cbest < best) {
            best = cbest;
            best_t = cand[c][0];
            best_w = cand[c][1];
            best_r = cand[c][2] != 0u;
            best_l = cand[c][3] != 0u;
        }
    }
    if (tmp_tab.ptr) (void)hipFree(tmp_tab.ptr);
    if (tmp_map.ptr) (void)hipFree(tmp_map.ptr);
    g.repop = best_r;
    g.lean = best_l;
    if (rc) return rc;
    g.threads = best_t;
    g.wg_per_cu = best_w;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = {best_t, best_w, best_r ? 1u : 0u, best_l ? 1u : 0u};
    disk_store(ctx, key, g_tune_cache[key]);
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
    b->item_count = static_cast<uint32_t>(items);
    auto fail = [&](int code) {
        free_batch(b);
        return code;
    };
#define FB_HIP(expr, what)                                          \
    do {                                                            \
        hipError_t e_ = (expr);                                     \
        if (e_ != hipSuccess) return fail(hip_fail(ctx, e_, what)); \
    } while (0)
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&b->ev_in) != hipSuccess || hipEventCreate(&b->ev0) != hipSuccess ||
        hipEventCreate(&b->ev1) != hipSuccess)
        return fail(set_err(ctx, FC_ERR_HIP, "creating the batch stream and events failed"));
    if (items == 0) {
        *out = b;
        return FC_OK;
    }

    // validate each distinct graph once
    if (!(flags & FC_FLAG_TRUSTED_GRAPH)) {
        std::vector<std::pair<const int32_t *, const double *>> seen;
        for (const fc_job &j : b->jobs) {
            const std::pair<const int32_t *, const double *> key(j.graph.row_ptr, j.graph.weights);
            if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
            seen.push_back(key);
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
    std::vector<size_t> pos(n_jobs, 0);  // job index -> place in `order`
    for (size_t k = 0; k < order.size(); ++k) pos[order[k]] = k;

    // vertex records of every job's G* and each graph's maximum degree
    std::vector<size_t> voff(order.size()), ioff(order.size());
    size_t vtotal = 0, itotal = 0;
    for (size_t k = 0; k < order.size(); ++k) {
        voff[k] = vtotal;
        ioff[k] = itotal;
        vtotal += static_cast<size_t>(b->jobs[order[k]].graph.n);
        itotal += (static_cast<size_t>(b->jobs[order[k]].graph.n) + 31) / 32;
    }
    if ((rc = ensure(ctx, b->vrec, sizeof(fc::VRec) * vtotal, "batch vertex records"))) return fail(rc);
    if ((rc = ensure(ctx, b->iso, 4 * itotal, "batch isolated bitmaps"))) return fail(rc);
    uint32_t *iso = static_cast<uint32_t *>(b->iso.ptr);
    if ((rc = ensure(ctx, b->dmax, 4 * order.size(), "batch degrees"))) return fail(rc);
    FB_HIP(hipMemsetAsync(b->dmax.ptr, 0, 4 * order.size(), b->stream), "memset degrees");
    if ((rc = ensure(ctx, b->wtot, 8 * order.size(), "batch weighted volumes"))) return fail(rc);
    FB_HIP(hipMemsetAsync(b->wtot.ptr, 0, 8 * order.size(), b->stream), "memset volumes");
    double *wtot_d = static_cast<double *>(b->wtot.ptr);
    fc::VRec *vrec = static_cast<fc::VRec *>(b->vrec.ptr);
    unsigned int *dmax_d = static_cast<unsigned int *>(b->dmax.ptr);
    // degree classes of each distinct graph, for the LDS-counter kernel
    struct GInfo {
        const int32_t *rp, *ci;
        const double *w;
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
        const double *w = gr.nnz ? gr.weights : nullptr;
        while (f < gs.size() && !(gs[f].rp == gr.row_ptr && gs[f].ci == gr.col_idx &&
                                  gs[f].w == w && gs[f].n == static_cast<uint32_t>(gr.n)))
            ++f;
        if (f == gs.size()) {
            gs.push_back({gr.row_ptr, gr.col_idx, w, static_cast<uint32_t>(gr.n), gr.nnz, tn, te, tb});
            tn += static_cast<size_t>(gr.n);
            te += static_cast<size_t>(gr.nnz);
            tb += fc::relabel_blocks(static_cast<uint32_t>(gr.n));
        }
        gof[k] = static_cast<uint32_t>(f);
    }
    // running row weight sums of each distinct weighted graph (same offsets as
    // its CSR entries), then the records with weighted root thresholds
    bool any_weighted = false;
    for (const GInfo &gi : gs) any_weighted = any_weighted || gi.w;
    if (any_weighted &&
        ((rc = ensure(ctx, b->wsum, 8 * std::max<size_t>(te, 1), "batch weight sums")) ||
         (rc = ensure(ctx, b->wthr, 4 * (te + fc::kWeightedScan), "batch step thresholds"))))
        return fail(rc);
    double *wsum = static_cast<double *>(b->wsum.ptr);
    uint32_t *wthr = static_cast<uint32_t *>(b->wthr.ptr);
    for (const GInfo &gi : gs)
        if (gi.w) {
            FB_HIP(fc::launch_row_wsum(gi.rp, gi.w, static_cast<int32_t>(gi.n), wsum + gi.off_e,
                                       b->stream), "row weight sums");
            FB_HIP(fc::launch_step_thresholds(gi.rp, wsum + gi.off_e, static_cast<int32_t>(gi.n),
                                              gi.nnz, wthr + gi.off_e, b->stream),
                   "step thresholds");
        }
    auto wsum_of = [&](size_t k) -> const double * {
        const GInfo &gi = gs[gof[k]];
        return gi.w ? wsum + gi.off_e : nullptr;
    };
    auto wthr_of = [&](size_t k) -> const uint32_t * {
        const GInfo &gi = gs[gof[k]];
        return gi.w ? wthr + gi.off_e : nullptr;
    };
    for (size_t k = 0; k < order.size(); ++k) {
        const fc_job &j = b->jobs[order[k]];
        FB_HIP(fc::launch_build_vrec(j.graph.row_ptr, wsum_of(k), j.graph.n, j.alpha, vrec + voff[k],
                                     dmax_d + k, iso + ioff[k], wtot_d + k, b->stream),
               "build_vrec");
    }
    const bool try_lds = ctx->coop_lds_counts && !order.empty() &&
                         n_max < (1u << fc::kRelabelIdBits);
    std::vector<unsigned int> bounds(4 * gs.size(), 0u);
    if (try_lds) {
        if ((rc = ensure(ctx, b->rl_blk, 4 * fc::kRelabelClasses * tb, "class counts")) ||
            (rc = ensure(ctx, b->rl_base, 4 * fc::kRelabelClasses * tb, "class offsets")) ||
            (rc = ensure(ctx, b->rl_bounds, 16 * gs.size(), "class bounds")))
            return fail(rc);
        uint32_t *blk = static_cast<uint32_t *>(b->rl_blk.ptr);
        uint32_t *base = static_cast<uint32_t *>(b->rl_base.ptr);
        uint32_t *bnd = static_cast<uint32_t *>(b->rl_bounds.ptr);
        for (size_t f = 0; f < gs.size(); ++f)
            FB_HIP(fc::launch_class_bounds(gs[f].rp, gs[f].n, false,
                                           blk + fc::kRelabelClasses * gs[f].off_b,
                                           base + fc::kRelabelClasses * gs[f].off_b, bnd + 4 * f,
                                           b->stream),
                   "class bounds");
        FB_HIP(hipMemcpyAsync(bounds.data(), bnd, 16 * gs.size(), hipMemcpyDeviceToHost, b->stream),
               "copy class bounds");
    }
    std::vector<unsigned int> dmax(order.size());
    FB_HIP(hipMemcpyAsync(dmax.data(), dmax_d, 4 * order.size(), hipMemcpyDeviceToHost, b->stream),
           "copy degrees");
    std::vector<double> wvol(order.size());
    FB_HIP(hipMemcpyAsync(wvol.data(), wtot_d, 8 * order.size(), hipMemcpyDeviceToHost, b->stream),
           "copy weighted volumes");
    FB_HIP(hipStreamSynchronize(b->stream), "batch preparation");
    std::vector<uint32_t> gwords(gs.size(), 0);
    bool use_lds = false;
    if (try_lds) {
        uint32_t words = 0;
        for (size_t f = 0; f < gs.size(); ++f) {
            gwords[f] = fc::count_layout(bounds[4 * f + 3], bounds[4 * f], bounds[4 * f + 1],
                                         bounds[4 * f + 2]).words;
            words = std::max(words, gwords[f]);
        }
        use_lds = 4u * static_cast<size_t>(words) + kLdsStaticBytes <= ctx->max_lds;
    }
    if (use_lds) {
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
            FB_HIP(fc::launch_relabel_graph(gi.rp, gi.ci, gi.n, gi.nnz,
                                            base + fc::kRelabelClasses * gi.off_b, fc::kRelabelIdBits,
                                            inv + gi.off_n, orig + gi.off_n, adj + gi.off_e,
                                            b->stream), "relabel");
        fc::VRec *vr = static_cast<fc::VRec *>(b->rl_vrec.ptr);
        for (size_t k = 0; k < order.size(); ++k)
            FB_HIP(fc::launch_relabel_vrec(vrec + voff[k], inv + gs[gof[k]].off_n,
                                           static_cast<uint32_t>(b->jobs[order[k]].graph.n),
                                           vr + voff[k], b->stream), "relabel records");
    }

    // launch groups: with LDS counters, jobs whose fields take at most a third
    // of the LDS form the narrow group (three workgroups per CU fit, as many as
    // the lean shape's registers allow at 512 threads); everything else is one
    // group
    for (size_t k = 0; k < order.size(); ++k) {
        const bool narrow = use_lds && 4u * static_cast<size_t>(gwords[gof[k]]) + kLdsStaticBytes <=
                                           ctx->max_lds / 3;
        b->grp[narrow ? 1 : 0].jobs.push_back(order[k]);
    }
    if (b->grp[0].jobs.empty()) std::swap(b->grp[0].jobs, b->grp[1].jobs);
    b->ngroups = b->grp[1].jobs.empty() ? 1 : 2;

    for (int gi = 0; gi < b->ngroups; ++gi) {
        Group &g = b->grp[gi];
        if ((rc = ensure(ctx, g.small, sizeof(Small), "batch counters"))) return fail(rc);
        g.use_lds = use_lds;
        g.word32 = ctx->coop_word32;
        for (int32_t j : g.jobs) {
            const size_t k = pos[j];
            g.n_max = std::max<uint32_t>(g.n_max, static_cast<uint32_t>(b->jobs[j].graph.n));
            g.item_count += b->jobs[j].tree_count;
            g.weighted = g.weighted || wsum_of(k) != nullptr;
            if (use_lds) g.lds_words = std::max(g.lds_words, gwords[gof[k]]);
            uint32_t ts;
            bool w32;
            word_layout(static_cast<uint32_t>(b->jobs[j].graph.n), dmax[k], true, &ts, &w32);
            g.word32 = g.word32 && w32;
        }
        g.repop = ctx->lds_repop >= 2 || (ctx->lds_repop == 1 && g.weighted);
        g.lds_bits = !use_lds && ctx->coop_lds_bits &&
                     fc::coop_lds_bytes(g.n_max) + 1024u <= ctx->max_lds;
        g.in_bits = g.lds_bits && ctx->coop_in_bits &&
                    2 * fc::coop_lds_bytes(g.n_max) + 1024u <= ctx->max_lds;

        // job table and item -> job map
        std::vector<fc::CoopJob> tab(g.jobs.size());
        std::vector<uint32_t> item_job(g.item_count);
        uint32_t first = 0;
        for (size_t t = 0; t < g.jobs.size(); ++t) {
            const fc_job &j = b->jobs[g.jobs[t]];
            const size_t k = pos[g.jobs[t]];
            fc::CoopJob &c = tab[t];
            std::memset(&c, 0, sizeof(c));
            c.vrec = vrec + voff[k];
            c.col_idx = j.graph.col_idx;
            c.wsum = wsum_of(k);
            c.wthr = wthr_of(k);
            c.n = static_cast<uint32_t>(j.graph.n);
            c.tree_count = j.tree_count;
            c.iso = use_lds ? nullptr : iso + ioff[k];
            if (use_lds) {
                const GInfo &gf = gs[gof[k]];
                c.vrec = static_cast<const fc::VRec *>(b->rl_vrec.ptr) + voff[k];
                c.adj = static_cast<const unsigned long long *>(b->rl_adj.ptr) + gf.off_e;
                c.orig = static_cast<const uint32_t *>(b->rl_orig.ptr) + gf.off_n;
                c.n0 = bounds[4 * gof[k]];
                c.n1 = bounds[4 * gof[k] + 1];
                c.n2 = bounds[4 * gof[k] + 2];
                c.n3 = bounds[4 * gof[k] + 3];
            }
            bool w32;
            word_layout(c.n, dmax[k], g.word32, &c.tshift, &w32);
            c.stream_id = j.stream_id;
            c.tree_begin = j.tree_begin;
            c.first_item = first;
            const double vol = c.wsum ? wvol[k] : static_cast<double>(j.graph.nnz);
            const double cap = 256.0 * (static_cast<double>(j.graph.n) + j.alpha * vol) + 1048576.0;
            c.step_cap = cap > 4.0e18 ? 4000000000000000000ull : static_cast<unsigned long long>(cap);
            c.root_counts = j.root_counts;
            c.tree_digests = reinterpret_cast<unsigned long long *>(j.tree_digests);
            std::fill(item_job.begin() + first, item_job.begin() + first + j.tree_count,
                      static_cast<uint32_t>(t));
            first += j.tree_count;
        }
        g.ntab = tab.size();
        if ((rc = ensure(ctx, g.jobtab, sizeof(fc::CoopJob) * tab.size(), "job table"))) return fail(rc);
        if ((rc = ensure(ctx, g.item_job, 4 * item_job.size(), "item map"))) return fail(rc);
        FB_HIP(hipMemcpyAsync(g.jobtab.ptr, tab.data(), sizeof(fc::CoopJob) * tab.size(),
                              hipMemcpyHostToDevice, b->stream), "copy job table");
        FB_HIP(hipMemcpyAsync(g.item_job.ptr, item_job.data(), 4 * item_job.size(),
                              hipMemcpyHostToDevice, b->stream), "copy item map");
        FB_HIP(hipStreamSynchronize(b->stream), "batch tables");

        fc::CoopArgs &a = g.args;
        std::memset(&a, 0, sizeof(a));
        a.n_max = g.n_max;
        a.item_count = g.item_count;
        a.key0 = static_cast<uint32_t>(seed);
        a.key1 = static_cast<uint32_t>(seed >> 32);
        a.max_rounds = 0x40000000u;
        a.k_limit = ctx->max_draws ? ctx->max_draws : use_lds ? 0xFFFFFFFFu : 0x7FFFFFFFu;
        Small *sm = static_cast<Small *>(g.small.ptr);
        a.queue = &sm->queue;
        a.totals = &sm->totals;
        a.phase_ticks = nullptr;
        a.jobs = static_cast<const fc::CoopJob *>(g.jobtab.ptr);
        a.item_job = static_cast<const uint32_t *>(g.item_job.ptr);
        if (use_lds) {
            g.threads = lds_threads_for(ctx, g.item_count, g.lds_words);
            g.wg_per_cu = ctx->lds_wg_per_cu ? ctx->lds_wg_per_cu : 64u;
            g.lean = ctx->lds_lean && g.threads <= 512u;
        } else {
            g.threads = ctx->coop_threads;
            g.wg_per_cu = ctx->coop_wg_per_cu;
        }
        if ((flags & FC_FLAG_AUTOTUNE) && (rc = autotune(b, g))) return fail(rc);
        if ((rc = size_scratch(ctx, g, slots_for(ctx, g, g.threads, g.wg_per_cu)))) return fail(rc);
    }

    // capture the run: per group, counter resets and the sampling kernel
    FB_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    hipError_t ce = hipSuccess;
    for (int gi = 0; gi < b->ngroups && ce == hipSuccess; ++gi)
        ce = enqueue_group(b->grp[gi], b->grp[gi].args, b->grp[gi].threads, b->stream);
    hipError_t ee = hipStreamEndCapture(b->stream, &b->graph);
    if (ce != hipSuccess) return fail(hip_fail(ctx, ce, "capturing the batch launch"));
    if (ee != hipSuccess) return fail(hip_fail(ctx, ee, "end capture"));
    FB_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "instantiate graph");
#undef FB_HIP
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
        const Group &g = b->grp[0];
        if (b->ngroups == 2)
            std::snprintf(stats->sampler, sizeof(stats->sampler), "%s:%u+%u",
                          g.use_lds ? "lbatch" : "batch", g.threads, b->grp[1].threads);
        else
            std::snprintf(stats->sampler, sizeof(stats->sampler), "%s:%ux%u",
                          g.use_lds ? "lbatch" : "batch", g.threads, g.wg_per_cu);
    }
    if (b->item_count == 0) return FC_OK;
    // order after the caller's earlier work on the context stream, and make the
    // context stream wait for the batch
    FC_HIP(ctx, hipEventRecord(b->ev_in, ctx->stream), "event");
    FC_HIP(ctx, hipStreamWaitEvent(b->stream, b->ev_in, 0), "wait");
    FC_HIP(ctx, hipEventRecord(b->ev0, b->stream), "event");
    FC_HIP(ctx, hipGraphLaunch(b->exec, b->stream), "graph launch");
    FC_HIP(ctx, hipEventRecord(b->ev1, b->stream), "event");
    Small sm[2];
    for (int gi = 0; gi < b->ngroups; ++gi)
        FC_HIP(ctx, hipMemcpyAsync(&sm[gi], b->grp[gi].small.ptr, sizeof(Small),
                                   hipMemcpyDeviceToHost, b->stream), "copy counters");
    FC_HIP(ctx, hipStreamSynchronize(b->stream), "batch run");
    FC_HIP(ctx, hipStreamWaitEvent(ctx->stream, b->ev1, 0), "wait");
    unsigned int error = 0;
    unsigned long long steps = 0, roots = 0, digests = 0;
    for (int gi = 0; gi < b->ngroups; ++gi) {
        error |= sm[gi].totals.error;
        steps += sm[gi].totals.walk_steps;
        roots += sm[gi].totals.roots;
        digests += sm[gi].totals.digest_sum;
    }
    if (error & fc::kErrStepCap)
        return set_err(ctx, FC_ERR_HIP, "a tree exceeded the step bound (internal fault)");
    if (error & fc::kErrVisitOverflow)
        return set_err(ctx, FC_ERR_OVERFLOW,
                       b->grp[0].use_lds ? "a per-vertex draw count exceeded 2^28 - 1 (LDS counters)"
                                         : "a per-vertex visit counter exceeded 2^31 - 1");
    if (stats) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, b->ev0, b->ev1);
        stats->trees_in_flight = b->grp[0].slots + (b->ngroups == 2 ? b->grp[1].slots : 0u);
        stats->walk_steps = steps;
        stats->roots = roots;
        stats->digest_sum = digests;
        stats->ms_sample = ms;
        stats->ms_total = now_ms() - t0;
    }
    return FC_OK;
}

int fc_batch_destroy(fc_batch *b) { return free_batch(b); }

}  // extern "C"
