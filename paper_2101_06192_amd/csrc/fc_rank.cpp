// fc_rank and fc_kendall_tau: the ranking output of the estimate (Section 6,
// "Vertex Ranking") on the device.
#include <cmath>
#include <cstring>
#include <limits>
#include <utility>
#include <vector>

#include "fc_internal.hpp"
#include "fc_rank_kernels.hpp"

using namespace fc_host;

namespace {

// rk_hist holds the 8 x 256 digit counts, the 8 x 256 digit bases, then a
// NaN flag and the four Kendall sums (u64 at word offset kOutWord).
constexpr size_t kHistWords = 8 * 256;
constexpr size_t kFlagWord = 2 * kHistWords;
constexpr size_t kOutWord = kFlagWord + 8;
constexpr size_t kSmallBytes = 4 * (2 * kHistWords + 64);

int ensure_sort(fc_ctx *ctx, size_t n) {
    int rc;
    if ((rc = ensure(ctx, ctx->rk_key0, 8 * n, "rank keys")) ||
        (rc = ensure(ctx, ctx->rk_key1, 8 * n, "rank keys")) ||
        (rc = ensure(ctx, ctx->rk_val0, 4 * n, "rank values")) ||
        (rc = ensure(ctx, ctx->rk_val1, 4 * n, "rank values")) ||
        (rc = ensure(ctx, ctx->rk_hist, kSmallBytes, "digit counts")) ||
        (rc = ensure(ctx, ctx->rk_thist,
                     4 * 256 * static_cast<size_t>(fc::rank_tiles(static_cast<uint32_t>(n))),
                     "tile counts")))
        return rc;
    return FC_OK;
}

// Stable sort of the keys in rk_key0 with the values in rk_val0 (rk_key0 /
// rk_val0 and rk_key1 / rk_val1 alternate); *keys and *vals point at the
// sorted arrays.  With score set, the keys are first made from the scores
// (FC_ERR_ARG when a score is NaN); else rk_key0 / rk_val0 hold them already.
int sort_keys(fc_ctx *ctx, const double *score, uint32_t n, bool descending,
              const uint64_t **keys, const int32_t **vals) {
    unsigned int *hist = static_cast<unsigned int *>(ctx->rk_hist.ptr);
    unsigned int *base_d = hist + kHistWords;
    unsigned int *bad_d = hist + kFlagWord;
    FC_HIP(ctx, hipMemsetAsync(hist, 0, 4 * (kFlagWord + 1), ctx->stream), "memset counts");
    if (score)
        FC_HIP(ctx, fc::launch_rank_keys(score, n, descending,
                                         static_cast<uint64_t *>(ctx->rk_key0.ptr),
                                         static_cast<int32_t *>(ctx->rk_val0.ptr), bad_d,
                                         ctx->stream),
               "rank keys");
    FC_HIP(ctx, fc::launch_digit_hist(static_cast<const uint64_t *>(ctx->rk_key0.ptr), n, hist,
                                      ctx->stream),
           "digit counts");
    std::vector<unsigned int> h(kHistWords + 1);
    FC_HIP(ctx, hipMemcpyAsync(h.data(), hist, 4 * kHistWords, hipMemcpyDeviceToHost, ctx->stream),
           "copy digit counts");
    FC_HIP(ctx, hipMemcpyAsync(&h[kHistWords], bad_d, 4, hipMemcpyDeviceToHost, ctx->stream),
           "copy flag");
    FC_HIP(ctx, hipStreamSynchronize(ctx->stream), "digit counts");
    if (h[kHistWords]) return set_err(ctx, FC_ERR_ARG, "score contains NaN");
    // passes whose byte differs between keys, with their digit bases
    std::vector<unsigned int> base(kHistWords, 0);
    bool active[8];
    for (int p = 0; p < 8; ++p) {
        active[p] = true;
        unsigned int run = 0;
        for (int d = 0; d < 256; ++d) {
            const unsigned int c = h[p * 256 + d];
            if (c == n) active[p] = false;
            base[p * 256 + d] = run;
            run += c;
        }
    }
    FC_HIP(ctx, hipMemcpyAsync(base_d, base.data(), 4 * kHistWords, hipMemcpyHostToDevice,
                               ctx->stream),
           "copy digit bases");
    DevBuf *kin = &ctx->rk_key0, *kout = &ctx->rk_key1, *vin = &ctx->rk_val0, *vout = &ctx->rk_val1;
    for (int p = 0; p < 8; ++p) {
        if (!active[p]) continue;
        FC_HIP(ctx, fc::launch_radix_pass(static_cast<const uint64_t *>(kin->ptr),
                                          static_cast<const int32_t *>(vin->ptr), n, 8u * p,
                                          static_cast<unsigned int *>(ctx->rk_thist.ptr),
                                          base_d + p * 256, static_cast<uint64_t *>(kout->ptr),
                                          static_cast<int32_t *>(vout->ptr), ctx->stream),
               "radix pass");
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    *keys = static_cast<const uint64_t *>(kin->ptr);
    *vals = static_cast<const int32_t *>(vin->ptr);
    return FC_OK;
}

}  // namespace

extern "C" int fc_rank(fc_ctx *ctx, const double *score, int32_t n, int32_t descending,
                       int32_t *order, int32_t *rank) {
    int rc = begin(ctx);
    if (rc) return rc;
    if (n < 0) return set_err(ctx, FC_ERR_ARG, "n must be >= 0");
    if (n == 0) return FC_OK;
    if (!score) return set_err(ctx, FC_ERR_ARG, "score is NULL");
    const uint32_t un = static_cast<uint32_t>(n);
    if ((rc = ensure_sort(ctx, static_cast<size_t>(n)))) return rc;
    const uint64_t *keys;
    const int32_t *sorted;
    if ((rc = sort_keys(ctx, score, un, descending != 0, &keys, &sorted))) return rc;
    if (order)
        FC_HIP(ctx, hipMemcpyAsync(order, sorted, 4 * static_cast<size_t>(n),
                                   hipMemcpyDeviceToDevice, ctx->stream),
               "copy order");
    if (rank) FC_HIP(ctx, fc::launch_rank_of(sorted, un, rank, ctx->stream), "rank");
    FC_HIP(ctx, hipStreamSynchronize(ctx->stream), "rank");
    return FC_OK;
}

extern "C" int fc_kendall_tau(fc_ctx *ctx, const double *a, const double *b, int32_t n,
                              double *tau_b, int64_t *counts) {
    int rc = begin(ctx);
    if (rc) return rc;
    if (n < 0) return set_err(ctx, FC_ERR_ARG, "n must be >= 0");
    if (static_cast<int64_t>(n) > 65535LL * 256)
        return set_err(ctx, FC_ERR_UNSUPPORTED, "n must be <= 65535 * 256");
    if (n > 0 && (!a || !b)) return set_err(ctx, FC_ERR_ARG, "a and b must be device pointers");
    const uint32_t un = static_cast<uint32_t>(n);
    // sums on the device: [0] n_c - n_d (pair kernel) or n_d (merge count),
    // [1] tied in a, [2] tied in b, [3] tied in both
    unsigned long long out[4] = {0, 0, 0, 0};
    const bool pairs = ctx->kendall_pairs;
    if (n > 0) {
        const size_t nn = static_cast<size_t>(n);
        if ((rc = ensure_sort(ctx, nn)) || (rc = ensure(ctx, ctx->rk_ra, 4 * nn, "ranks")) ||
            (rc = ensure(ctx, ctx->rk_rb, 4 * nn, "ranks")) ||
            (rc = ensure(ctx, ctx->rk_s, 8 * nn, "merge runs")))
            return rc;
        unsigned long long *out_d =
            reinterpret_cast<unsigned long long *>(static_cast<unsigned int *>(ctx->rk_hist.ptr) +
                                                   kOutWord);
        // each vector's scores -> min-ranks (equal scores share a rank) and its ties
        const double *src[2] = {a, b};
        DevBuf *dst[2] = {&ctx->rk_ra, &ctx->rk_rb};
        for (int v = 0; v < 2; ++v) {
            const uint64_t *keys;
            const int32_t *ids;
            if ((rc = sort_keys(ctx, src[v], un, false, &keys, &ids))) return rc;
            if (v == 0) FC_HIP(ctx, hipMemsetAsync(out_d, 0, sizeof(out), ctx->stream), "memset sums");
            FC_HIP(ctx, fc::launch_min_rank(keys, ids, un, static_cast<uint32_t *>(dst[v]->ptr),
                                            out_d + 1 + v, ctx->stream),
                   "min ranks");
        }
        const uint32_t *ra = static_cast<const uint32_t *>(ctx->rk_ra.ptr);
        const uint32_t *rb = static_cast<const uint32_t *>(ctx->rk_rb.ptr);
        if (pairs) {  // all n(n-1)/2 pairs compared (the definition, tiled)
            FC_HIP(ctx, hipMemsetAsync(out_d, 0, sizeof(out), ctx->stream), "memset sums");
            FC_HIP(ctx, fc::launch_kendall(ra, rb, un, out_d, ctx->stream), "kendall");
        } else {
            // pairs tied in both: equal (rank a, rank b); discordant pairs: strict
            // inversions of rank b in the order of the (a, b) sort
            FC_HIP(ctx, fc::launch_pair_keys(ra, rb, un, static_cast<uint64_t *>(ctx->rk_key0.ptr),
                                             static_cast<int32_t *>(ctx->rk_val0.ptr), ctx->stream),
                   "pair keys");
            const uint64_t *keys;
            const int32_t *ids;
            if ((rc = sort_keys(ctx, nullptr, un, false, &keys, &ids))) return rc;
            FC_HIP(ctx, fc::launch_min_rank(keys, ids, un, nullptr, out_d + 3, ctx->stream),
                   "joint ties");
            uint32_t *sbuf = static_cast<uint32_t *>(ctx->rk_s.ptr);
            FC_HIP(ctx, fc::launch_inversions(rb, ids, un, sbuf, sbuf + nn, out_d, ctx->stream),
                   "inversions");
        }
        FC_HIP(ctx, hipMemcpyAsync(out, out_d, sizeof(out), hipMemcpyDeviceToHost, ctx->stream),
               "copy sums");
        FC_HIP(ctx, hipStreamSynchronize(ctx->stream), "kendall");
    }
    const int64_t n0 = static_cast<int64_t>(n) * (n - 1) / 2;
    const int64_t ta = static_cast<int64_t>(out[1]), tb = static_cast<int64_t>(out[2]),
                  tab = static_cast<int64_t>(out[3]);
    const int64_t untied = n0 - ta - tb + tab;  // n_c + n_d
    const int64_t s = pairs ? static_cast<int64_t>(out[0]) : untied - 2 * static_cast<int64_t>(out[0]);
    if (counts) {
        counts[0] = (untied + s) / 2;
        counts[1] = (untied - s) / 2;
        counts[2] = ta;
        counts[3] = tb;
        counts[4] = tab;
    }
    if (tau_b) {
        const int64_t d1 = n0 - ta, d2 = n0 - tb;
        *tau_b = (d1 == 0 || d2 == 0)
                     ? std::numeric_limits<double>::quiet_NaN()
                     : static_cast<double>(s) /
                           std::sqrt(static_cast<double>(d1) * static_cast<double>(d2));
    }
    return FC_OK;
}
