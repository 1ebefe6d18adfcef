// fc_group_closeness: the greedy group forest closeness maximiser of
// Algorithm 2 (Section 5) on dense device matrices.
#include <cmath>
#include <cstring>
#include <vector>

#include "fc_internal.hpp"
#include "fc_group_kernels.hpp"

using namespace fc_host;

extern "C" int fc_group_closeness(fc_ctx *ctx, const fc_graph *g, double alpha, int32_t k,
                                  int32_t flags, int32_t *group, double *farness) {
    int rc = begin(ctx);
    if (rc) return rc;
    if (!valid_alpha(alpha)) return set_err(ctx, FC_ERR_ARG, "alpha must be finite and > 0");
    if (!group) return set_err(ctx, FC_ERR_ARG, "group is NULL");
    GraphView gv;
    if ((rc = prepare_graph(ctx, g, flags & FC_FLAG_TRUSTED_GRAPH, &gv))) return rc;
    if (gv.n < 1 || k < 1 || k > gv.n) return set_err(ctx, FC_ERR_ARG, "need 1 <= k <= n");
    if (gv.n > 65535) return set_err(ctx, FC_ERR_UNSUPPORTED, "dense group closeness needs n <= 65535");
    const uint32_t n = static_cast<uint32_t>(gv.n);
    const uint32_t N = fc::group_dim(n);
    const size_t chunks = fc::group_chunks(n);
    if ((rc = ensure(ctx, ctx->g_mat, sizeof(double) * N * static_cast<size_t>(N), "dense matrix")) ||
        (rc = ensure(ctx, ctx->g_vec,
                     sizeof(double) * (4 * static_cast<size_t>(n) + 64 * 64 + 16 + 2 * static_cast<size_t>(k)),
                     "group vectors")) ||
        (rc = ensure(ctx, ctx->g_scr, sizeof(double) * fc::group_scratch_doubles(N), "inverse scratch")) ||
        (rc = ensure(ctx, ctx->g_part, sizeof(double) * chunks * N, "column sums")) ||
        (rc = ensure(ctx, ctx->g_taken, n, "group flags")))
        return rc;
    double *A = static_cast<double *>(ctx->g_mat.ptr);
    double *vec = static_cast<double *>(ctx->g_vec.ptr);
    double *cv = vec, *rv = vec + n, *diag = vec + 2 * n;
    // per gain block (256 ids): largest gain's bits and its smallest id
    unsigned long long *bmax = reinterpret_cast<unsigned long long *>(vec + 3 * n);
    double *bdiag = vec + 3 * static_cast<size_t>(n) + (n + 255) / 256;
    uint32_t *bid = reinterpret_cast<uint32_t *>(bdiag + (n + 255) / 256);
    double *scal = vec + 4 * static_cast<size_t>(n) + 64 * 64;  // [0] trace, [1] pivot
    unsigned long long *sel = reinterpret_cast<unsigned long long *>(scal + 4);
    uint32_t *bad = reinterpret_cast<uint32_t *>(scal + 6);
    double *fout = scal + 16;                                     // f(S) of step s
    int32_t *gout = reinterpret_cast<int32_t *>(fout + k);         // vertex of step s
    double *part = static_cast<double *>(ctx->g_part.ptr);
    uint8_t *taken = static_cast<uint8_t *>(ctx->g_taken.ptr);

    // Omega = (alpha L + I)^{-1}; the first vertex minimises Omega_vv (Algorithm 2
    // takes the minimiser of n P[v, v] + tr(P), P = pinv(L*), whose V-block is Omega
    // minus a constant)
    FC_HIP(ctx, fc::launch_group_build(gv.row_ptr, gv.col_idx, gv.weights, n, alpha, A, ctx->stream),
           "dense build");
    FC_HIP(ctx, fc::launch_group_invert(A, N, static_cast<double *>(ctx->g_scr.ptr), ctx->stream),
           "dense inverse");
    FC_HIP(ctx, hipMemsetAsync(sel, 0xFF, 2 * sizeof(unsigned long long), ctx->stream), "memset");
    FC_HIP(ctx, fc::launch_group_first(A, n, N, diag, sel, ctx->stream), "first vertex");
    unsigned long long hsel[2];
    FC_HIP(ctx, hipMemcpyAsync(hsel, sel, sizeof(hsel), hipMemcpyDeviceToHost, ctx->stream), "copy");
    FC_HIP(ctx, hipStreamSynchronize(ctx->stream), "first vertex");
    if (hsel[1] >= n) return set_err(ctx, FC_ERR_HIP, "no first vertex (non-finite inverse)");
    const uint32_t v0 = static_cast<uint32_t>(hsel[1]);
    // M = inverse of L* without v0 (slot v0 now stands for u*)
    FC_HIP(ctx, fc::launch_group_reground(A, n, N, v0, cv, ctx->stream), "change of ground");
    FC_HIP(ctx, hipMemsetAsync(taken, 0, n, ctx->stream), "memset flags");
    FC_HIP(ctx, hipMemsetAsync(taken + v0, 1, 1, ctx->stream), "flag");
    FC_HIP(ctx, fc::launch_group_trace(A, n, N, n, scal, scal + 1, ctx->stream), "trace");
    FC_HIP(ctx, fc::launch_group_colsq(A, n, N, n, cv, rv, scal + 1, part, ctx->stream), "column sums");
    double tr = 0.0;
    FC_HIP(ctx, hipMemcpyAsync(&tr, scal, sizeof(tr), hipMemcpyDeviceToHost, ctx->stream), "copy");
    FC_HIP(ctx, hipStreamSynchronize(ctx->stream), "trace");
    group[0] = static_cast<int32_t>(v0);
    if (farness) farness[0] = tr;
    if (k == 1) return FC_OK;
    // the remaining steps run back to back on the device (each choice is read by
    // the next step's kernels there); choices and f(S) come back once at the end
    FC_HIP(ctx, hipMemsetAsync(bad, 0, sizeof(uint32_t), ctx->stream), "memset");
    for (int32_t s = 1; s < k; ++s)
        FC_HIP(ctx, fc::launch_group_step(A, n, N, part, taken, bmax, bid, bdiag, sel + 1, cv, rv,
                                          scal + 1, gout, farness ? fout : nullptr,
                                          static_cast<uint32_t>(s), bad, ctx->stream),
               "greedy step");
    if (farness)  // f(S) after the last step
        FC_HIP(ctx, fc::launch_group_trace(A, n, N, n, fout + (k - 1), nullptr, ctx->stream), "trace");
    uint32_t hbad = 0;
    std::vector<int32_t> hg(static_cast<size_t>(k));
    FC_HIP(ctx, hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, ctx->stream), "copy");
    FC_HIP(ctx, hipMemcpyAsync(hg.data() + 1, gout + 1, sizeof(int32_t) * (k - 1), hipMemcpyDeviceToHost,
                               ctx->stream), "copy");
    if (farness)
        FC_HIP(ctx, hipMemcpyAsync(farness + 1, fout + 1, sizeof(double) * (k - 1), hipMemcpyDeviceToHost,
                                   ctx->stream), "copy");
    FC_HIP(ctx, hipStreamSynchronize(ctx->stream), "group closeness");
    if (hbad & 2u) return set_err(ctx, FC_ERR_HIP, "a greedy step met a NaN gain (non-finite entries in the inverse)");
    if (hbad) return set_err(ctx, FC_ERR_HIP, "a greedy step found no candidate vertex");
    std::memcpy(group + 1, hg.data() + 1, sizeof(int32_t) * (k - 1));
    return FC_OK;
}
