// fc_solve: block CG on (alpha L + I) X = B in binary64, or binary32 CG
// inside binary64 iterative refinement (residual and update in binary64).
// L is the Laplacian of the graph, weighted when the graph carries weights.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "fc_internal.hpp"

using namespace fc_host;

extern "C" int fc_solve(fc_ctx *ctx, const fc_graph *g, double alpha, const double *B, double *X,
                        int32_t nrhs, double rtol, int32_t precision, int32_t max_iters,
                        int32_t flags, int32_t *iters_out, double *relres_out) {
    int rc = begin(ctx);
    if (rc) return rc;
    if (iters_out) *iters_out = 0;
    if (!valid_alpha(alpha)) return set_err(ctx, FC_ERR_ARG, "alpha must be finite and > 0");
    if (nrhs < 1) return set_err(ctx, FC_ERR_ARG, "nrhs must be >= 1");
    if (nrhs > 64) return set_err(ctx, FC_ERR_UNSUPPORTED, "nrhs must be <= 64 (split the columns)");
    if (!(rtol > 0.0) || !std::isfinite(rtol)) return set_err(ctx, FC_ERR_ARG, "rtol must be > 0");
    if (precision != FC_PREC_FP64 && precision != FC_PREC_FP32_REFINED)
        return set_err(ctx, FC_ERR_ARG, "unknown precision");
    if (max_iters < 1) return set_err(ctx, FC_ERR_ARG, "max_iters must be >= 1");
    GraphView gv;
    if ((rc = prepare_graph(ctx, g, flags & FC_FLAG_TRUSTED_GRAPH, &gv))) return rc;
    const uint32_t n = static_cast<uint32_t>(gv.n), k = static_cast<uint32_t>(nrhs);
    if (n == 0) {
        if (relres_out) std::fill(relres_out, relres_out + k, 0.0);
        return FC_OK;
    }
    if (!B || !X) return set_err(ctx, FC_ERR_ARG, "B and X must be device pointers");

    const bool fp32 = precision == FC_PREC_FP32_REFINED;
    const size_t nk = static_cast<size_t>(n) * k;
    const size_t tb = fp32 ? 4 : 8;
    const uint32_t max_blocks = std::max<uint32_t>(64, ctx->cu_count * 8);
    // workspace is cached in the context (grow-only), like the sampler scratch
    struct {
        DevBuf &r64, &r, &z, &p, &q, &d, &pa, &pb, &small;
    } sb{ctx->s_r64, ctx->s_r, ctx->s_z, ctx->s_p, ctx->s_q, ctx->s_d, ctx->s_pa, ctx->s_pb, ctx->s_small};
    auto fail = [&](int code) { return code; };
    if ((rc = ensure(ctx, sb.r64, 8 * nk, "residual")) || (rc = ensure(ctx, sb.r, tb * nk, "r")) ||
        (rc = ensure(ctx, sb.z, tb * nk, "z")) || (rc = ensure(ctx, sb.p, tb * nk, "p")) ||
        (rc = ensure(ctx, sb.q, tb * nk, "q")) || (rc = ensure(ctx, sb.d, tb * nk, "d")) ||
        (rc = ensure(ctx, sb.pa, 8 * 64 * static_cast<size_t>(max_blocks), "partials")) ||
        (rc = ensure(ctx, sb.pb, 8 * 64 * static_cast<size_t>(max_blocks), "partials")) ||
        (rc = ensure(ctx, sb.small, 8 * (512 + 64 + 64 + 64) + 64, "solver scalars")))
        return fail(rc);
    double *small = static_cast<double *>(sb.small.ptr);
    fc::CgWork w{};
    w.row_ptr = gv.row_ptr;
    w.col_idx = gv.col_idx;
    if (gv.weights) {  // weighted Laplacian: the weights and the weighted degrees
        if ((rc = ensure(ctx, ctx->s_wdeg, 8 * static_cast<size_t>(n), "weighted degrees")))
            return fail(rc);
        FC_HIP(ctx, fc::launch_row_wdeg(gv.row_ptr, gv.weights, gv.n,
                                        static_cast<double *>(ctx->s_wdeg.ptr), ctx->stream),
               "weighted degrees");
        w.weights = gv.weights;
        w.wdeg = static_cast<const double *>(ctx->s_wdeg.ptr);
    }
    w.n = n;
    w.k = k;
    w.alpha = alpha;
    w.max_blocks = max_blocks;
    w.B = B;
    w.X = X;
    w.R64 = static_cast<double *>(sb.r64.ptr);
    w.r = sb.r.ptr;
    w.z = sb.z.ptr;
    w.p = sb.p.ptr;
    w.q = sb.q.ptr;
    w.d = sb.d.ptr;
    w.partial_a = static_cast<double *>(sb.pa.ptr);
    w.partial_b = static_cast<double *>(sb.pb.ptr);
    w.scalars = small;
    w.scale = small + 512;
    w.res_rr = small + 576;
    w.res_bb = small + 640;
    w.any = reinterpret_cast<unsigned int *>(small + 704);

    std::vector<double> rr(k), bb(k), scale(k), tol2(64, 0.0);
    uint32_t total = 0;
    bool first = true, converged = false;
    for (int sweep = 0; sweep < 64; ++sweep) {
        FC_HIP(ctx, fc::cg_residual(w, first, ctx->stream), "residual");
        FC_HIP(ctx, hipMemcpyAsync(rr.data(), w.res_rr, 8 * k, hipMemcpyDeviceToHost, ctx->stream), "copy");
        if (first)
            FC_HIP(ctx, hipMemcpyAsync(bb.data(), w.res_bb, 8 * k, hipMemcpyDeviceToHost, ctx->stream),
                   "copy");
        FC_HIP(ctx, hipStreamSynchronize(ctx->stream), "residual");
        first = false;
        converged = true;
        for (uint32_t j = 0; j < k; ++j) {
            const double rel = bb[j] > 0.0 ? std::sqrt(rr[j] / bb[j]) : std::sqrt(rr[j]);
            if (relres_out) relres_out[j] = rel;
            const bool done = rel <= rtol;
            converged = converged && done;
            scale[j] = done ? 0.0 : std::sqrt(rr[j]);
            // inner target: binary32 gains about five digits per sweep (its
            // recurrence stays trustworthy down to ~1e-6 on a unit residual);
            // binary64 aims straight at the outer tolerance (with a safety factor)
            const double target = fp32 ? 1e-5
                                       : std::max(1e-300, 0.5 * rtol * std::sqrt(bb[j]) / std::sqrt(rr[j]));
            tol2[j] = done ? 0.0 : target * target;
        }
        if (converged || total >= static_cast<uint32_t>(max_iters)) break;
        FC_HIP(ctx, hipMemcpyAsync(w.scale, scale.data(), 8 * k, hipMemcpyHostToDevice, ctx->stream),
               "copy scale");
        FC_HIP(ctx, hipMemcpyAsync(small + 256, tol2.data(), 8 * 64, hipMemcpyHostToDevice, ctx->stream),
               "copy tolerances");
        uint32_t it = 0;
        const uint32_t budget = static_cast<uint32_t>(max_iters) - total;
        hipError_t e = fp32 ? fc::cg_inner<float>(w, budget, 8, &it, ctx->stream)
                            : fc::cg_inner<double>(w, budget, 8, &it, ctx->stream);
        if (e != hipSuccess) return fail(hip_fail(ctx, e, "inner CG"));
        total += it;
    }
    FC_HIP(ctx, hipStreamSynchronize(ctx->stream), "solve");
    if (iters_out) *iters_out = static_cast<int32_t>(total);
    return FC_OK;
}
