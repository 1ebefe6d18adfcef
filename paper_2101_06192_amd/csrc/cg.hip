// Block conjugate gradients for (alpha L + I) X = B with up to 64 right-hand
// sides (the linear system of Algorithm 1, and the CG ground truth of the
// paper's experiments).  All vectors are row-major n x k (row v holds the k
// values of vertex v), so a neighbour row is one contiguous, coalesced load.
//
// Mapping: a wave covers 64 / kk rows (kk = k rounded up to a power of two),
// lane = (row-in-wave, column).  Per-column dot products are reduced in two
// deterministic stages: each block writes its partial sums, then one block
// adds the partials in a fixed order.  Per-column CG scalars live on the
// device; the host only polls a convergence flag.
#include "fc_kernels.hpp"

#pragma clang fp contract(off)

namespace fc {

namespace {

constexpr int kThreads = 256;

struct Lane {
    uint32_t kk;     // columns per row group (power of two, <= 64)
    uint32_t rsub;   // row within the wave's group
    uint32_t col;    // column of this lane
    bool valid;      // col < k
};

__device__ __forceinline__ Lane lane_map(uint32_t k) {
    uint32_t kk = 1;
    while (kk < k) kk <<= 1;
    const uint32_t lane = threadIdx.x & 63u;
    return {kk, lane / kk, lane % kk, (lane % kk) < k};
}

// Rows handled by a wave: group g covers rows g * (64/kk) .. + 64/kk - 1.
__device__ __forceinline__ void row_range(uint32_t kk, uint32_t *first_group, uint32_t *stride) {
    const uint32_t waves_per_block = blockDim.x / 64u;
    *first_group = blockIdx.x * waves_per_block + (threadIdx.x >> 6);
    *stride = gridDim.x * waves_per_block;
    (void)kk;
}

// sum over the neighbours u of v of X[u][col] (kWeighted: of w_vu X[u][col],
// the off-diagonal of the weighted Laplacian), eight independent gathers in
// flight (fixed association: deterministic).
template <typename T, bool kWeighted>
__device__ __forceinline__ T neighbour_sum(const int32_t *__restrict__ col_idx,
                                           const double *__restrict__ wt, int32_t b, int32_t e,
                                           const T *__restrict__ X, uint32_t k, uint32_t col) {
    constexpr int U = 8;
    T s[U];
#pragma unroll
    for (int i = 0; i < U; ++i) s[i] = T(0);
    int32_t q = b;
    for (; q + U <= e; q += U) {
        int32_t u[U];
#pragma unroll
        for (int i = 0; i < U; ++i) u[i] = col_idx[q + i];
        if (kWeighted) {
            T c[U];
#pragma unroll
            for (int i = 0; i < U; ++i) c[i] = static_cast<T>(wt[q + i]);
#pragma unroll
            for (int i = 0; i < U; ++i) s[i] += c[i] * X[static_cast<size_t>(u[i]) * k + col];
        } else {
#pragma unroll
            for (int i = 0; i < U; ++i) s[i] += X[static_cast<size_t>(u[i]) * k + col];
        }
    }
    for (int i = 0; q < e; ++q, ++i) {
        const T xu = X[static_cast<size_t>(col_idx[q]) * k + col];
        s[i] += kWeighted ? static_cast<T>(wt[q]) * xu : xu;
    }
    return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// Diagonal of L at v: the degree, or the weighted degree wdeg[v] when given.
__device__ __forceinline__ double degree_of(const int32_t *__restrict__ row_ptr,
                                            const double *__restrict__ wdeg, uint32_t v) {
    return wdeg ? wdeg[v] : static_cast<double>(row_ptr[v + 1] - row_ptr[v]);
}

// Block-level per-column reduction of `acc` into partial[blockIdx.x * k + col].
template <typename A>
__device__ __forceinline__ void block_column_sum(A acc, const Lane &ln, uint32_t k, A *partial,
                                                 A *lds) {
    lds[threadIdx.x] = ln.valid ? acc : A(0);
    __syncthreads();
    if (threadIdx.x < k) {
        A s = A(0);
        // threads with the same column: lanes col, col + kk, ... in every wave
        for (uint32_t t = threadIdx.x; t < blockDim.x; t += ln.kk) s += lds[t];
        partial[static_cast<size_t>(blockIdx.x) * k + threadIdx.x] = s;
    }
    __syncthreads();
}

// Y = A X with A = alpha L + I; optional partial dots sum_v X[v][j] Y[v][j].
template <typename T, bool kWeighted>
__global__ __launch_bounds__(kThreads) void apply_kernel(const int32_t *__restrict__ row_ptr,
                                                         const int32_t *__restrict__ col_idx,
                                                         const double *__restrict__ wt,
                                                         const double *__restrict__ wdeg,
                                                         uint32_t n, uint32_t k, double alpha,
                                                         const T *__restrict__ X, T *__restrict__ Y,
                                                         double *__restrict__ partial) {
    __shared__ double lds[kThreads];
    const Lane ln = lane_map(k);
    const uint32_t rows_per_group = 64u / ln.kk;
    uint32_t g0, gs;
    row_range(ln.kk, &g0, &gs);
    const T a = static_cast<T>(alpha);
    double acc = 0.0;
    for (uint32_t g = g0; static_cast<size_t>(g) * rows_per_group < n; g += gs) {
        const uint32_t v = g * rows_per_group + ln.rsub;
        if (v < n && ln.valid) {
            const int32_t b = row_ptr[v], e = row_ptr[v + 1];
            const T s = neighbour_sum<T, kWeighted>(col_idx, wt, b, e, X, k, ln.col);
            const T x = X[static_cast<size_t>(v) * k + ln.col];
            const T d = kWeighted ? static_cast<T>(wdeg[v]) : static_cast<T>(e - b);
            const T y = (T(1) + a * d) * x - a * s;
            Y[static_cast<size_t>(v) * k + ln.col] = y;
            acc += static_cast<double>(x) * static_cast<double>(y);
        }
    }
    if (partial) block_column_sum(acc, ln, k, partial, lds);
}

// R = B - A X in binary64; partial sums of R_j . R_j (and of B_j . B_j).
template <bool kWeighted>
__global__ __launch_bounds__(kThreads) void residual_kernel(const int32_t *__restrict__ row_ptr,
                                                            const int32_t *__restrict__ col_idx,
                                                            const double *__restrict__ wt,
                                                            const double *__restrict__ wdeg,
                                                            uint32_t n, uint32_t k, double alpha,
                                                            const double *__restrict__ B,
                                                            const double *__restrict__ X,
                                                            double *__restrict__ R,
                                                            double *__restrict__ partial_rr,
                                                            double *__restrict__ partial_bb) {
    __shared__ double lds[kThreads];
    const Lane ln = lane_map(k);
    const uint32_t rows_per_group = 64u / ln.kk;
    uint32_t g0, gs;
    row_range(ln.kk, &g0, &gs);
    double rr = 0.0, bb = 0.0;
    for (uint32_t g = g0; static_cast<size_t>(g) * rows_per_group < n; g += gs) {
        const uint32_t v = g * rows_per_group + ln.rsub;
        if (v < n && ln.valid) {
            const int32_t b = row_ptr[v], e = row_ptr[v + 1];
            const double s = neighbour_sum<double, kWeighted>(col_idx, wt, b, e, X, k, ln.col);
            const size_t i = static_cast<size_t>(v) * k + ln.col;
            const double dv = kWeighted ? wdeg[v] : static_cast<double>(e - b);
            const double ax = (1.0 + alpha * dv) * X[i] - alpha * s;
            const double r = B[i] - ax;
            R[i] = r;
            rr += r * r;
            bb += B[i] * B[i];
        }
    }
    block_column_sum(rr, ln, k, partial_rr, lds);
    if (partial_bb) block_column_sum(bb, ln, k, partial_bb, lds);
}

// out[j] = sum over blocks of partial[b * k + j] in a fixed order (deterministic):
// thread (g, j) of kReduceGroups groups sums blocks b = g (mod kReduceGroups) in
// four interleaved accumulators, then group sums are added in group order.
constexpr int kReduceGroups = 16;
__global__ __launch_bounds__(64 * kReduceGroups) void reduce_kernel(const double *__restrict__ partial,
                                                                   uint32_t blocks, uint32_t k,
                                                                   double *__restrict__ out) {
    __shared__ double s_sum[kReduceGroups][64];
    const uint32_t j = threadIdx.x & 63u, g = threadIdx.x >> 6;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (j < k) {
        constexpr uint32_t G = kReduceGroups;
        uint32_t b = g;
        for (; b + 3u * G < blocks; b += 4u * G) {
            a0 += partial[static_cast<size_t>(b) * k + j];
            a1 += partial[static_cast<size_t>(b + G) * k + j];
            a2 += partial[static_cast<size_t>(b + 2u * G) * k + j];
            a3 += partial[static_cast<size_t>(b + 3u * G) * k + j];
        }
        for (; b < blocks; b += G) a0 += partial[static_cast<size_t>(b) * k + j];
    }
    s_sum[g][j] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (g == 0 && j < k) {
        double t = 0.0;
        for (uint32_t q = 0; q < kReduceGroups; ++q) t += s_sum[q][j];
        out[j] = t;
    }
}

// Inner CG start on the scaled residual: r = R64 / scale_j (as T), d = 0,
// z = Minv r, p = z; partial sums of r.z.
template <typename T>
__global__ __launch_bounds__(kThreads) void start_kernel(const int32_t *__restrict__ row_ptr,
                                                         const double *__restrict__ wdeg,
                                                         uint32_t n, uint32_t k, double alpha,
                                                         const double *__restrict__ R64,
                                                         const double *__restrict__ scale,
                                                         T *__restrict__ r, T *__restrict__ z,
                                                         T *__restrict__ p, T *__restrict__ d,
                                                         double *__restrict__ partial,
                                                         double *__restrict__ partial_rr) {
    __shared__ double lds[kThreads];
    const Lane ln = lane_map(k);
    const uint32_t rows_per_group = 64u / ln.kk;
    uint32_t g0, gs;
    row_range(ln.kk, &g0, &gs);
    double acc = 0.0, rr = 0.0;
    for (uint32_t g = g0; static_cast<size_t>(g) * rows_per_group < n; g += gs) {
        const uint32_t v = g * rows_per_group + ln.rsub;
        if (v < n && ln.valid) {
            const size_t i = static_cast<size_t>(v) * k + ln.col;
            const double sc = scale[ln.col];
            const T rv = static_cast<T>(sc > 0.0 ? R64[i] / sc : 0.0);
            const T minv = static_cast<T>(1.0 / (1.0 + alpha * degree_of(row_ptr, wdeg, v)));
            const T zv = minv * rv;
            r[i] = rv;
            z[i] = zv;
            p[i] = zv;
            d[i] = T(0);
            acc += static_cast<double>(rv) * static_cast<double>(zv);
            rr += static_cast<double>(rv) * static_cast<double>(rv);
        }
    }
    block_column_sum(acc, ln, k, partial, lds);
    block_column_sum(rr, ln, k, partial_rr, lds);
}

// d += a_j p; r -= a_j q; z = Minv r; partial sums of r.z and r.r.
template <typename T>
__global__ __launch_bounds__(kThreads) void update_kernel(const int32_t *__restrict__ row_ptr,
                                                          const double *__restrict__ wdeg,
                                                          uint32_t n, uint32_t k, double alpha,
                                                          const double *__restrict__ step,
                                                          const T *__restrict__ p,
                                                          const T *__restrict__ q, T *__restrict__ d,
                                                          T *__restrict__ r, T *__restrict__ z,
                                                          double *__restrict__ partial_rz,
                                                          double *__restrict__ partial_rr) {
    __shared__ double lds[kThreads];
    const Lane ln = lane_map(k);
    const uint32_t rows_per_group = 64u / ln.kk;
    uint32_t g0, gs;
    row_range(ln.kk, &g0, &gs);
    const T a = ln.valid ? static_cast<T>(step[ln.col]) : T(0);
    double rz = 0.0, rr = 0.0;
    for (uint32_t g = g0; static_cast<size_t>(g) * rows_per_group < n; g += gs) {
        const uint32_t v = g * rows_per_group + ln.rsub;
        if (v < n && ln.valid) {
            const size_t i = static_cast<size_t>(v) * k + ln.col;
            d[i] = d[i] + a * p[i];
            const T rv = r[i] - a * q[i];
            const T minv = static_cast<T>(1.0 / (1.0 + alpha * degree_of(row_ptr, wdeg, v)));
            const T zv = minv * rv;
            r[i] = rv;
            z[i] = zv;
            rz += static_cast<double>(rv) * static_cast<double>(zv);
            rr += static_cast<double>(rv) * static_cast<double>(rv);
        }
    }
    block_column_sum(rz, ln, k, partial_rz, lds);
    block_column_sum(rr, ln, k, partial_rr, lds);
}

// p = z + b_j p
template <typename T>
__global__ __launch_bounds__(kThreads) void direction_kernel(uint32_t n, uint32_t k,
                                                             const double *__restrict__ beta,
                                                             const T *__restrict__ z,
                                                             T *__restrict__ p) {
    const Lane ln = lane_map(k);
    const uint32_t rows_per_group = 64u / ln.kk;
    uint32_t g0, gs;
    row_range(ln.kk, &g0, &gs);
    const T b = ln.valid ? static_cast<T>(beta[ln.col]) : T(0);
    for (uint32_t g = g0; static_cast<size_t>(g) * rows_per_group < n; g += gs) {
        const uint32_t v = g * rows_per_group + ln.rsub;
        if (v < n && ln.valid) {
            const size_t i = static_cast<size_t>(v) * k + ln.col;
            p[i] = z[i] + b * p[i];
        }
    }
}

// X += scale_j * d (binary64 refinement update)
template <typename T>
__global__ __launch_bounds__(kThreads) void correct_kernel(uint32_t n, uint32_t k,
                                                           const double *__restrict__ scale,
                                                           const T *__restrict__ d,
                                                           double *__restrict__ X) {
    const Lane ln = lane_map(k);
    const uint32_t rows_per_group = 64u / ln.kk;
    uint32_t g0, gs;
    row_range(ln.kk, &g0, &gs);
    const double sc = ln.valid ? scale[ln.col] : 0.0;
    for (uint32_t g = g0; static_cast<size_t>(g) * rows_per_group < n; g += gs) {
        const uint32_t v = g * rows_per_group + ln.rsub;
        if (v < n && ln.valid) {
            const size_t i = static_cast<size_t>(v) * k + ln.col;
            X[i] = X[i] + sc * static_cast<double>(d[i]);
        }
    }
}

// Per-column CG scalars (one block, thread j = column j).
//   mode 0 (after start):  rz_j = rzn_j; active_j = rz_j > 0
//   mode 1 (after A p):    step_j = active ? rz_j / pq_j : 0
//   mode 2 (after update): beta_j = active ? rzn_j / rz_j : 0; rz_j = rzn_j;
//                          active_j &= rr_j > tol2_j; *any = any active column
__global__ void scalars_kernel(int mode, uint32_t k, double *__restrict__ s, unsigned int *any) {
    const uint32_t j = threadIdx.x;
    double *rz = s, *rzn = s + 64, *pq = s + 128, *rr = s + 192, *tol2 = s + 256, *step = s + 320,
           *beta = s + 384, *active = s + 448;
    __shared__ unsigned int s_any;
    if (j == 0) s_any = 0;
    __syncthreads();
    if (j < k) {
        if (mode == 0) {
            rz[j] = rzn[j];
            active[j] = (rz[j] > 0.0 && rr[j] > tol2[j]) ? 1.0 : 0.0;
        } else if (mode == 1) {
            step[j] = (active[j] != 0.0 && pq[j] > 0.0) ? rz[j] / pq[j] : 0.0;
        } else {
            beta[j] = (active[j] != 0.0 && rz[j] > 0.0) ? rzn[j] / rz[j] : 0.0;
            rz[j] = rzn[j];
            if (!(rr[j] > tol2[j])) active[j] = 0.0;
        }
        if (active[j] != 0.0) atomicOr(&s_any, 1u);
    }
    __syncthreads();
    if (j == 0 && any) *any = s_any;
}

inline unsigned int grid_for(uint32_t n, uint32_t k, uint32_t max_blocks) {
    uint32_t kk = 1;
    while (kk < k) kk <<= 1;
    const size_t groups = (static_cast<size_t>(n) + (64 / kk) - 1) / (64 / kk);
    size_t blocks = (groups + (kThreads / 64) - 1) / (kThreads / 64);
    if (blocks > max_blocks) blocks = max_blocks;
    if (blocks < 1) blocks = 1;
    return static_cast<unsigned int>(blocks);
}

}  // namespace

// Solve state: scalars (8 x 64 doubles) and partial-sum buffers are owned by
// the caller; see CgWork in fc_kernels.hpp.
template <typename T>
hipError_t cg_inner(const CgWork &w, uint32_t max_iters, uint32_t poll, uint32_t *iters,
                    hipStream_t stream) {
    const uint32_t n = w.n, k = w.k;
    const unsigned int blocks = grid_for(n, k, w.max_blocks);
    T *r = static_cast<T *>(w.r), *z = static_cast<T *>(w.z), *p = static_cast<T *>(w.p),
      *q = static_cast<T *>(w.q), *d = static_cast<T *>(w.d);
    double *S = w.scalars;
    double *rz = S, *rzn = S + 64, *pq = S + 128, *rr = S + 192, *step = S + 320, *beta = S + 384;
    (void)rz;
    hipError_t e;
    // start: r = R64 / scale, z = Minv r, p = z, d = 0; rz = r.z; rr = |r|^2
    start_kernel<T><<<blocks, kThreads, 0, stream>>>(w.row_ptr, w.wdeg, n, k, w.alpha, w.R64,
                                                     w.scale, r, z, p, d, w.partial_a, w.partial_b);
    reduce_kernel<<<1, 64 * kReduceGroups, 0, stream>>>(w.partial_a, blocks, k, rzn);
    reduce_kernel<<<1, 64 * kReduceGroups, 0, stream>>>(w.partial_b, blocks, k, rr);
    scalars_kernel<<<1, 64, 0, stream>>>(0, k, S, w.any);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    uint32_t it = 0;
    while (it < max_iters) {
        if (w.weights)
            apply_kernel<T, true><<<blocks, kThreads, 0, stream>>>(w.row_ptr, w.col_idx, w.weights,
                                                                   w.wdeg, n, k, w.alpha, p, q,
                                                                   w.partial_a);
        else
            apply_kernel<T, false><<<blocks, kThreads, 0, stream>>>(w.row_ptr, w.col_idx, nullptr,
                                                                    nullptr, n, k, w.alpha, p, q,
                                                                    w.partial_a);
        reduce_kernel<<<1, 64 * kReduceGroups, 0, stream>>>(w.partial_a, blocks, k, pq);
        scalars_kernel<<<1, 64, 0, stream>>>(1, k, S, nullptr);
        update_kernel<T><<<blocks, kThreads, 0, stream>>>(w.row_ptr, w.wdeg, n, k, w.alpha, step, p,
                                                          q, d, r, z, w.partial_a, w.partial_b);
        reduce_kernel<<<1, 64 * kReduceGroups, 0, stream>>>(w.partial_a, blocks, k, rzn);
        reduce_kernel<<<1, 64 * kReduceGroups, 0, stream>>>(w.partial_b, blocks, k, rr);
        scalars_kernel<<<1, 64, 0, stream>>>(2, k, S, w.any);
        direction_kernel<T><<<blocks, kThreads, 0, stream>>>(n, k, beta, z, p);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        ++it;
        if (it % poll == 0 || it == max_iters) {
            unsigned int any = 0;
            if ((e = hipMemcpyAsync(&any, w.any, sizeof(any), hipMemcpyDeviceToHost, stream)) != hipSuccess)
                return e;
            if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
            if (!any) break;
        }
    }
    correct_kernel<T><<<blocks, kThreads, 0, stream>>>(n, k, w.scale, d, w.X);
    *iters = it;
    return hipGetLastError();
}

template hipError_t cg_inner<float>(const CgWork &, uint32_t, uint32_t, uint32_t *, hipStream_t);
template hipError_t cg_inner<double>(const CgWork &, uint32_t, uint32_t, uint32_t *, hipStream_t);

hipError_t cg_residual(const CgWork &w, bool with_b, hipStream_t stream) {
    const unsigned int blocks = grid_for(w.n, w.k, w.max_blocks);
    if (w.weights)
        residual_kernel<true><<<blocks, kThreads, 0, stream>>>(
            w.row_ptr, w.col_idx, w.weights, w.wdeg, w.n, w.k, w.alpha, w.B, w.X, w.R64,
            w.partial_a, with_b ? w.partial_b : nullptr);
    else
        residual_kernel<false><<<blocks, kThreads, 0, stream>>>(
            w.row_ptr, w.col_idx, nullptr, nullptr, w.n, w.k, w.alpha, w.B, w.X, w.R64,
            w.partial_a, with_b ? w.partial_b : nullptr);
    reduce_kernel<<<1, 64 * kReduceGroups, 0, stream>>>(w.partial_a, blocks, w.k, w.res_rr);
    if (with_b) reduce_kernel<<<1, 64 * kReduceGroups, 0, stream>>>(w.partial_b, blocks, w.k, w.res_bb);
    return hipGetLastError();
}

}  // namespace fc
