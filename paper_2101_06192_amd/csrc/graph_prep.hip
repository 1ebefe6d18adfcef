// CSR validation and the per-vertex records of the augmented graph G*.
//
// G* (Section 4.1 of the paper) is never materialised: u* is the id n, the
// edges {u*, v} are implicit, and a walk leaves v to u* with probability
// 1 / (1 + alpha d_v) (edge weight 1 against d_v edges of weight alpha).
#include "fc_kernels.hpp"

#pragma clang fp contract(off)

namespace fc {

namespace {

__global__ void validate_rows_kernel(const int32_t *__restrict__ row_ptr, int32_t n, int64_t nnz,
                                     unsigned int *err) {
    const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v > n) return;
    const int64_t a = row_ptr[v];
    bool bad = a < 0 || a > nnz;
    if (v == 0) bad |= (a != 0);
    if (v == n) bad |= (a != nnz);
    if (v < n) bad |= (row_ptr[v + 1] < a);
    if (bad) atomicOr(err, kErrGraphRowPtr);
}

// Edge-parallel: each thread checks kColChunk consecutive CSR entries.  It
// finds the row of its first entry by binary search over row_ptr, then walks
// rows forward; every entry is checked for range, self-loop, strict order
// against the previous entry of its row, and symmetry by binary search of the
// row vertex in the row of the neighbour (rows are sorted, which this kernel
// also checks).  Work is proportional to nnz whatever the degree spread.
constexpr int64_t kColChunk = 16;

__global__ void validate_cols_kernel(const int32_t *__restrict__ row_ptr,
                                     const int32_t *__restrict__ col_idx,
                                     const double *__restrict__ weights, int32_t n, int64_t nnz,
                                     unsigned int *err) {
    const int64_t e0 = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) * kColChunk;
    if (e0 >= nnz) return;
    const int64_t e1 = e0 + kColChunk < nnz ? e0 + kColChunk : nnz;
    // row v with row_ptr[v] <= e0 < row_ptr[v + 1] (row_ptr is monotone: pass 1)
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo + 1) >> 1);
        if (row_ptr[mid] <= e0) lo = mid;
        else hi = mid - 1;
    }
    int32_t v = lo;
    int64_t row_end = row_ptr[v + 1];
    unsigned int e = 0;
    for (int64_t j = e0; j < e1; ++j) {
        while (j >= row_end) {  // skip to the row holding entry j (empty rows included)
            ++v;
            row_end = row_ptr[v + 1];
        }
        const int32_t u = col_idx[j];
        if (u < 0 || u >= n) {
            e |= kErrGraphColumn;
            continue;
        }
        if (u == v) e |= kErrGraphSelfLoop;
        if (j > row_ptr[v] && col_idx[j - 1] >= u) e |= kErrGraphOrder;
        int32_t a = row_ptr[u], b = row_ptr[u + 1];
        while (a < b) {
            const int32_t mid = a + ((b - a) >> 1);
            if (col_idx[mid] < v) a = mid + 1;
            else b = mid;
        }
        if (a >= row_ptr[u + 1] || col_idx[a] != v) {
            e |= kErrGraphAsymmetric;
            continue;
        }
        if (weights) {  // 0 or in [2^-64, 2^64] (NaN fails both), equal to the reverse entry's
            const double w = weights[j];
            if (!(w == 0.0 || (w >= 0x1p-64 && w <= 0x1p64))) e |= kErrGraphWeight;
            if (!(weights[a] == w)) e |= kErrGraphWeightAsym;
        }
    }
    if (e) atomicOr(err, e);
}

// thr(d) = floor(2^32 * (1 / ((alpha * d) + 1))), each operation rounded to
// binary64 (IEEE division; no contraction in this file).
// The weighted threshold is the same expression in the weighted degree W
// (an integer d is exact in binary64, so W = d gives thr(d)).
__device__ __forceinline__ unsigned long long root_threshold_w(double alpha, double W) {
    if (W == 0.0) return 1ull << 32;
    const double aw = alpha * W;
    const double den = aw + 1.0;
    const double p = 1.0 / den;
    return static_cast<unsigned long long>(p * 4294967296.0);
}
__device__ __forceinline__ unsigned long long root_threshold(double alpha, uint32_t d) {
    return root_threshold_w(alpha, static_cast<double>(d));
}

// One thread per row; the sum is sequential by definition (its rounding is
// part of the randomness contract), so rows are not split.
__global__ void row_wsum_kernel(const int32_t *__restrict__ row_ptr,
                                const double *__restrict__ weights, int32_t n,
                                double *__restrict__ S) {
    const int32_t v = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (v >= n) return;
    const int32_t b = row_ptr[v], e = row_ptr[v + 1];
    double s = 0.0;
#pragma unroll 8
    for (int32_t q = b; q < e; ++q) {
        s += weights[q];
        S[q] = s;
    }
}

// Step thresholds: entry-parallel like the column check (kColChunk entries
// per thread, the row of the first found by binary search over row_ptr).
__global__ void step_thr_kernel(const int32_t *__restrict__ row_ptr, const double *__restrict__ S,
                                int32_t n, int64_t nnz, uint32_t *__restrict__ T) {
    const int64_t e0 = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) * kColChunk;
    if (e0 >= nnz) return;
    const int64_t e1 = e0 + kColChunk < nnz ? e0 + kColChunk : nnz;
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo + 1) >> 1);
        if (row_ptr[mid] <= e0) lo = mid;
        else hi = mid - 1;
    }
    int32_t v = lo;
    int64_t row_end = row_ptr[v + 1];
    for (int64_t j = e0; j < e1; ++j) {
        while (j >= row_end) {
            ++v;
            row_end = row_ptr[v + 1];
        }
        const double W = S[row_end - 1], s = S[j];
        // smallest x in [0, 2^32] with (x * W) * 2^-32 >= s (x = 2^32 gives W >= s)
        uint64_t a = 0, b = 1ull << 32;
        while (a < b) {
            const uint64_t mid = (a + b) >> 1;
            if ((static_cast<double>(mid) * W) * 0x1p-32 >= s) b = mid;
            else a = mid + 1;
        }
        T[j] = static_cast<uint32_t>(a < 1 ? 1 : a > 0xFFFFFFFFull ? 0xFFFFFFFFull : a);
    }
}

__global__ void row_wdeg_kernel(const int32_t *__restrict__ row_ptr,
                                const double *__restrict__ weights, int32_t n,
                                double *__restrict__ W) {
    const int32_t v = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (v >= n) return;
    const int32_t b = row_ptr[v], e = row_ptr[v + 1];
    double s = 0.0;
#pragma unroll 8
    for (int32_t q = b; q < e; ++q) s += weights[q];
    W[v] = s;
}

__global__ void build_vrec_kernel(const int32_t *__restrict__ row_ptr,
                                  const double *__restrict__ S, int32_t n, double alpha,
                                  VRec *__restrict__ vrec, unsigned int *dmax,
                                  uint32_t *__restrict__ iso, double *wtotal) {
    const int32_t v = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    uint32_t d = 0;
    int32_t a = 0;
    if (v < n) {
        a = row_ptr[v];
        d = static_cast<uint32_t>(row_ptr[v + 1] - a);
    }
    uint32_t m = d;  // maximum degree: wave reduction, one atomic per wave
    for (int off = 32; off > 0; off >>= 1) m = max(m, static_cast<uint32_t>(__shfl_down(m, off, 64)));
    if ((threadIdx.x & 63u) == 0 && m) atomicMax(dmax, m);
    if (iso) {  // 64 vertices per wave: two bitmap words (blocks are whole waves)
        const uint64_t bits = __ballot(v < n && d == 0);
        const int32_t w0 = static_cast<int32_t>((blockIdx.x * blockDim.x + (threadIdx.x & ~63u)) >> 5);
        const int32_t nw = (n + 31) >> 5;
        if ((threadIdx.x & 63u) == 0 && w0 < nw) iso[w0] = static_cast<uint32_t>(bits);
        if ((threadIdx.x & 63u) == 32 && w0 + 1 < nw) iso[w0 + 1] = static_cast<uint32_t>(bits >> 32);
    }
    const double W = S && d ? S[a + static_cast<int32_t>(d) - 1] : 0.0;
    if (S && wtotal) {  // sum of the weighted degrees (bounds the expected walk length)
        double sw = W;
        for (int off = 32; off > 0; off >>= 1) sw += __shfl_down(sw, off, 64);
        if ((threadIdx.x & 63u) == 0 && sw > 0.0) atomicAdd(wtotal, sw);
    }
    if (v >= n) return;
    const unsigned long long t = S ? root_threshold_w(alpha, W) : root_threshold(alpha, d);
    VRec r;
    r.start = a;
    r.deg = d;
    r.thr = static_cast<uint32_t>(t);
    r.always_root = (t >> 32) ? 1u : 0u;
    vrec[v] = r;
}

__global__ void thresholds_kernel(double alpha, int32_t d_max, unsigned long long *out) {
    const int32_t d = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (d > d_max) return;
    out[d] = root_threshold(alpha, static_cast<uint32_t>(d));
}

inline unsigned int blocks_for(int64_t items, int threads) {
    return static_cast<unsigned int>((items + threads - 1) / threads);
}

}  // namespace

hipError_t launch_validate_rows(const int32_t *row_ptr, int32_t n, int64_t nnz,
                                unsigned int *err, hipStream_t stream) {
    validate_rows_kernel<<<blocks_for(static_cast<int64_t>(n) + 1, 256), 256, 0, stream>>>(
        row_ptr, n, nnz, err);
    return hipGetLastError();
}

hipError_t launch_validate_cols(const int32_t *row_ptr, const int32_t *col_idx,
                                const double *weights, int32_t n, int64_t nnz, unsigned int *err,
                                hipStream_t stream) {
    if (n == 0 || nnz == 0) return hipSuccess;
    validate_cols_kernel<<<blocks_for((nnz + kColChunk - 1) / kColChunk, 256), 256, 0, stream>>>(
        row_ptr, col_idx, weights, n, nnz, err);
    return hipGetLastError();
}

hipError_t launch_row_wsum(const int32_t *row_ptr, const double *weights, int32_t n, double *S,
                           hipStream_t stream) {
    if (n == 0) return hipSuccess;
    row_wsum_kernel<<<blocks_for(n, 256), 256, 0, stream>>>(row_ptr, weights, n, S);
    return hipGetLastError();
}

hipError_t launch_step_thresholds(const int32_t *row_ptr, const double *S, int32_t n,
                                  int64_t nnz, uint32_t *T, hipStream_t stream) {
    if (n == 0 || nnz == 0) return hipSuccess;
    step_thr_kernel<<<blocks_for((nnz + kColChunk - 1) / kColChunk, 256), 256, 0, stream>>>(
        row_ptr, S, n, nnz, T);
    return hipGetLastError();
}

hipError_t launch_row_wdeg(const int32_t *row_ptr, const double *weights, int32_t n, double *W,
                           hipStream_t stream) {
    if (n == 0) return hipSuccess;
    row_wdeg_kernel<<<blocks_for(n, 256), 256, 0, stream>>>(row_ptr, weights, n, W);
    return hipGetLastError();
}

hipError_t launch_build_vrec(const int32_t *row_ptr, const double *S, int32_t n, double alpha,
                             VRec *vrec, unsigned int *dmax, uint32_t *iso, double *wtotal,
                             hipStream_t stream) {
    if (n == 0) return hipSuccess;
    build_vrec_kernel<<<blocks_for(n, 256), 256, 0, stream>>>(row_ptr, S, n, alpha, vrec, dmax,
                                                              iso, wtotal);
    return hipGetLastError();
}

hipError_t launch_thresholds(double alpha, int32_t d_max, unsigned long long *out,
                             hipStream_t stream) {
    thresholds_kernel<<<blocks_for(static_cast<int64_t>(d_max) + 1, 256), 256, 0, stream>>>(
        alpha, d_max, out);
    return hipGetLastError();
}

}  // namespace fc
