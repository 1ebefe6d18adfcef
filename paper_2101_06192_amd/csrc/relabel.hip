// Degree-class relabelling for the LDS-counter sampler.
//
// That sampler keeps the in-arrow count of every vertex of a tree in LDS.  A
// count never exceeds the vertex degree, so a vertex of degree d gets a field
// of 4 << c bits, c = class(d): 4 bits up to degree 15, 8 up to 255, 16 up to
// 65535, else 32.  Isolated vertices form a fifth class with no field: they
// are never a target, and in every tree they are roots after one draw.
// Vertices are renumbered so that each class is a contiguous range of
// internal ids (class 0 first, isolated vertices last; original order kept
// inside a class), which makes a field's LDS word and shift plain arithmetic
// on the internal id.  Randomness and every output stay on original ids: the relabelled
// vertex record carries the original id, and the relabelled adjacency holds
// (internal, original) pairs of each neighbour at the same CSR positions
// (internal id in the low bits, original id shifted by 18 for the LDS sampler
// or 32 for the hybrid one), so the neighbour chosen by a draw is the one the
// original CSR gives.
#include "fc_kernels.hpp"

namespace fc {

namespace {

constexpr int kPlaceThreads = 1024;
constexpr uint32_t kClasses = kRelabelClasses;  // four field widths, then isolated vertices

__device__ __forceinline__ uint32_t deg_class(uint32_t d) {
    return d == 0u ? 4u : d <= 15u ? 0u : d <= 255u ? 1u : d <= 65535u ? 2u : 3u;
}

// Per block of kPlaceThreads vertices: how many fall in each class.
__global__ __launch_bounds__(kPlaceThreads) void class_count_kernel(
    const int32_t *__restrict__ row_ptr, uint32_t n, uint32_t *__restrict__ blk) {
    __shared__ uint32_t s[kClasses];
    if (threadIdx.x < kClasses) s[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t v = blockIdx.x * kPlaceThreads + threadIdx.x;
    const uint32_t c =
        v < n ? deg_class(static_cast<uint32_t>(row_ptr[v + 1] - row_ptr[v])) : kClasses;
    for (uint32_t k = 0; k < kClasses; ++k) {
        const uint64_t m = __ballot(c == k);
        if ((threadIdx.x & 63u) == 0 && m) atomicAdd(&s[k], static_cast<uint32_t>(__popcll(m)));
    }
    __syncthreads();
    if (threadIdx.x < kClasses) blk[blockIdx.x * kClasses + threadIdx.x] = s[threadIdx.x];
}

// Rank of class c in the id order: narrowest field first (LDS sampler) or
// widest first (hybrid sampler, whose LDS holds a prefix of the ids: the
// highest-degree vertices, which receive most arrows); isolated vertices last.
__device__ __forceinline__ uint32_t class_rank(uint32_t c, bool widest_first) {
    return c == 4u || !widest_first ? c : 3u - c;
}

// One block of kClasses threads, thread k serial over the blocks of class k:
// base[b][k] = first internal id of class k in block b; bounds[r] = end of the
// class of rank r, r < 4 (bounds[3] = number of vertices that are not
// isolated).
__global__ void class_scan_kernel(const uint32_t *__restrict__ blk, uint32_t nb, int widest_first,
                                  uint32_t *__restrict__ base, uint32_t *__restrict__ bounds) {
    __shared__ uint32_t tot[kClasses];
    const uint32_t k = threadIdx.x;
    uint32_t s = 0;
    for (uint32_t b = 0; b < nb; ++b) s += blk[b * kClasses + k];
    tot[class_rank(k, widest_first)] = s;
    __syncthreads();
    const uint32_t r = class_rank(k, widest_first);
    uint32_t start = 0;
    for (uint32_t j = 0; j < r; ++j) start += tot[j];
    if (r + 1 < kClasses) bounds[r] = start + tot[r];
    for (uint32_t b = 0; b < nb; ++b) {
        base[b * kClasses + k] = start;
        start += blk[b * kClasses + k];
    }
}

// inv[v] = internal id of v, orig[internal] = v: rank inside the block from
// per-wave ballots, waves in order.
__global__ __launch_bounds__(kPlaceThreads) void class_place_kernel(
    const int32_t *__restrict__ row_ptr, uint32_t n, const uint32_t *__restrict__ base,
    uint32_t *__restrict__ inv, uint32_t *__restrict__ orig) {
    constexpr uint32_t kWaves = kPlaceThreads / 64;
    __shared__ uint32_t s_wave[kWaves][kClasses];
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t v = blockIdx.x * kPlaceThreads + threadIdx.x;
    const uint32_t c =
        v < n ? deg_class(static_cast<uint32_t>(row_ptr[v + 1] - row_ptr[v])) : kClasses;
    uint64_t mine = 0;
    for (uint32_t k = 0; k < kClasses; ++k) {
        const uint64_t m = __ballot(c == k);
        if (c == k) mine = m;
        if (lane == 0) s_wave[wave][k] = static_cast<uint32_t>(__popcll(m));
    }
    __syncthreads();
    if (v >= n) return;
    uint32_t id = base[blockIdx.x * kClasses + c];
    for (uint32_t w = 0; w < wave; ++w) id += s_wave[w][c];
    id += static_cast<uint32_t>(__popcll(mine & ((1ull << lane) - 1ull)));
    inv[v] = id;
    orig[id] = v;
}

// Relabelled records: field always_root becomes original id | always_root << 31.
__global__ void relabel_vrec_kernel(const VRec *__restrict__ vrec, const uint32_t *__restrict__ inv,
                                    uint32_t n, VRec *__restrict__ out) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    VRec r = vrec[v];
    r.always_root = v | (r.always_root ? 0x80000000u : 0u);
    out[inv[v]] = r;
}

__global__ void relabel_adj_kernel(const int32_t *__restrict__ col_idx, int64_t nnz,
                                   const uint32_t *__restrict__ inv, uint32_t orig_shift,
                                   unsigned long long *__restrict__ adj) {
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < nnz;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const uint32_t u = static_cast<uint32_t>(col_idx[e]);
        adj[e] = static_cast<unsigned long long>(inv[u]) |
                 (static_cast<unsigned long long>(u) << orig_shift);
    }
}

}  // namespace

uint32_t relabel_blocks(uint32_t n) { return (n + kPlaceThreads - 1) / kPlaceThreads; }

hipError_t launch_class_bounds(const int32_t *row_ptr, uint32_t n, bool widest_first, uint32_t *blk,
                               uint32_t *base, uint32_t *bounds, hipStream_t stream) {
    const uint32_t nb = relabel_blocks(n);
    if (nb == 0) return hipSuccess;
    class_count_kernel<<<nb, kPlaceThreads, 0, stream>>>(row_ptr, n, blk);
    class_scan_kernel<<<1, kClasses, 0, stream>>>(blk, nb, widest_first ? 1 : 0, base, bounds);
    return hipGetLastError();
}

hipError_t launch_relabel_vrec(const VRec *vrec, const uint32_t *inv, uint32_t n, VRec *vrec_r,
                               hipStream_t stream) {
    if (n == 0) return hipSuccess;
    relabel_vrec_kernel<<<(n + 255) / 256, 256, 0, stream>>>(vrec, inv, n, vrec_r);
    return hipGetLastError();
}

hipError_t launch_relabel_graph(const int32_t *row_ptr, const int32_t *col_idx, uint32_t n,
                                int64_t nnz, const uint32_t *base, uint32_t orig_shift,
                                uint32_t *inv, uint32_t *orig, unsigned long long *adj,
                                hipStream_t stream) {
    const uint32_t nb = relabel_blocks(n);
    if (nb == 0) return hipSuccess;
    class_place_kernel<<<nb, kPlaceThreads, 0, stream>>>(row_ptr, n, base, inv, orig);
    if (nnz > 0) {
        int64_t blocks = (nnz + 255) / 256;
        if (blocks > 16384) blocks = 16384;
        relabel_adj_kernel<<<static_cast<unsigned int>(blocks), 256, 0, stream>>>(
            col_idx, nnz, inv, orig_shift, adj);
    }
    return hipGetLastError();
}

}  // namespace fc
