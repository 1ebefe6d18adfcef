// Ranking output: the vertex ranking by a score vector (stable LSD radix
// sort of order-preserving 64-bit keys, vertex ids as values) and Kendall's
// tau-b between two score vectors (exact integer pair counts).
//
// The top vertices of the forest closeness ranking are those with the lowest
// Omega_vv (Eq. "eq-fdistu-tr": farness grows with Omega_vv); the paper ranks
// the vertices by the estimate and reports Kendall's rank correlation against
// the ground truth (Section 6, "Vertex Ranking").
#include "fc_rank_kernels.hpp"

namespace fc {

namespace {

constexpr uint32_t kRankThreads = 256;
constexpr uint32_t kTileRounds = 16;  // a tile is kTileRounds x kRankThreads keys

// Order-preserving map of a binary64 to uint64 (-0 and +0 map alike): flip
// every bit of a negative number, set the sign bit of a positive one.
__device__ __forceinline__ uint64_t order_key(double x) {
    uint64_t u = __double_as_longlong(x == 0.0 ? 0.0 : x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__global__ __launch_bounds__(kRankThreads) void keys_kernel(const double *__restrict__ score,
                                                             uint32_t n, uint32_t descending,
                                                             uint64_t *__restrict__ key,
                                                             int32_t *__restrict__ val,
                                                             unsigned int *bad) {
    const uint32_t i = blockIdx.x * kRankThreads + threadIdx.x;
    if (i >= n) return;
    const double x = score[i];
    if (x != x) atomicOr(bad, 1u);
    const uint64_t k = order_key(x);
    key[i] = descending ? ~k : k;
    if (val) val[i] = static_cast<int32_t>(i);
}

// All eight 8-bit digit histograms of the keys in one pass (hist[p * 256 + d]).
__global__ __launch_bounds__(kRankThreads) void digit_hist_kernel(const uint64_t *__restrict__ key,
                                                                  uint32_t n,
                                                                  unsigned int *__restrict__ hist) {
    __shared__ unsigned int h[8 * 256];
    for (uint32_t i = threadIdx.x; i < 8 * 256; i += kRankThreads) h[i] = 0;
    __syncthreads();
    for (uint32_t i = blockIdx.x * kRankThreads + threadIdx.x; i < n;
         i += gridDim.x * kRankThreads) {
        const uint64_t k = key[i];
#pragma unroll
        for (uint32_t p = 0; p < 8; ++p) atomicAdd(&h[p * 256 + ((k >> (8 * p)) & 255u)], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < 8 * 256; i += kRankThreads)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

// Digit counts of one tile: thist[d * ntiles + tile].
__global__ __launch_bounds__(kRankThreads) void tile_hist_kernel(const uint64_t *__restrict__ key,
                                                                 uint32_t n, uint32_t shift,
                                                                 uint32_t ntiles,
                                                                 unsigned int *__restrict__ thist) {
    __shared__ unsigned int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const size_t base = static_cast<size_t>(blockIdx.x) * kTileRounds * kRankThreads;
#pragma unroll 4
    for (uint32_t r = 0; r < kTileRounds; ++r) {
        const size_t i = base + r * kRankThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(key[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    thist[static_cast<size_t>(threadIdx.x) * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Exclusive offsets: thread d turns its row of tile counts into the position
// of the tile's first key with digit d (base[d] = keys with a smaller digit).
__global__ __launch_bounds__(256) void tile_scan_kernel(unsigned int *__restrict__ thist,
                                                        uint32_t ntiles,
                                                        const unsigned int *__restrict__ base) {
    const uint32_t d = threadIdx.x;
    unsigned int run = base[d];
    unsigned int *row = thist + static_cast<size_t>(d) * ntiles;
    for (uint32_t t = 0; t < ntiles; ++t) {
        const unsigned int c = row[t];
        row[t] = run;
        run += c;
    }
}

// Stable scatter of one tile: keys are taken in position order, 256 at a
// time (wave w holds positions 64 w .. 64 w + 63 of the round); a key's place
// is its digit's running offset plus the keys with the same digit earlier in
// the round (earlier waves, then earlier lanes, found with eight ballots).
__global__ __launch_bounds__(kRankThreads) void tile_scatter_kernel(
    const uint64_t *__restrict__ key, const int32_t *__restrict__ val, uint32_t n, uint32_t shift,
    uint32_t ntiles, const unsigned int *__restrict__ thist, uint64_t *__restrict__ okey,
    int32_t *__restrict__ oval) {
    __shared__ unsigned int run[256];
    __shared__ unsigned int cnt[kRankThreads / 64][256];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    run[tid] = thist[static_cast<size_t>(tid) * ntiles + blockIdx.x];
#pragma unroll
    for (uint32_t w = 0; w < kRankThreads / 64; ++w) cnt[w][tid] = 0;
    __syncthreads();
    const size_t base = static_cast<size_t>(blockIdx.x) * kTileRounds * kRankThreads;
    const uint64_t below = (1ull << lane) - 1ull;
    for (uint32_t r = 0; r < kTileRounds; ++r) {
        const size_t i = base + r * kRankThreads + tid;
        const bool valid = i < n;
        const uint64_t k = valid ? key[i] : 0ull;
        const int32_t v = valid ? val[i] : 0;
        const uint32_t d = static_cast<uint32_t>((k >> shift) & 255u);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (uint32_t b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t before = static_cast<uint32_t>(__popcll(peers & below));
        if (valid && before == 0) cnt[wave][d] = static_cast<uint32_t>(__popcll(peers));
        __syncthreads();
        if (valid) {
            unsigned int pos = run[d] + before;
            for (uint32_t w = 0; w < wave; ++w) pos += cnt[w][d];
            okey[pos] = k;
            oval[pos] = v;
        }
        __syncthreads();
        unsigned int add = 0;
#pragma unroll
        for (uint32_t w = 0; w < kRankThreads / 64; ++w) {
            add += cnt[w][tid];
            cnt[w][tid] = 0;
        }
        run[tid] += add;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kRankThreads) void rank_of_kernel(const int32_t *__restrict__ order,
                                                               uint32_t n,
                                                               int32_t *__restrict__ rank) {
    const uint32_t i = blockIdx.x * kRankThreads + threadIdx.x;
    if (i < n) rank[order[i]] = static_cast<int32_t>(i);
}

// Min-rank of every key after the sort: the number of keys strictly below it
// (equal keys share it), found by binary search in the sorted keys and
// scattered to the key's original index.
// Also adds sum over positions of (i - min-rank) into *ties: a run of t equal
// keys contributes 0 + 1 + ... + (t - 1) = t(t - 1)/2, its tied pairs.
__device__ __forceinline__ void block_add_u64(unsigned long long x, unsigned long long *out) {
    __shared__ unsigned long long red[kRankThreads / 64];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if ((threadIdx.x & 63u) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (uint32_t w = 0; w < kRankThreads / 64; ++w) t += red[w];
        if (t) atomicAdd(out, t);
    }
}

__global__ __launch_bounds__(kRankThreads) void min_rank_kernel(const uint64_t *__restrict__ skey,
                                                                const int32_t *__restrict__ sval,
                                                                uint32_t n,
                                                                uint32_t *__restrict__ out,
                                                                unsigned long long *__restrict__ ties) {
    const uint32_t i = blockIdx.x * kRankThreads + threadIdx.x;
    unsigned long long t = 0;
    if (i < n) {
        const uint64_t k = skey[i];
        uint32_t lo = 0, hi = i;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (skey[mid] < k) lo = mid + 1;
            else hi = mid;
        }
        if (out) out[sval[i]] = lo;
        t = i - lo;
    }
    block_add_u64(t, ties);
}

// Composite keys (ra[i] << 32 | rb[i]) with the indices as values.
__global__ __launch_bounds__(kRankThreads) void pair_keys_kernel(const uint32_t *__restrict__ ra,
                                                                 const uint32_t *__restrict__ rb,
                                                                 uint32_t n,
                                                                 uint64_t *__restrict__ key,
                                                                 int32_t *__restrict__ val) {
    const uint32_t i = blockIdx.x * kRankThreads + threadIdx.x;
    if (i >= n) return;
    key[i] = (static_cast<uint64_t>(ra[i]) << 32) | rb[i];
    val[i] = static_cast<int32_t>(i);
}

// s[i] = rb[id[i]]: rank b in the order of the (a, b) sort.
__global__ __launch_bounds__(kRankThreads) void gather_kernel(const uint32_t *__restrict__ rb,
                                                              const int32_t *__restrict__ id,
                                                              uint32_t n, uint32_t *__restrict__ s) {
    const uint32_t i = blockIdx.x * kRankThreads + threadIdx.x;
    if (i < n) s[i] = rb[id[i]];
}

// One level of a bottom-up merge sort of s with strict-inversion counts: runs
// of `width` are sorted; each element finds its place in the merged run by
// binary search in the sibling run (a left element after the right elements
// below it, a right element after the left elements not above it, so equal
// values keep their order), and a right element adds the left elements above
// it to *inv (pairs p < q with s_p > s_q).
__global__ __launch_bounds__(kRankThreads) void merge_level_kernel(const uint32_t *__restrict__ in,
                                                                   uint32_t n, uint32_t width,
                                                                   uint32_t *__restrict__ out,
                                                                   unsigned long long *__restrict__ inv) {
    const uint32_t i = blockIdx.x * kRankThreads + threadIdx.x;
    unsigned long long c = 0;
    if (i < n) {
        const uint32_t x = in[i];
        const uint32_t l0 = (i / (2 * width)) * (2 * width);
        const uint32_t r0 = min(l0 + width, n), r1 = min(l0 + 2 * width, n);
        if (i < r0) {  // left run: count right elements < x
            uint32_t lo = r0, hi = r1;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (in[mid] < x) lo = mid + 1;
                else hi = mid;
            }
            out[l0 + (i - l0) + (lo - r0)] = x;
        } else {  // right run: count left elements <= x
            uint32_t lo = l0, hi = r0;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (in[mid] <= x) lo = mid + 1;
                else hi = mid;
            }
            out[l0 + (i - r0) + (lo - l0)] = x;
            c = r0 - lo;
        }
    }
    block_add_u64(c, inv);
}

// Kendall pair counts on min-ranks (ties exactly where the scores tie).
// Block (x, y): i-tile y (one vertex per thread), j-tiles x * kPairTiles ..
// (those not before the i-tile) staged in LDS.  Per pair, with
// da = sign(a_j - a_i), db = sign(b_j - b_i) in {-1, 0, 1} (ranks < 2^31, so
// the differences do not overflow): s += da db, qa += da^2, qb += db^2,
// qab += (da db)^2; then tied in a = pairs - qa, tied in b = pairs - qb, tied
// in both = pairs - qa - qb + qab.
constexpr uint32_t kPairTiles = 8;

// sign(x) as one v_med3_i32 (the compiler rewrites min/max into compares and
// selects); register-only, no memory operand.
__device__ __forceinline__ int32_t sign3(int32_t x) {
    int32_t r;
    asm("v_med3_i32 %0, %1, -1, 1" : "=v"(r) : "v"(x));
    return r;
}

__global__ __launch_bounds__(kRankThreads) void kendall_kernel(const uint32_t *__restrict__ ra,
                                                               const uint32_t *__restrict__ rb,
                                                               uint32_t n,
                                                               unsigned long long *__restrict__ out) {
    __shared__ uint2 sj[kRankThreads];
    __shared__ long long red[5][kRankThreads / 64];
    const uint32_t ti = blockIdx.y, tid = threadIdx.x;
    const uint32_t i = ti * kRankThreads + tid;
    const int32_t ai = i < n ? static_cast<int32_t>(ra[i]) : 0;
    const int32_t bi = i < n ? static_cast<int32_t>(rb[i]) : 0;
    int32_t s = 0, qa = 0, qb = 0, qab = 0, pairs = 0;
    const uint32_t ntiles = (n + kRankThreads - 1) / kRankThreads;
    auto pair = [&](uint2 j) {
        const int32_t da = sign3(static_cast<int32_t>(j.x) - ai);
        const int32_t db = sign3(static_cast<int32_t>(j.y) - bi);
        const int32_t p = da * db;
        s += p;
        qa += da * da;
        qb += db * db;
        qab += p * p;
    };
    for (uint32_t q = 0; q < kPairTiles; ++q) {
        const uint32_t tj = blockIdx.x * kPairTiles + q;
        if (tj >= ntiles) break;
        if (tj < ti) continue;  // uniform over the block
        const uint32_t j0 = tj * kRankThreads;
        __syncthreads();
        sj[tid] = j0 + tid < n ? make_uint2(ra[j0 + tid], rb[j0 + tid]) : make_uint2(0u, 0u);
        __syncthreads();
        if (i >= n) continue;
        if (tj != ti && j0 + kRankThreads <= n) {  // a full tile off the diagonal
#pragma unroll 8
            for (uint32_t jj = 0; jj < kRankThreads; ++jj) pair(sj[jj]);
            pairs += kRankThreads;
        } else {  // pairs (i, j), i < j < n
            const uint32_t jlo = tj == ti ? tid + 1 : 0, jhi = min(kRankThreads, n - j0);
            for (uint32_t jj = jlo; jj < jhi; ++jj) pair(sj[jj]);
            pairs += static_cast<int32_t>(jhi > jlo ? jhi - jlo : 0u);
        }
    }
    // block sums, one atomic each: s, tied in a, tied in b, tied in both
    const long long v[5] = {s, pairs - qa, pairs - qb, pairs - qa - qb + qab, 0};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        long long x = v[c];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if ((tid & 63u) == 0) red[c][tid >> 6] = x;
    }
    __syncthreads();
    if (tid < 4) {
        long long x = 0;
        for (uint32_t w = 0; w < kRankThreads / 64; ++w) x += red[tid][w];
        if (x) atomicAdd(&out[tid], static_cast<unsigned long long>(x));
    }
}

inline unsigned int blocks_for(uint64_t items, uint32_t threads) {
    return static_cast<unsigned int>((items + threads - 1) / threads);
}

}  // namespace

uint32_t rank_tiles(uint32_t n) { return (n + kTileRounds * kRankThreads - 1) / (kTileRounds * kRankThreads); }

hipError_t launch_rank_keys(const double *score, uint32_t n, bool descending, uint64_t *key,
                            int32_t *val, unsigned int *bad, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    keys_kernel<<<blocks_for(n, kRankThreads), kRankThreads, 0, stream>>>(
        score, n, descending ? 1u : 0u, key, val, bad);
    return hipGetLastError();
}

hipError_t launch_digit_hist(const uint64_t *key, uint32_t n, unsigned int *hist,
                             hipStream_t stream) {
    if (n == 0) return hipSuccess;
    uint32_t blocks = blocks_for(n, kRankThreads * 16u);
    if (blocks > 2048) blocks = 2048;
    digit_hist_kernel<<<blocks, kRankThreads, 0, stream>>>(key, n, hist);
    return hipGetLastError();
}

hipError_t launch_radix_pass(const uint64_t *key, const int32_t *val, uint32_t n, uint32_t shift,
                             unsigned int *thist, const unsigned int *base, uint64_t *okey,
                             int32_t *oval, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint32_t ntiles = rank_tiles(n);
    tile_hist_kernel<<<ntiles, kRankThreads, 0, stream>>>(key, n, shift, ntiles, thist);
    tile_scan_kernel<<<1, 256, 0, stream>>>(thist, ntiles, base);
    tile_scatter_kernel<<<ntiles, kRankThreads, 0, stream>>>(key, val, n, shift, ntiles, thist,
                                                             okey, oval);
    return hipGetLastError();
}

hipError_t launch_rank_of(const int32_t *order, uint32_t n, int32_t *rank, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    rank_of_kernel<<<blocks_for(n, kRankThreads), kRankThreads, 0, stream>>>(order, n, rank);
    return hipGetLastError();
}

hipError_t launch_min_rank(const uint64_t *skey, const int32_t *sval, uint32_t n, uint32_t *out,
                           unsigned long long *ties, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    min_rank_kernel<<<blocks_for(n, kRankThreads), kRankThreads, 0, stream>>>(skey, sval, n, out, ties);
    return hipGetLastError();
}

hipError_t launch_pair_keys(const uint32_t *ra, const uint32_t *rb, uint32_t n, uint64_t *key,
                            int32_t *val, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    pair_keys_kernel<<<blocks_for(n, kRankThreads), kRankThreads, 0, stream>>>(ra, rb, n, key, val);
    return hipGetLastError();
}

hipError_t launch_inversions(const uint32_t *rb, const int32_t *id, uint32_t n, uint32_t *s,
                             uint32_t *tmp, unsigned long long *inv, hipStream_t stream) {
    if (n < 2) return hipSuccess;
    gather_kernel<<<blocks_for(n, kRankThreads), kRankThreads, 0, stream>>>(rb, id, n, s);
    uint32_t *a = s, *b = tmp;
    for (uint32_t w = 1; w < n; w *= 2) {
        merge_level_kernel<<<blocks_for(n, kRankThreads), kRankThreads, 0, stream>>>(a, n, w, b, inv);
        uint32_t *t = a;
        a = b;
        b = t;
        if (w > 0x7FFFFFFFu) break;
    }
    return hipGetLastError();
}

hipError_t launch_kendall(const uint32_t *ra, const uint32_t *rb, uint32_t n,
                          unsigned long long *out, hipStream_t stream) {
    if (n < 2) return hipSuccess;
    const uint32_t ntiles = (n + kRankThreads - 1) / kRankThreads;
    const dim3 grid((ntiles + kPairTiles - 1) / kPairTiles, ntiles);
    kendall_kernel<<<grid, kRankThreads, 0, stream>>>(ra, rb, n, out);
    return hipGetLastError();
}

}  // namespace fc
