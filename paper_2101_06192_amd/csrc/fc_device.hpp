// Device-side building blocks of the sampler: the Philox4x32-10 block
// function, the per-vertex record, the packed per-tree state word and the
// digest mixer.  gfx950 (CDNA4), wave64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fc {

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011): ten rounds of two
// 32x32->64 multiplies with the odd constants below, XOR of the high halves
// with the other two words and the round key, then a word permutation; the
// key advances by the 32-bit Weyl constants of the golden ratio and of
// sqrt(3)-1 between rounds.
struct Philox4 {
    uint32_t x0, x1, x2, x3;
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1) {
    constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
    constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 product each (a single v_mad_u64_u32 rather than
        // separate high and low multiplies)
        const uint64_t p0 = static_cast<uint64_t>(kM0) * c0;
        const uint64_t p1 = static_cast<uint64_t>(kM1) * c2;
        const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
        const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += kW0;
        k1 += kW1;
    }
    return {c0, c1, c2, c3};
}

// SplitMix64 output function (Steele, Lea and Flood 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Per-vertex record of G* for one alpha, 16 bytes, one dwordx4 load:
// first CSR entry, degree, low 32 bits of the root threshold, and a flag
// for "every step goes to u*" (threshold >= 2^32, e.g. isolated vertices).
struct __align__(16) VRec {
    int32_t start;
    uint32_t deg;
    uint32_t thr;
    uint32_t always_root;
};

__device__ __forceinline__ VRec load_vrec(const VRec *__restrict__ vrec, uint32_t v) {
    const uint4 q = reinterpret_cast<const uint4 *>(vrec)[v];
    return {static_cast<int32_t>(q.x), q.y, q.z, q.w};
}

// Makes all four words of a record live at this point (call it where the draw
// starts).  Left alone, the compiler fetches each field where it is first used
// -- the flag word, the threshold after Philox, start and degree behind the
// root test -- each fetch waiting for the one before: up to four round trips
// to memory per draw instead of one 16-byte load.  (An empty asm statement: it
// only keeps the values in registers; it reads and writes no memory.)
__device__ __forceinline__ void hold_vrec(VRec &r) {
    asm volatile("" : "+v"(r.start), "+v"(r.deg), "+v"(r.thr), "+v"(r.always_root));
}


// Weighted step (Section 2's non-negative edge weights; a walk leaves v along
// an edge with probability proportional to its weight).  With S[0..deg) the
// row's running weight sums (binary64, added in CSR order from 0, so
// S[deg - 1] = W_v > 0) the step takes the first entry i with u < S[i],
// u = (x1 * W_v) * 2^-32.  With W_v in [2^-64, 2^95], u < W_v for every x1,
// so the entry exists.
//
// u(x) is non-decreasing in the integer x (a product by a positive constant
// and rounding are both monotone), so {x : u(x) < S[i]} is a prefix [0, T_i)
// of the integers, T_i in [0, 2^32], non-decreasing in i.  The tables hold
// T_i clamped to [1, 2^32 - 1] (launch_step_thresholds), which decides
// "x1 < T_i" exactly for every x1 in [1, 2^32 - 2]; the two extreme words
// (probability 2^-31) take the binary64 search over S instead.  Either way
// the entry is the contract's, bit for bit.
__device__ __forceinline__ uint32_t weighted_entry_exact(const double *__restrict__ S,
                                                         uint32_t deg, uint32_t x1) {
    const double W = S[deg - 1];
    const double u = (static_cast<double>(x1) * W) * 0x1p-32;
    uint32_t lo = 0, hi = deg - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (u < S[mid]) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// T is scanned in chunks of kWeightedScan entries with unconditional loads:
// every threshold table carries kWeightedScan entries of padding after its
// last row, so a chunk that runs past the row (or the table) stays in bounds;
// entries past the row are masked out of the count.
constexpr uint32_t kWeightedScan = 8;

// First i in [base, m) of the chunk t = T[base .. base + kWeightedScan) with
// x1 < T[i], or m: the entries of the chunk below m that are <= x1, counted
// (T is non-decreasing).
__device__ __forceinline__ uint32_t weighted_chunk_count(const uint32_t (&t)[kWeightedScan],
                                                         uint32_t base, uint32_t m, uint32_t x1) {
    uint32_t c = base;
#pragma unroll
    for (uint32_t i = 0; i < kWeightedScan; ++i) c += (base + i < m && t[i] <= x1) ? 1u : 0u;
    return c;
}

__device__ __forceinline__ void load_chunk(const uint32_t *__restrict__ T,
                                           uint32_t (&t)[kWeightedScan]) {
#pragma unroll
    for (uint32_t i = 0; i < kWeightedScan; ++i) t[i] = T[i];
}

// Chunk of the answer in a row of m > kWeightedScan candidates: the first
// chunk whose last entry exceeds x1 (binary search over chunk ends), or the
// last chunk.
__device__ __forceinline__ uint32_t weighted_chunk(const uint32_t *__restrict__ T, uint32_t m,
                                                   uint32_t x1) {
    uint32_t lo = 0, hi = (m - 1) / kWeightedScan;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (x1 < T[mid * kWeightedScan + kWeightedScan - 1]) hi = mid;
        else lo = mid + 1;
    }
    return lo * kWeightedScan;
}

__device__ __forceinline__ uint32_t weighted_entry(const double *__restrict__ S,
                                                   const uint32_t *__restrict__ T, uint32_t deg,
                                                   uint32_t x1) {
    if (x1 - 1u >= 0xFFFFFFFEu) return weighted_entry_exact(S, deg, x1);  // x1 = 0 or 2^32 - 1
    const uint32_t m = deg - 1;  // the last entry is taken when every T_i <= x1 (i < m)
    const uint32_t base = m > kWeightedScan ? weighted_chunk(T, m, x1) : 0u;
    uint32_t t[kWeightedScan];
    load_chunk(T + base, t);
    return weighted_chunk_count(t, base, m, x1);
}

// Entry of v's row taken by a step that does not go to u*: uniform
// (floor(x1 * d / 2^32)) or, with the weight tables of the graph, weighted.
template <bool kWeighted>
__device__ __forceinline__ uint32_t neighbour_entry(const VRec &r, uint32_t x1,
                                                    const double *__restrict__ S,
                                                    const uint32_t *__restrict__ T) {
    if (kWeighted && S) return weighted_entry(S + r.start, T + r.start, r.deg, x1);
    return __umulhi(x1, r.deg);
}

// One arrow of v: returns the successor (n = u*) given Philox words x0, x1.
template <bool kWeighted>
__device__ __forceinline__ uint32_t arrow_target(const VRec &r, uint32_t x0, uint32_t x1,
                                                 const int32_t *__restrict__ col_idx,
                                                 const double *__restrict__ S,
                                                 const uint32_t *__restrict__ T, uint32_t n) {
    if (r.always_root || x0 < r.thr) return n;
    const uint32_t idx = neighbour_entry<kWeighted>(r, x1, S, T);
    return static_cast<uint32_t>(col_idx[r.start + static_cast<int32_t>(idx)]);
}

// Packed per-tree state word of one vertex (lane-per-tree sampler):
//   bits  0..30  next   successor drawn last (u* = n), valid when visited
//   bit   31     in_tree
//   bits 32..62  k      number of arrows drawn at the vertex in this tree
//   bit   63     epoch  parity of the tree the word belongs to; a word of the
//                       other parity is "fresh" (k = 0, not in the tree), so
//                       no per-tree clearing pass is needed.
namespace sw {
constexpr uint64_t kNextMask = 0x7FFFFFFFull;
constexpr uint64_t kInTree = 1ull << 31;
constexpr uint32_t kKMask = 0x7FFFFFFFu;
constexpr int kKShift = 32;
constexpr int kEpochShift = 63;

__device__ __forceinline__ bool current(uint64_t w, uint32_t ep) {
    return static_cast<uint32_t>(w >> kEpochShift) == ep;
}
__device__ __forceinline__ bool in_tree(uint64_t w, uint32_t ep) {
    return current(w, ep) && (w & kInTree);
}
__device__ __forceinline__ uint32_t visits(uint64_t w, uint32_t ep) {
    return current(w, ep) ? static_cast<uint32_t>(w >> kKShift) & kKMask : 0u;
}
__device__ __forceinline__ uint32_t next(uint64_t w) {
    return static_cast<uint32_t>(w & kNextMask);
}
__device__ __forceinline__ uint64_t pack(uint32_t nxt, uint32_t k, uint32_t ep) {
    return static_cast<uint64_t>(nxt) | (static_cast<uint64_t>(k & kKMask) << kKShift) |
           (static_cast<uint64_t>(ep) << kEpochShift);
}
}  // namespace sw

// Error bits reported by kernels through a device word.
constexpr uint32_t kErrVisitOverflow = 1u;
constexpr uint32_t kErrGraphRowPtr = 2u;
constexpr uint32_t kErrGraphColumn = 4u;
constexpr uint32_t kErrGraphSelfLoop = 8u;
constexpr uint32_t kErrGraphOrder = 16u;
constexpr uint32_t kErrGraphAsymmetric = 32u;
constexpr uint32_t kErrStepCap = 64u;
constexpr uint32_t kErrGraphWeight = 128u;     // weight not 0 or in [2^-64, 2^64]
constexpr uint32_t kErrGraphWeightAsym = 256u; // weight differs from its reverse entry's

// Device-side totals shared by a launch.
struct Totals {
    unsigned long long walk_steps;
    unsigned long long roots;
    unsigned long long digest_sum;
    unsigned int error;
    unsigned int pad;
};

}  // namespace fc
