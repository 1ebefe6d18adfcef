// Host-side launch wrappers of the ranking output kernels (rank.hip).  Every wrapper
// enqueues on `stream` and returns the launch status; none synchronises.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fc {

// Ranking output (rank.hip).  Keys: order-preserving uint64 of each score
// (complemented when descending), val[i] = i when val is not null; *bad |= 1
// when a score is NaN.
hipError_t launch_rank_keys(const double *score, uint32_t n, bool descending, uint64_t *key,
                            int32_t *val, unsigned int *bad, hipStream_t stream);
// hist[p * 256 + d] += keys whose byte p is d (hist zeroed by the caller).
hipError_t launch_digit_hist(const uint64_t *key, uint32_t n, unsigned int *hist,
                             hipStream_t stream);
// Tiles of the radix sort (thist holds 256 * rank_tiles(n) counters).
uint32_t rank_tiles(uint32_t n);
// One stable pass on byte shift / 8: (key, val) -> (okey, oval); base[d] =
// keys whose byte is below d.
hipError_t launch_radix_pass(const uint64_t *key, const int32_t *val, uint32_t n, uint32_t shift,
                             unsigned int *thist, const unsigned int *base, uint64_t *okey,
                             int32_t *oval, hipStream_t stream);
hipError_t launch_rank_of(const int32_t *order, uint32_t n, int32_t *rank, hipStream_t stream);
// out[sval[i]] = the number of sorted keys below skey[i] (skey ascending; out
// may be null); *ties += pairs of equal keys.
hipError_t launch_min_rank(const uint64_t *skey, const int32_t *sval, uint32_t n, uint32_t *out,
                           unsigned long long *ties, hipStream_t stream);
// key[i] = ra[i] << 32 | rb[i], val[i] = i.
hipError_t launch_pair_keys(const uint32_t *ra, const uint32_t *rb, uint32_t n, uint64_t *key,
                            int32_t *val, hipStream_t stream);
// *inv += strict inversions of s = rb[id[.]] (pairs p < q with s_p > s_q) by a
// bottom-up merge sort (s and tmp: n scratch each).
hipError_t launch_inversions(const uint32_t *rb, const int32_t *id, uint32_t n, uint32_t *s,
                             uint32_t *tmp, unsigned long long *inv, hipStream_t stream);
// Kendall pair counts of two rank vectors (< 2^31) over all pairs i < j
// (n <= 65535 * 256): out[0] += sum of sign products, out[1..3] += pairs tied in
// a, in b, in both (out zeroed by the caller; out[0] is two's complement).
hipError_t launch_kendall(const uint32_t *ra, const uint32_t *rb, uint32_t n,
                          unsigned long long *out, hipStream_t stream);

}  // namespace fc
