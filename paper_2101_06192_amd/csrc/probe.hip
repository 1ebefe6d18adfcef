// Memory-system probes (measurement only, outside the method): the rate of
// independent random 4-byte loads, or of random 4-byte atomic adds, over a
// footprint of a chosen size.  The sampler's random accesses are bounded by
// this rate, so it is the denominator of its random-access roofline.
#include "fc_kernels.hpp"

namespace fc {

namespace {

// xorshift32 (Marsaglia 2003): a cheap index stream per lane.
__device__ __forceinline__ uint32_t xs32(uint32_t x) {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}

__global__ __launch_bounds__(256) void random_load_kernel(const uint32_t *__restrict__ data,
                                                          uint32_t mask, uint32_t iters,
                                                          uint32_t *__restrict__ sink) {
    uint32_t s[8];
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int q = 0; q < 8; ++q) s[q] = 0x9E3779B9u * (gid * 8u + q + 1u);
    uint32_t acc = 0;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            s[q] = xs32(s[q]);
            acc += data[s[q] & mask];
        }
    }
    if (acc == 0xFFFFFFFFu) sink[0] = acc;  // keeps the loads alive
}

__global__ __launch_bounds__(256) void random_atomic_kernel(uint32_t *__restrict__ data, uint32_t mask,
                                                            uint32_t iters) {
    uint32_t s = 0x9E3779B9u * (blockIdx.x * blockDim.x + threadIdx.x + 1u);
    for (uint32_t it = 0; it < iters; ++it)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            s = xs32(s);
            atomicAdd(&data[s & mask], 1u);
        }
}

}  // namespace

hipError_t launch_random_access(uint32_t *data, uint32_t words_pow2, uint32_t iters, bool atomics,
                                uint32_t blocks, uint32_t *sink, hipStream_t stream) {
    const uint32_t mask = words_pow2 - 1u;
    if (atomics) random_atomic_kernel<<<blocks, 256, 0, stream>>>(data, mask, iters);
    else random_load_kernel<<<blocks, 256, 0, stream>>>(data, mask, iters, sink);
    return hipGetLastError();
}

}  // namespace fc
