// Wave-level helpers shared by the workgroup-per-tree samplers (wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fc {

__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// x of lane i (i uniform across the wave; a scalar read, no LDS round trip).
__device__ __forceinline__ uint32_t lane_of(uint32_t x, int32_t i) {
    return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), i));
}

// Order this wave's LDS accesses before and after (single-wave phases).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Workgroup barrier that orders LDS accesses only: global stores issued before
// it are not waited for (use it where they are read only after a full barrier).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Appends R items per lane (item[q] where pred[q]) to a list whose tail
// counter lives in LDS, with one LDS atomic per wave: item q of every lane
// goes after items 0..q-1 of all the wave's lanes.  Entries past `cap` are
// dropped and reported through *overflow.  Every lane of the wave must reach
// the call.
template <int R>
__device__ __forceinline__ void wave_append_many(uint64_t *__restrict__ list, uint32_t *tail,
                                                 uint32_t cap, uint32_t *overflow,
                                                 const uint64_t (&item)[R], const bool (&pred)[R]) {
    uint32_t total = 0;
#pragma unroll
    for (int q = 0; q < R; ++q) total += static_cast<uint32_t>(__popcll(__ballot(pred[q])));
    if (total == 0) return;
    const uint32_t lane = __lane_id();
    uint32_t base = 0;
    if (lane == 0) {
        base = atomicAdd(tail, total);
        if (base + total > cap) atomicOr(overflow, 1u);
    }
    base = __shfl(base, 0, 64);
    const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const uint64_t mask = __ballot(pred[q]);  // recomputed: fewer live scalar registers
        if (pred[q]) {
            const uint32_t at = base + static_cast<uint32_t>(__popcll(mask & below));
            if (at < cap) list[at] = item[q];
        }
        base += static_cast<uint32_t>(__popcll(mask));
    }
}

// Adds the sum over the wave of each lane's `count` to an LDS counter with one
// atomic.  Every lane of the wave must reach the call.
__device__ __forceinline__ void wave_count(uint32_t *counter, uint32_t count) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) count += __shfl_xor(count, off, 64);
    if (__lane_id() == 0 && count != 0u) atomicAdd(counter, count);
}

__device__ __forceinline__ void wave_append(uint64_t *__restrict__ list, uint32_t *tail,
                                            uint32_t cap, uint32_t *overflow, uint64_t item,
                                            bool pred) {
    const uint64_t it[1] = {item};
    const bool p[1] = {pred};
    wave_append_many<1>(list, tail, cap, overflow, it, p);
}

}  // namespace fc
