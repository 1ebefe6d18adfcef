// Workgroup-per-tree sampler: Wilson's cycle popping, all vertices at once.
//
// Wilson's algorithm (Algorithm 3 of the paper) is the sequential schedule
// of "cycle popping": give every vertex a stack of random arrows (here the
// Philox arrows of the randomness contract, indexed by the per-vertex draw
// count k_v); while the top arrows contain a cycle, pop the arrows of one
// cycle.  The final top arrows form the spanning tree of G* rooted at u*,
// and Wilson's theorem says that the popped cycles -- hence the tree and
// every k_v -- are the same for every popping order.  This kernel pops ALL
// cycles present at once, round after round, which makes every round data
// parallel over the vertices of one tree:
//
//   round 0   reveal the first arrow of every vertex.
//   round r   U = vertices not yet known to reach u*.  Count, for each
//             t in U, the arrows from U into t; peel vertices of in-degree
//             0 level by level (Kahn).  What cannot be peeled lies on a
//             cycle.  Sweeping the peeled levels in reverse marks every
//             vertex whose arrow chain ends at u* or at a settled vertex as
//             settled.  Cycle vertices draw their next arrow (k_v + 1).
//   stop      when a round finds no cycle: every vertex reaches u*.
//
// One workgroup owns one tree at a time (tree ids come from a device
// queue); all phase changes are workgroup barriers, with no spin-waits.
// Per-slot device memory, n vertices:
//   word[v] (u64)  low 32: arrow target (u* = n) | settled << 31
//                  high 32: in-degree counter of the current round
//   kk[v]   (u32)  arrows drawn at v (k_v)
//   lists   (u32)  two unsettled lists (double buffer), the peel order and
//                  the peel level boundaries.
#include "fc_kernels.hpp"

namespace fc {

namespace {

constexpr uint32_t kSettled = 0x80000000u;
constexpr uint64_t kCntOne = 1ull << 32;

__device__ __forceinline__ uint32_t target_of(uint64_t w) {
    return static_cast<uint32_t>(w) & 0x7FFFFFFFu;
}
__device__ __forceinline__ bool settled_of(uint64_t w) {
    return (static_cast<uint32_t>(w) & kSettled) != 0;
}
__device__ __forceinline__ uint32_t cnt_of(uint64_t w) { return static_cast<uint32_t>(w >> 32); }

// Wave-aggregated append of `v` to `list` when `pred` holds: one LDS atomic
// per wave.  Must be reached by every lane of the wave (uniform control flow).
__device__ __forceinline__ void wave_append(uint32_t *__restrict__ list, uint32_t *tail,
                                            uint32_t v, bool pred) {
    const uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    const uint32_t lane = __lane_id();
    const uint32_t leader = __ffsll(static_cast<unsigned long long>(mask)) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(tail, static_cast<uint32_t>(__popcll(mask)));
    base = __shfl(base, leader, 64);
    if (pred) {
        const uint32_t off = static_cast<uint32_t>(__popcll(mask & ((1ull << lane) - 1ull)));
        list[base + off] = v;
    }
}

// One arrow of v in tree t with draw index k.
__device__ __forceinline__ uint32_t draw(const CoopArgs &a, uint32_t v, uint32_t k, uint32_t t) {
    const VRec r = load_vrec(a.vrec, v);
    const Philox4 x = philox4x32_10(v, k, t, a.stream_id, a.key0, a.key1);
    return arrow_target(r, x.x0, x.x1, a.col_idx, a.n);
}

__global__ __launch_bounds__(1024) void wilson_coop_kernel(CoopArgs a) {
    __shared__ uint32_t s_tree, s_u, s_p, s_cycles;
    __shared__ unsigned long long s_steps, s_digest, s_roots;

    const uint32_t n = a.n;
    const uint32_t T = blockDim.x;
    const uint32_t tid = threadIdx.x;
    const uint32_t wave_base = tid & ~63u;
    const uint32_t lane = tid & 63u;
    const size_t slot = blockIdx.x;
    uint64_t *__restrict__ word = a.word + slot * n;
    uint32_t *__restrict__ kk = a.kk + slot * n;
    uint32_t *__restrict__ listA = a.lists + slot * (4ull * n + 2);
    uint32_t *__restrict__ listB = listA + n;
    uint32_t *__restrict__ peel = listB + n;
    uint32_t *__restrict__ lvl = peel + n;  // n + 2 entries
    unsigned int err = 0;

    for (;;) {
        __syncthreads();
        if (tid == 0) s_tree = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t ti = s_tree;
        if (ti >= a.tree_count) break;
        const uint32_t t = a.tree_begin + ti;
        if (tid == 0) {
            s_u = 0;
            s_p = 0;
            s_steps = 0;
            s_digest = 0;
            s_roots = 0;
        }
        __syncthreads();

        // round 0: the first arrow of every vertex
        for (uint32_t base = wave_base; base < n; base += T) {
            const uint32_t v = base + lane;
            uint32_t tg = n;
            if (v < n) {
                tg = draw(a, v, 0u, t);
                word[v] = static_cast<uint64_t>(tg | (tg == n ? kSettled : 0u));
                kk[v] = 1u;
            }
            wave_append(listA, &s_u, v, v < n && tg != n);
        }
        __syncthreads();
        uint32_t ucount = s_u;
        uint32_t *U = listA, *Unext = listB;
        unsigned long long draws = n;
        uint32_t rounds = 0;

        while (ucount > 0) {
            if (++rounds > a.max_rounds || draws > a.step_cap) {
                err |= kErrStepCap;
                break;
            }
            // in-degree of each unsettled vertex from arrows of unsettled vertices
            for (uint32_t i = tid; i < ucount; i += T) {
                const uint32_t v = U[i];
                const uint32_t tg = target_of(word[v]);
                if (tg != n && !settled_of(word[tg])) atomicAdd(&word[tg], kCntOne);
            }
            if (tid == 0) s_p = 0;  // last read of s_p was followed by barriers
            __syncthreads();
            // level 0 of the peel: in-degree zero
            for (uint32_t base = wave_base; base < ucount; base += T) {
                const uint32_t i = base + lane;
                uint32_t v = 0;
                bool leaf = false;
                if (i < ucount) {
                    v = U[i];
                    leaf = cnt_of(word[v]) == 0u;
                }
                wave_append(peel, &s_p, v, leaf);
            }
            __syncthreads();
            uint32_t lo = 0, hi = s_p, nlev = 0;
            if (tid == 0) lvl[0] = 0;
            // peel level by level; the arrow target of a peeled vertex loses one in-arrow
            while (lo < hi) {
                if (tid == 0) lvl[nlev + 1] = hi;
                for (uint32_t base = lo + wave_base; base < hi; base += T) {
                    const uint32_t i = base + lane;
                    uint32_t tg = 0;
                    bool push = false;
                    if (i < hi) {
                        const uint32_t v = peel[i];
                        tg = target_of(word[v]);
                        if (tg != n && !settled_of(word[tg])) {
                            const uint64_t old = atomicAdd(&word[tg], ~kCntOne + 1ull);  // -1 in the high half
                            push = cnt_of(old) == 1u;
                        }
                    }
                    wave_append(peel, &s_p, tg, push);
                }
                __syncthreads();
                ++nlev;
                lo = hi;
                hi = s_p;
                __syncthreads();  // every wave has read s_p before the next level appends
            }
            const uint32_t peeled = hi;
            // reverse sweep: a vertex is settled when its arrow reaches u* or a settled vertex
            for (int32_t L = static_cast<int32_t>(nlev) - 1; L >= 0; --L) {
                const uint32_t a0 = lvl[L], a1 = lvl[L + 1];
                for (uint32_t i = a0 + tid; i < a1; i += T) {
                    const uint32_t v = peel[i];
                    const uint32_t tg = target_of(word[v]);
                    if (tg == n || settled_of(word[tg]))
                        word[v] = static_cast<uint64_t>(tg | kSettled);
                }
                __syncthreads();
            }
            if (peeled == ucount) {  // no cycle left: every vertex is settled
                ucount = 0;
                break;
            }
            // pop every cycle: vertices that kept in-arrows draw their next arrow
            if (tid == 0) {  // last reads of s_u / s_cycles were followed by barriers
                s_u = 0;
                s_cycles = 0;
            }
            __syncthreads();
            uint32_t my_cycles = 0;
            for (uint32_t base = wave_base; base < ucount; base += T) {
                const uint32_t i = base + lane;
                uint32_t v = 0;
                bool keep = false;
                if (i < ucount) {
                    v = U[i];
                    const uint64_t w = word[v];
                    if (cnt_of(w) > 0u) {
                        const uint32_t k = kk[v];
                        const uint32_t tg = draw(a, v, k, t);
                        if (k + 1u > 0x7FFFFFFFu) err |= kErrVisitOverflow;
                        kk[v] = k + 1u;
                        word[v] = static_cast<uint64_t>(tg | (tg == n ? kSettled : 0u));
                        keep = tg != n;
                        ++my_cycles;
                    } else {
                        keep = !settled_of(w);
                    }
                }
                wave_append(Unext, &s_u, v, keep);
            }
            if (my_cycles) atomicAdd(&s_cycles, my_cycles);
            __syncthreads();
            draws += s_cycles;
            ucount = s_u;
            uint32_t *tmp = U;
            U = Unext;
            Unext = tmp;
        }
        __syncthreads();
        if (err & kErrStepCap) break;  // the call fails; stop this workgroup

        // the tree: top arrows; R, digest, steps, optional per-tree dumps
        unsigned long long my_steps = 0, my_digest = 0, my_roots = 0;
        for (uint32_t v = tid; v < n; v += T) {
            const uint32_t tg = target_of(word[v]);
            const uint32_t k = kk[v];
            my_steps += k;
            my_digest += mix64((static_cast<unsigned long long>(v) << 32) | tg);
            if (tg == n) {
                ++my_roots;
                atomicAdd(&a.root_counts[v], 1u);
            }
            if (a.visit_counts) atomicAdd(&a.visit_counts[v], static_cast<unsigned long long>(k));
            if (a.parents) a.parents[static_cast<size_t>(ti) * n + v] = static_cast<int32_t>(tg);
            if (a.tree_visits) a.tree_visits[static_cast<size_t>(ti) * n + v] = k;
        }
        for (int off = 32; off > 0; off >>= 1) {
            my_steps += __shfl_down(my_steps, off, 64);
            my_digest += __shfl_down(my_digest, off, 64);
            my_roots += __shfl_down(my_roots, off, 64);
        }
        if (lane == 0) {
            atomicAdd(&s_steps, my_steps);
            atomicAdd(&s_digest, my_digest);
            atomicAdd(&s_roots, my_roots);
        }
        __syncthreads();
        if (tid == 0) {
            if (a.tree_digests) a.tree_digests[ti] = s_digest;
            if (a.tree_steps) a.tree_steps[ti] = s_steps;
            atomicAdd(&a.totals->walk_steps, s_steps);
            atomicAdd(&a.totals->roots, s_roots);
            atomicAdd(&a.totals->digest_sum, s_digest);
        }
    }
    if (err) atomicOr(&a.totals->error, err);
}

}  // namespace

hipError_t launch_wilson_coop(const CoopArgs &a, uint32_t threads, hipStream_t stream) {
    if (a.n == 0 || a.tree_count == 0 || a.slots == 0) return hipSuccess;
    wilson_coop_kernel<<<a.slots, threads, 0, stream>>>(a);
    return hipGetLastError();
}

}  // namespace fc
