// Workgroup-per-tree sampler with every in-arrow counter in LDS.
//
// Same cycle popping as the global-word sampler (Wilson's theorem: popping
// every cycle of the top arrows, round after round, yields the tree and the
// per-vertex arrow counts of Wilson's walk), but the per-round in-arrow
// counts that drive the Kahn peel are LDS fields sized by degree, so the
// counting and peeling phases issue no global atomics.  Vertices are on
// degree-class internal ids (see relabel.hip); Philox counters, the digest
// and all outputs use original ids.
//
// Per round r, with U the unsettled vertices as (v, target) pairs:
//   count    cnt[t] += 1 for every arrow of U into an unsettled target t
//            (merged into the draw pass in round 0)
//   level 0  v with cnt[v] == 0 starts the peel list
//   peel     a peeled x decrements cnt[target(x)]; the one that drops it to 0
//            appends (target, its own target) to the list (a global load of
//            the target's tree word)
//   sweep    peel levels in reverse: x is settled when its target is
//   redraw   what is left with cnt[v] == 1 lies on a cycle: v draws its next
//            arrow (cnt[v] back to 0); vertices hanging off a cycle keep theirs
// A count is exact for every unsettled vertex: after the peel, peeled
// vertices are at 0 and cycle vertices at 1 (one arrow from the cycle, a
// functional graph's leftover after Kahn peeling is a union of cycles), so
// the redraw pass leaves all unsettled counts at 0 before the next count.
// Counts of settled vertices are never read again; they stay at most the
// degree, so no field overflows into its neighbour.
//
// Memory per tree (slot), n vertices:
//   word[v]  u64 global  internal target | original target << 32 (u* = n)
//   kk[v]    u64 global  (epoch << 32) | k_v for redrawn vertices
//   lists    u64 global  (v, target) pairs: two unsettled lists, peel order
//   levels   u32 global  peel level boundaries
//   LDS      count fields (4/8/16/32 bits by class), then the settled bitmap
#include "fc_kernels.hpp"

namespace fc {

namespace {

__device__ __forceinline__ uint32_t lo32(uint64_t w) { return static_cast<uint32_t>(w); }
__device__ __forceinline__ uint32_t hi32(uint64_t w) { return static_cast<uint32_t>(w >> 32); }
__device__ __forceinline__ uint64_t pair(uint32_t v, uint32_t tg) {
    return static_cast<uint64_t>(v) | (static_cast<uint64_t>(tg) << 32);
}
__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// Wave-aggregated append with a capacity check: one LDS atomic per wave;
// entries past `cap` are dropped and reported through *overflow.  Every
// lane of the wave must reach it.
__device__ __forceinline__ void wave_append(uint64_t *__restrict__ list, uint32_t *tail,
                                            uint32_t cap, uint32_t *overflow, uint64_t item,
                                            bool pred) {
    const uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    const uint32_t lane = __lane_id();
    const uint32_t leader = __ffsll(static_cast<unsigned long long>(mask)) - 1;
    uint32_t base = 0;
    if (lane == leader) {
        const uint32_t cnt = static_cast<uint32_t>(__popcll(mask));
        base = atomicAdd(tail, cnt);
        if (base + cnt > cap) atomicOr(overflow, 1u);
    }
    base = __shfl(base, leader, 64);
    if (pred) {
        const uint32_t at = base + static_cast<uint32_t>(__popcll(mask & ((1ull << lane) - 1ull)));
        if (at < cap) list[at] = item;
    }
}

enum Phase : int { kPhDraw0 = 0, kPhIndeg, kPhLevel0, kPhPeel, kPhSweep, kPhRedraw, kPhOutput,
                   kPhCount };

// Counter field of internal id x: LDS word, shift and mask.
struct Field {
    uint32_t w, sh, mask;
};
struct Classes {
    uint32_t n0, n1, n2, o1, o2, o3;
};
__device__ __forceinline__ Field field_of(const Classes &c, uint32_t x) {
    if (x < c.n0) return {x >> 3, (x & 7u) << 2, 0xFu};
    if (x < c.n1) {
        const uint32_t j = x - c.n0;
        return {c.o1 + (j >> 2), (j & 3u) << 3, 0xFFu};
    }
    if (x < c.n2) {
        const uint32_t j = x - c.n1;
        return {c.o2 + (j >> 1), (j & 1u) << 4, 0xFFFFu};
    }
    return {c.o3 + (x - c.n2), 0u, 0xFFFFFFFFu};
}

// One arrow of internal vertex v (record r) with draw index k in tree t:
// internal | original target, (n | n << 32) for u*.
__device__ __forceinline__ uint64_t draw(const CoopJob &j, const VRec &r, uint32_t key0,
                                         uint32_t key1, uint32_t k, uint32_t t) {
    const uint32_t orig = r.always_root & 0x7FFFFFFFu;
    const Philox4 x = philox4x32_10(orig, k, t, j.stream_id, key0, key1);
    if ((r.always_root >> 31) || x.x0 < r.thr) return pair(j.n, j.n);
    const uint32_t idx = __umulhi(x.x1, r.deg);
    return j.adj[r.start + static_cast<int32_t>(idx)];
}

__global__ __launch_bounds__(1024) void wilson_lds_kernel(CoopArgs a) {
    extern __shared__ uint32_t s_lds[];
    __shared__ uint32_t s_item, s_u, s_p, s_cycles, s_over;
    __shared__ unsigned long long s_digest, s_roots;
    __shared__ unsigned long long s_ph[kPhCount + 1];

    const uint32_t T = blockDim.x;
    const uint32_t tid = threadIdx.x;
    const uint32_t wave_base = tid & ~63u;
    const uint32_t lane = tid & 63u;
    const size_t slot = blockIdx.x;
    const size_t stride = a.n_max;
    uint64_t *__restrict__ word = static_cast<uint64_t *>(a.word) + slot * stride;
    uint64_t *__restrict__ kk = a.kk + slot * stride;
    uint64_t *__restrict__ listA = a.lists + slot * (3ull * stride);
    uint64_t *__restrict__ listB = listA + stride;
    uint64_t *__restrict__ peel = listB + stride;
    uint32_t *__restrict__ lvl = a.levels + slot * (stride + 2);
    unsigned int err = 0;
    uint32_t epoch = 0;

    const bool timing = a.phase_ticks != nullptr;
    if (tid == 0) s_over = 0;
    if (timing && tid == 0) {
        for (int i = 0; i < kPhCount; ++i) s_ph[i] = 0;
        s_ph[kPhCount] = wall_clock64();
    }
    auto mark = [&](int which) {
        if (timing && tid == 0) {
            const unsigned long long now = wall_clock64();
            s_ph[which] += now - s_ph[kPhCount];
            s_ph[kPhCount] = now;
        }
    };

    for (;;) {
        __syncthreads();
        if (tid == 0) s_item = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t item = uniform(s_item);
        if (item >= a.item_count) break;
        const CoopJob job = a.jobs ? a.jobs[uniform(a.item_job[item])] : a.single;
        const uint32_t ti = item - job.first_item;
        const uint32_t t = job.tree_begin + ti;
        const uint32_t n = job.n;
        const CountLayout L = count_layout(n, job.n0, job.n1, job.n2);
        const Classes C{job.n0, job.n1, job.n2, L.o1, L.o2, L.o3};
        uint32_t *__restrict__ bits = s_lds + L.ob;

        auto is_settled = [&](uint32_t v) -> bool {
            return v >= n || ((bits[v >> 5] >> (v & 31u)) & 1u);
        };
        auto set_settled = [&](uint32_t v) { atomicOr(&bits[v >> 5], 1u << (v & 31u)); };
        auto count_of = [&](uint32_t v) -> uint32_t {
            const Field f = field_of(C, v);
            return (s_lds[f.w] >> f.sh) & f.mask;
        };
        auto count_add = [&](uint32_t v) {
            const Field f = field_of(C, v);
            atomicAdd(&s_lds[f.w], 1u << f.sh);
        };
        // decrement; returns the count before
        auto count_dec = [&](uint32_t v) -> uint32_t {
            const Field f = field_of(C, v);
            return (atomicAdd(&s_lds[f.w], 0u - (1u << f.sh)) >> f.sh) & f.mask;
        };

        ++epoch;
        if (tid == 0) {
            s_u = 0;
            s_p = 0;
            s_digest = 0;
            s_roots = 0;
        }
        for (uint32_t i = tid; i < L.words; i += T) s_lds[i] = 0u;
        __syncthreads();

        // round 0: the first arrow of every vertex, and the first in-arrow count
        // (arrows into vertices that turn out settled are counted too; those
        // counts are never read)
        for (uint32_t base = wave_base; base < n; base += T) {
            const uint32_t v = base + lane;
            uint32_t tg = n;
            if (v < n) {
                const VRec r = load_vrec(job.vrec, v);
                const uint64_t w = draw(job, r, a.key0, a.key1, 0u, t);
                word[v] = w;
                tg = lo32(w);
                if (tg == n) set_settled(v);
                else count_add(tg);
            }
            wave_append(listA, &s_u, n, &s_over, pair(v, tg), v < n && tg != n);
        }
        __syncthreads();
        mark(kPhDraw0);
        uint32_t ucount = uniform(s_u);
        uint64_t *U = listA, *Unext = listB;
        unsigned long long draws = n;
        uint32_t rounds = 0;
        bool counted = true;

        while (ucount > 0) {
            if (++rounds > a.max_rounds || draws > job.step_cap || s_over) {
                err |= kErrStepCap;
                break;
            }
            if (!counted) {
                for (uint32_t i = tid; i < ucount; i += T) {
                    const uint32_t tg = hi32(U[i]);
                    if (!is_settled(tg)) count_add(tg);
                }
                __syncthreads();
            }
            counted = false;
            if (tid == 0) s_p = 0;
            mark(kPhIndeg);
            // level 0 of the peel: no in-arrows
            for (uint32_t base = wave_base; base < ucount; base += 2 * T) {
                uint64_t it[2];
                bool leaf[2];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const uint32_t i = base + q * T + lane;
                    it[q] = i < ucount ? U[i] : 0ull;
                    leaf[q] = i < ucount && count_of(lo32(it[q])) == 0u;
                }
#pragma unroll
                for (int q = 0; q < 2; ++q) wave_append(peel, &s_p, n, &s_over, it[q], leaf[q]);
            }
            __syncthreads();
            mark(kPhLevel0);
            uint32_t lo = 0, hi = min(uniform(s_p), n), nlev = 0;
            if (tid == 0) lvl[0] = 0;
            while (lo < hi) {
                if (tid == 0) lvl[nlev + 1] = hi;
                for (uint32_t base = lo + wave_base; base < hi; base += 2 * T) {
                    uint32_t tg[2];
                    bool push[2];
                    uint64_t nx[2];
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const uint32_t i = base + q * T + lane;
                        tg[q] = i < hi ? hi32(peel[i]) : n;
                        push[q] = false;
                    }
#pragma unroll
                    for (int q = 0; q < 2; ++q)
                        if (!is_settled(tg[q])) push[q] = count_dec(tg[q]) == 1u;
#pragma unroll
                    for (int q = 0; q < 2; ++q) nx[q] = push[q] ? word[tg[q]] : 0ull;
#pragma unroll
                    for (int q = 0; q < 2; ++q)
                        wave_append(peel, &s_p, n, &s_over, pair(tg[q], lo32(nx[q])), push[q]);
                }
                __syncthreads();
                ++nlev;
                lo = hi;
                hi = min(uniform(s_p), n);
                __syncthreads();  // every wave has read s_p before the next level appends
            }
            const uint32_t peeled = hi;
            mark(kPhPeel);
            if (peeled == ucount) {  // no cycle: every unsettled vertex reaches u*
                ucount = 0;
                break;
            }
            for (int32_t Lv = static_cast<int32_t>(nlev) - 1; Lv >= 0; --Lv) {
                const uint32_t a0 = uniform(lvl[Lv]), a1 = uniform(lvl[Lv + 1]);
                for (uint32_t i = a0 + tid; i < a1; i += T) {
                    const uint64_t p = peel[i];
                    if (is_settled(hi32(p))) set_settled(lo32(p));
                }
                __syncthreads();
            }
            mark(kPhSweep);
            if (tid == 0) {
                s_u = 0;
                s_cycles = 0;
            }
            __syncthreads();
            uint32_t my_cycles = 0;
            for (uint32_t base = wave_base; base < ucount; base += 2 * T) {
                uint64_t it[2];
                bool keep[2];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const uint32_t i = base + q * T + lane;
                    it[q] = i < ucount ? U[i] : pair(n, n);
                    keep[q] = false;
                }
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const uint32_t v = lo32(it[q]);
                    if (is_settled(v)) continue;
                    if (count_of(v) != 0u) {  // on a cycle: pop it
                        (void)count_dec(v);
                        const uint64_t kv = kk[v];
                        const uint32_t k = hi32(kv) == epoch ? lo32(kv) : 1u;
                        const VRec r = load_vrec(job.vrec, v);
                        const uint64_t w = draw(job, r, a.key0, a.key1, k, t);
                        if (k + 1u > 0x7FFFFFFFu) err |= kErrVisitOverflow;
                        kk[v] = (static_cast<uint64_t>(epoch) << 32) | (k + 1u);
                        word[v] = w;
                        it[q] = pair(v, lo32(w));
                        if (lo32(w) == n) set_settled(v);
                        else keep[q] = true;
                        ++my_cycles;
                    } else {  // hanging off a cycle
                        keep[q] = true;
                    }
                }
#pragma unroll
                for (int q = 0; q < 2; ++q) wave_append(Unext, &s_u, n, &s_over, it[q], keep[q]);
            }
            if (my_cycles) atomicAdd(&s_cycles, my_cycles);
            __syncthreads();
            mark(kPhRedraw);
            draws += uniform(s_cycles);
            ucount = min(uniform(s_u), n);
            uint64_t *tmp = U;
            U = Unext;
            Unext = tmp;
        }
        __syncthreads();
        if (err & kErrStepCap) break;

        unsigned long long my_digest = 0, my_roots = 0;
        const bool want_k = job.visit_counts || job.tree_visits;
        for (uint32_t v = tid; v < n; v += T) {
            const uint64_t w = word[v];
            const uint32_t ov = job.orig[v];
            const uint32_t otg = hi32(w);
            my_digest += mix64((static_cast<unsigned long long>(ov) << 32) | otg);
            if (lo32(w) == n) {
                ++my_roots;
                atomicAdd(&job.root_counts[ov], 1u);
            }
            if (job.parents) job.parents[static_cast<size_t>(ti) * n + ov] = static_cast<int32_t>(otg);
            if (want_k) {
                const uint64_t kv = kk[v];
                const uint32_t k = hi32(kv) == epoch ? lo32(kv) : 1u;
                if (job.visit_counts)
                    atomicAdd(&job.visit_counts[ov], static_cast<unsigned long long>(k));
                if (job.tree_visits) job.tree_visits[static_cast<size_t>(ti) * n + ov] = k;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            my_digest += __shfl_down(my_digest, off, 64);
            my_roots += __shfl_down(my_roots, off, 64);
        }
        if (lane == 0) {
            atomicAdd(&s_digest, my_digest);
            atomicAdd(&s_roots, my_roots);
        }
        __syncthreads();
        if (tid == 0) {
            if (job.tree_digests) job.tree_digests[ti] = s_digest;
            if (job.tree_steps) job.tree_steps[ti] = draws;
            atomicAdd(&a.totals->walk_steps, draws);
            atomicAdd(&a.totals->roots, s_roots);
            atomicAdd(&a.totals->digest_sum, s_digest);
        }
        mark(kPhOutput);
    }
    if (timing && tid == 0)
        for (int i = 0; i < kPhCount; ++i) atomicAdd(&a.phase_ticks[i], s_ph[i]);
    if (err) atomicOr(&a.totals->error, err);
}

}  // namespace

hipError_t lds_set_limit(uint32_t lds_words) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&wilson_lds_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               static_cast<int>(4u * lds_words));
}

int lds_max_active(uint32_t threads, uint32_t lds_words) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &blocks, reinterpret_cast<const void *>(&wilson_lds_kernel), static_cast<int>(threads),
            4u * static_cast<size_t>(lds_words)) != hipSuccess)
        return 0;
    return blocks;
}

hipError_t launch_wilson_lds(const CoopArgs &a, uint32_t threads, uint32_t lds_words,
                             hipStream_t stream) {
    if (a.n_max == 0 || a.item_count == 0 || a.slots == 0) return hipSuccess;
    wilson_lds_kernel<<<a.slots, threads, 4u * static_cast<size_t>(lds_words), stream>>>(a);
    return hipGetLastError();
}

}  // namespace fc
