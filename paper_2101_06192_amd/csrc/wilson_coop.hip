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
//
// Memory per tree (slot), n vertices:
//   word[v]  u32 or u64    arrow target (u* = n) in the low `tshift` bits,
//            global        in-arrow count of the current round above it; a
//                          32-bit word when ceil(log2(n+1)) + ceil(log2(dmax+1))
//                          fits (the count never exceeds the degree)
//   kk[v]    u64  global   (epoch << 32) | k_v, written only when v draws a
//                          second arrow; a stale epoch means k_v = 1
//   lists    u64  global   (vertex, target) pairs: two unsettled lists
//                          (double buffer) and the peel order; plus the peel
//                          level boundaries (u32)
//   settled  bit  LDS      one bit per vertex when n/8 bytes fit the LDS
//                          budget, else a per-slot global bitmap
//   filter   bit  LDS      re-pop filter (when re-formed 2-cycles are popped
//                          within their round): one bit per id modulo its size
#include "fc_kernels.hpp"

namespace fc {

namespace {

__device__ __forceinline__ uint32_t lo32(uint64_t w) { return static_cast<uint32_t>(w); }
__device__ __forceinline__ uint32_t hi32(uint64_t w) { return static_cast<uint32_t>(w >> 32); }
__device__ __forceinline__ uint64_t pair(uint32_t v, uint32_t tg) {
    return static_cast<uint64_t>(v) | (static_cast<uint64_t>(tg) << 32);
}

// Wave-aggregated append of `item` to `list` when `pred` holds: one LDS
// atomic per wave.  Every lane of the wave must reach it (uniform control).
__device__ __forceinline__ void wave_append(uint64_t *__restrict__ list, uint32_t *tail,
                                            uint64_t item, bool pred) {
    const uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    const uint32_t lane = __lane_id();
    const uint32_t leader = __ffsll(static_cast<unsigned long long>(mask)) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(tail, static_cast<uint32_t>(__popcll(mask)));
    base = __shfl(base, leader, 64);
    if (pred) {
        const uint32_t off = static_cast<uint32_t>(__popcll(mask & ((1ull << lane) - 1ull)));
        list[base + off] = item;
    }
}

// As wave_append, two items per lane (adjacent), dropping items at or past
// `cap`; the tail still counts them, so a tail above `cap` reports the overflow.
__device__ __forceinline__ void wave_append2(uint64_t *__restrict__ list, uint32_t *tail,
                                             uint64_t a0, uint64_t a1, bool pred, uint32_t cap) {
    const uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    const uint32_t lane = __lane_id();
    const uint32_t leader = __ffsll(static_cast<unsigned long long>(mask)) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(tail, 2u * static_cast<uint32_t>(__popcll(mask)));
    base = __shfl(base, leader, 64);
    if (pred) {
        const uint32_t i = base + 2u * static_cast<uint32_t>(__popcll(mask & ((1ull << lane) - 1ull)));
        if (i + 1u < cap) {
            list[i] = a0;
            list[i + 1u] = a1;
        }
    }
}

// The per-tree arrays belong to one workgroup for the whole launch, so their
// atomics only need workgroup scope (no cross-XCD coherence).
template <typename W>
__device__ __forceinline__ W wg_fetch_add(W *p, W v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void wg_fetch_or(uint32_t *p, uint32_t v) {
    (void)__hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Order this wave's LDS accesses before and after (single-wave phases).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Items per lane per iteration of the streaming passes (loads in flight).
constexpr int kR = 2;

// Per-phase wall-clock accounting (tid 0 of each workgroup), when requested.
enum Phase : int { kPhDraw0 = 0, kPhIndeg, kPhLevel0, kPhPeel, kPhSweep, kPhRedraw, kPhOutput,
                   kPhCount };

// A value read from LDS that every lane of the wave holds: tell the compiler,
// so that what depends on it lives in scalar registers.
__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// One arrow of v in tree t with draw index k (kWeighted: the job may carry
// running weight sums).
template <bool kWeighted>
__device__ __forceinline__ uint32_t draw(const CoopJob &j, uint32_t key0, uint32_t key1,
                                         uint32_t v, uint32_t k, uint32_t t) {
    VRec r = load_vrec(j.vrec, v);
    hold_vrec(r);
    if (r.always_root) return j.n;  // the arrow is u* whatever the Philox words are
    const Philox4 x = philox4x32_10(v, k, t, j.stream_id, key0, key1);
    return arrow_target<kWeighted>(r, x.x0, x.x1, j.col_idx, j.wsum, j.wthr, j.n);
}

// Work items are trees; a single-graph launch has one implicit job, a batch
// launch maps item w to job item_job[w] and tree w - job.first_item.
// kInBits (with kLdsBits): a second LDS bitmap marks unsettled vertices that
// still have in-arrows in the current round -- set while counting, cleared
// when the vertex is peeled -- so peel level 0 and cycle detection read LDS
// instead of the global tree words.
template <bool kLdsBits, typename W, bool kInBits, bool kWeighted>
// At most 512 threads, and registers for six waves per SIMD (24 per CU):
// the phases are latency bound, so resident waves matter more than unrolling.
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(6, 6)))
void wilson_coop_kernel(CoopArgs a, uint32_t fwords) {
    extern __shared__ uint32_t s_dyn[];
    __shared__ uint32_t s_item, s_u, s_p, s_cycles, s_over, s_nlev, s_rp[2];
    __shared__ uint64_t s_tail[64];
    __shared__ unsigned long long s_digest, s_roots;

    const uint32_t T = blockDim.x;
    const uint32_t tid = threadIdx.x;
    const uint32_t wave_base = tid & ~63u;
    const uint32_t lane = tid & 63u;
    const size_t slot = blockIdx.x;
    const size_t stride = a.n_max;
    const size_t bstride = (stride + 31u) >> 5;
    W *__restrict__ word = static_cast<W *>(a.word) + slot * stride;
    uint64_t *__restrict__ kk = a.kk + slot * stride;
    uint64_t *__restrict__ listA = a.lists + slot * (3ull * stride);
    uint64_t *__restrict__ listB = listA + stride;
    uint64_t *__restrict__ peel = listB + stride;
    uint32_t *__restrict__ lvl = a.levels + slot * (stride + 2);
    uint32_t *__restrict__ bits = kLdsBits ? s_dyn : a.bits + slot * bstride;
    uint32_t *__restrict__ inb = s_dyn + bstride;  // used only when kInBits
    // re-pop filter (fwords > 0): one bit per vertex id modulo its size, set for
    // vertices popped again within a round
    uint32_t *__restrict__ filt = s_dyn + (kLdsBits ? (kInBits ? 2u : 1u) * bstride : 0u);
    const uint32_t fmask = fwords * 32u - 1u;
    unsigned int err = 0;
    uint32_t epoch = 0;  // per-slot tree sequence number of this launch (kk was zeroed)

    // phase accounting lives in LDS (thread 0 only) to keep it out of registers
    __shared__ unsigned long long s_ph[kPhCount + 1];
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
        const uint32_t nwords = (n + 31u) >> 5;
        const uint32_t tshift = job.tshift;
        const W tmask = (static_cast<W>(1) << tshift) - static_cast<W>(1);
        const W cnt_one = static_cast<W>(1) << tshift;
        const W cnt_minus_one = static_cast<W>(0) - cnt_one;
        auto target_of = [&](W w) -> uint32_t { return static_cast<uint32_t>(w & tmask); };
        auto cnt_of = [&](W w) -> uint32_t { return static_cast<uint32_t>(w >> tshift); };
        auto is_settled = [&](uint32_t v) -> bool {
            return v >= n || ((bits[v >> 5] >> (v & 31u)) & 1u);
        };
        auto set_settled = [&](uint32_t v) { wg_fetch_or(&bits[v >> 5], 1u << (v & 31u)); };
        auto has_in = [&](uint32_t v) -> bool { return (inb[v >> 5] >> (v & 31u)) & 1u; };
        auto set_in = [&](uint32_t v) { atomicOr(&inb[v >> 5], 1u << (v & 31u)); };
        auto clear_in = [&](uint32_t v) { atomicAnd(&inb[v >> 5], ~(1u << (v & 31u))); };

        ++epoch;
        if (tid == 0) {
            s_u = 0;
            s_p = 0;
            s_digest = 0;
            s_roots = 0;
        }
        for (uint32_t i = tid; i < nwords; i += T) {
            bits[i] = 0u;
            if (kInBits) inb[i] = 0u;
        }
        __syncthreads();

        // round 0: the first arrow of every vertex
        for (uint32_t base = wave_base; base < n; base += 2 * T) {
            uint32_t tg[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const uint32_t v = base + q * T + lane;
                tg[q] = v < n ? draw<kWeighted>(job, a.key0, a.key1, v, 0u, t) : n;
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const uint32_t v = base + q * T + lane;
                if (v < n) {
                    word[v] = static_cast<W>(tg[q]);
                    if (tg[q] == n) set_settled(v);
                }
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const uint32_t v = base + q * T + lane;
                wave_append(listA, &s_u, pair(v, tg[q]), v < n && tg[q] != n);
            }
        }
        __syncthreads();
        mark(kPhDraw0);
        uint32_t ucount = uniform(s_u);
        uint64_t *U = listA, *Unext = listB;
        unsigned long long draws = n;
        uint32_t rounds = 0;

        while (ucount > 0) {
            if (++rounds > a.max_rounds || draws > job.step_cap || s_over) {
                err |= kErrStepCap;
                break;
            }
            // in-arrows of unsettled targets from unsettled vertices (no return value:
            // the atomics do not stall the thread)
            for (uint32_t base = tid; base < ucount; base += kR * T) {
                uint32_t tg[kR];
#pragma unroll
                for (int q = 0; q < kR; ++q) {
                    const uint32_t i = base + q * T;
                    tg[q] = i < ucount ? hi32(U[i]) : n;
                }
#pragma unroll
                for (int q = 0; q < kR; ++q) {
                    if (!is_settled(tg[q])) {
                        (void)wg_fetch_add(&word[tg[q]], cnt_one);
                        if (kInBits) set_in(tg[q]);
                    }
                }
            }
            if (tid == 0) s_p = 0;  // last read of s_p was followed by barriers
            __syncthreads();
            mark(kPhIndeg);
            // level 0 of the peel: no in-arrows
            for (uint32_t base = wave_base; base < ucount; base += kR * T) {
                uint64_t it[kR];
                bool leaf[kR];
#pragma unroll
                for (int q = 0; q < kR; ++q) {
                    const uint32_t i = base + q * T + lane;
                    it[q] = i < ucount ? U[i] : 0ull;
                    leaf[q] = false;
                }
#pragma unroll
                for (int q = 0; q < kR; ++q) {
                    const uint32_t i = base + q * T + lane;
                    if (i < ucount)
                        leaf[q] = kInBits ? !has_in(lo32(it[q])) : cnt_of(word[lo32(it[q])]) == 0u;
                }
#pragma unroll
                for (int q = 0; q < kR; ++q) wave_append(peel, &s_p, it[q], leaf[q]);
            }
            __syncthreads();
            mark(kPhLevel0);
            uint32_t lo = 0, hi = min(uniform(s_p), n), nlev = 0;
            if (tid == 0) lvl[0] = 0;
            // peel level by level: a peeled vertex's target loses one in-arrow; the
            // atomic returns the target's own arrow, which goes into the list with it
            while (hi - lo > 64u) {
                if (tid == 0) lvl[nlev + 1] = hi;
                for (uint32_t base = lo + wave_base; base < hi; base += kR * T) {
                    uint32_t tg[kR];
                    W old[kR];
                    bool push[kR];
#pragma unroll
                    for (int q = 0; q < kR; ++q) {
                        const uint32_t i = base + q * T + lane;
                        tg[q] = i < hi ? hi32(peel[i]) : n;
                        push[q] = false;
                        old[q] = 0;
                    }
#pragma unroll
                    for (int q = 0; q < kR; ++q)
                        if (!is_settled(tg[q])) old[q] = wg_fetch_add(&word[tg[q]], cnt_minus_one);
#pragma unroll
                    for (int q = 0; q < kR; ++q) {
                        push[q] = !is_settled(tg[q]) && cnt_of(old[q]) == 1u;
                        if (kInBits && push[q]) clear_in(tg[q]);
                    }
#pragma unroll
                    for (int q = 0; q < kR; ++q)
                        wave_append(peel, &s_p, pair(tg[q], target_of(old[q])), push[q]);
                }
                __syncthreads();
                ++nlev;
                lo = hi;
                hi = min(uniform(s_p), n);
                __syncthreads();  // every wave has read s_p before the next level appends
            }
            // No level is larger than the one before it (a peeled vertex frees at
            // most its own target): once a level fits in one wave, wave 0 peels the
            // rest alone, without workgroup barriers, the frontier compacted
            // through LDS and appended to the list for the sweep.
            const uint32_t tail0 = nlev;
            if (lo < hi) {
                if (wave_base == 0) {
                    uint32_t cnt = hi - lo, pos = hi, nl = nlev;
                    uint64_t it = lane < cnt ? peel[lo + lane] : 0ull;
                    while (cnt > 0) {
                        if (lane == 0) lvl[nl + 1] = pos;
                        const uint32_t tg = hi32(it);
                        bool push = false;
                        W old = 0;
                        if (lane < cnt && !is_settled(tg)) {
                            old = wg_fetch_add(&word[tg], cnt_minus_one);
                            push = cnt_of(old) == 1u;
                            if (kInBits && push) clear_in(tg);
                        }
                        const uint64_t mask = __ballot(push);
                        const uint32_t m = static_cast<uint32_t>(__popcll(mask));
                        if (pos + m > n) {  // only with counts a valid graph cannot produce
                            if (lane == 0) s_over = 1u;
                            break;
                        }
                        if (push) {
                            const uint32_t r =
                                static_cast<uint32_t>(__popcll(mask & ((1ull << lane) - 1ull)));
                            const uint64_t nx = pair(tg, target_of(old));
                            s_tail[r] = nx;
                            peel[pos + r] = nx;
                        }
                        wave_sync();
                        it = lane < m ? s_tail[lane] : 0ull;
                        wave_sync();
                        pos += m;
                        cnt = m;
                        ++nl;
                    }
                    if (lane == 0) {
                        s_p = pos;
                        s_nlev = nl;
                    }
                }
                __syncthreads();
                hi = uniform(s_p);
                nlev = uniform(s_nlev);
            }
            const uint32_t peeled = hi;
            mark(kPhPeel);
            if (peeled == ucount) {  // no cycle left: every vertex reaches u*, the tree is done
                ucount = 0;
                break;
            }
            // reverse sweep: settled when the arrow reaches u* or a settled vertex;
            // the narrow tail levels first by wave 0 alone, then the wide ones
            if (wave_base == 0 && nlev > tail0) {
                for (int32_t top = static_cast<int32_t>(nlev) - 1; top >= static_cast<int32_t>(tail0);
                     top -= 63) {
                    const int32_t li = top + 1 - static_cast<int32_t>(lane);  // lane j: lvl[top + 1 - j]
                    const uint32_t bnd = li >= static_cast<int32_t>(tail0) ? lvl[li] : 0u;
                    const int32_t levels = min(63, top - static_cast<int32_t>(tail0) + 1);
                    for (int32_t j = 0; j < levels; ++j) {
                        const uint32_t a1 = __shfl(bnd, j, 64), a0 = __shfl(bnd, j + 1, 64);
                        if (lane < a1 - a0) {
                            const uint64_t p = peel[a0 + lane];
                            if (is_settled(hi32(p))) set_settled(lo32(p));
                        }
                        wave_sync();
                    }
                }
            }
            __syncthreads();
            for (int32_t L = static_cast<int32_t>(tail0) - 1; L >= 0; --L) {
                const uint32_t a0 = uniform(lvl[L]), a1 = uniform(lvl[L + 1]);
                for (uint32_t i = a0 + tid; i < a1; i += T) {
                    const uint64_t p = peel[i];
                    if (is_settled(hi32(p))) set_settled(lo32(p));
                }
                __syncthreads();
            }
            mark(kPhSweep);
            // split the unsettled vertices: those hanging off a cycle keep their
            // arrow (next list); cycle vertices (in-arrows left) go to a cycle
            // list in the dead peel buffer
            if (tid == 0) {  // last reads of s_u / s_cycles were followed by barriers
                s_u = 0;
                s_cycles = 0;
            }
            __syncthreads();
            uint64_t *__restrict__ cyc = peel;
            for (uint32_t base = wave_base; base < ucount; base += kR * T) {
                uint64_t it[kR];
                W w[kR];
                bool keep[kR], pop[kR];
#pragma unroll
                for (int q = 0; q < kR; ++q) {
                    const uint32_t i = base + q * T + lane;
                    it[q] = i < ucount ? U[i] : pair(n, n);
                    w[q] = 0;
                }
#pragma unroll
                for (int q = 0; q < kR; ++q)
                    if (!kInBits && !is_settled(lo32(it[q]))) w[q] = word[lo32(it[q])];
#pragma unroll
                for (int q = 0; q < kR; ++q) {
                    const uint32_t v = lo32(it[q]);
                    const bool live = !is_settled(v);
                    pop[q] = live && (kInBits ? has_in(v) : cnt_of(w[q]) > 0u);
                    keep[q] = live && !pop[q];
                }
#pragma unroll
                for (int q = 0; q < kR; ++q) {
                    wave_append(Unext, &s_u, it[q], keep[q]);
                    wave_append(cyc, &s_cycles, it[q], pop[q]);
                }
            }
            __syncthreads();
            // the hanging vertices' entries end here; the redrawn ones follow
            const uint32_t u_hang = uniform(s_u);
            if (fwords) {  // every wave reads s_u before the redraw appends
                if (tid == 0) s_rp[0] = s_rp[1] = 0u;
                for (uint32_t i = tid; i < fwords; i += T) filt[i] = 0u;
                __syncthreads();
            }
            // pop every cycle: each cycle vertex draws its next arrow
            const uint32_t ccount = min(uniform(s_cycles), n);
            for (uint32_t base = wave_base; base < ccount; base += 2 * T) {
                uint32_t v[2], k[2], tg[2];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const uint32_t i = base + q * T + lane;
                    v[q] = i < ccount ? lo32(cyc[i]) : n;
                    k[q] = 1u;
                    if (v[q] < n) {
                        const uint64_t kv = kk[v[q]];
                        if (hi32(kv) == epoch) k[q] = lo32(kv);
                    }
                }
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    tg[q] = v[q] < n ? draw<kWeighted>(job, a.key0, a.key1, v[q], k[q], t) : n;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    if (v[q] < n) {
                        if (kInBits) clear_in(v[q]);
                        if (k[q] + 1u > a.k_limit) err |= kErrVisitOverflow;
                        kk[v[q]] = (static_cast<uint64_t>(epoch) << 32) | (k[q] + 1u);
                        // count back to 0 with it, or 1 (redrawn in re-pop pass 0)
                        word[v[q]] = static_cast<W>(tg[q]) | (fwords && tg[q] != n ? cnt_one : W(0));
                        if (tg[q] == n) set_settled(v[q]);
                    }
                }
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    wave_append(Unext, &s_u, pair(v[q], tg[q]), v[q] < n && tg[q] != n);
            }
            __syncthreads();
            // Re-formed 2-cycles: a redrawn vertex u whose new arrow goes to an
            // unsettled tg whose arrow goes back to u closes a cycle of the current
            // arrows, which may be popped at once (any cycle may be popped at any
            // time) instead of a round later with everything that hangs off it.
            // Passes repeat over the vertices just redrawn.  Their tree words carry
            // an in-arrow count of 1 (set by the store of the new arrow) while the
            // pass looks for pairs: a pair whose both ends were redrawn in the same
            // pass is popped by the smaller id, any other by u's lane; a lane that
            // finds no pair clears its own mark (the mark is read only through a
            // word whose target matches, which that lane would have seen).  The
            // popped vertices already sit in the next list with their old targets:
            // the LDS filter flags their ids (modulo its size), and a pass over the
            // list re-reads the word of every flagged entry.  A pass's pops go to one
            // half of the dead peel buffer; one that would overflow it clears the
            // marks and ends the loop, and so does the pass after the last allowed.
            if (fwords) {
                constexpr uint32_t kPasses = 32;
                const uint32_t cap = n >> 1;
                const uint32_t u_end = min(uniform(s_u), n), u_beg = min(u_hang, u_end);
                const uint64_t *cur = Unext + u_beg;
                uint32_t ccur = u_end - u_beg;
                bool any = false;
                for (uint32_t pass = 0; ccur > 0u; ++pass) {
                    uint32_t *rp = &s_rp[pass & 1u];
                    uint64_t *__restrict__ nxt = peel + ((pass & 1u) ? cap : 0u);
                    const bool final = pass == kPasses;
                    for (uint32_t base = wave_base; base < ccur; base += T) {
                        const uint32_t i = base + lane;
                        uint32_t u = n, tg = n;
                        bool lead = false;
                        if (i < ccur) {
                            const uint64_t e = cur[i];
                            u = lo32(e);
                            tg = hi32(e);
                            bool pp = false;
                            if (!final && !is_settled(tg)) {
                                const W w = word[tg];
                                pp = target_of(w) == u;
                                lead = pp && (cnt_of(w) == 0u || u < tg);
                            }
                            if (!pp && tg < n) word[u] = static_cast<W>(tg);
                        }
                        wave_append2(nxt, rp, pair(u, 0u), pair(tg, 0u), lead, cap);
                    }
                    __syncthreads();
                    const uint32_t cn = uniform(*rp);
                    if (cn > cap) {  // not every pop was listed: pop none, clear the marks
                        for (uint32_t i = tid; i < ccur; i += T) {
                            const uint64_t e = cur[i];
                            if (hi32(e) < n) word[lo32(e)] = static_cast<W>(hi32(e));
                        }
                        __syncthreads();
                        break;
                    }
                    if (cn == 0u) break;
                    for (uint32_t i = tid; i < cn; i += T) {
                        const uint32_t v = lo32(nxt[i]);
                        uint32_t k = 1u;
                        const uint64_t kv = kk[v];
                        if (hi32(kv) == epoch) k = lo32(kv);
                        if (k + 1u > a.k_limit) err |= kErrVisitOverflow;
                        const uint32_t tg = draw<kWeighted>(job, a.key0, a.key1, v, k, t);
                        kk[v] = (static_cast<uint64_t>(epoch) << 32) | (k + 1u);
                        word[v] = static_cast<W>(tg) | (tg != n ? cnt_one : W(0));
                        if (tg == n) set_settled(v);
                        nxt[i] = pair(v, tg);
                        atomicOr(&filt[(v & fmask) >> 5], 1u << (v & 31u));
                    }
                    if (tid == 0) s_rp[(pass + 1u) & 1u] = 0u;  // last read before the barrier above
                    draws += cn;
                    any = true;
                    cur = nxt;
                    ccur = cn;
                    __syncthreads();
                }
                if (any) {
                    const uint32_t nu = min(uniform(s_u), n);
                    for (uint32_t i = tid; i < nu; i += T) {
                        const uint32_t v = lo32(Unext[i]);
                        if ((filt[(v & fmask) >> 5] >> (v & 31u)) & 1u)
                            Unext[i] = pair(v, target_of(word[v]));
                    }
                }
                __syncthreads();
            }
            mark(kPhRedraw);
            draws += ccount;
            ucount = min(uniform(s_u), n);
            uint64_t *tmp = U;
            U = Unext;
            Unext = tmp;
        }
        __syncthreads();
        if (err & kErrStepCap) break;  // the call fails; stop this workgroup

        // the tree: top arrows; R, digest, optional per-tree dumps
        unsigned long long my_digest = 0, my_roots = 0;
        const bool want_k = job.visit_counts || job.tree_visits;
        constexpr int kO = 8;  // vertices whose loads each thread keeps in flight
        for (uint32_t base = tid; base < n; base += kO * T) {
            uint32_t tgs[kO], isw[kO];
#pragma unroll
            for (int q = 0; q < kO; ++q) {
                const uint32_t v = base + q * T;
                tgs[q] = v < n ? target_of(word[v]) : 0u;
                isw[q] = v < n && job.iso ? job.iso[v >> 5] : 0u;
            }
#pragma unroll
            for (int q = 0; q < kO; ++q) {
                const uint32_t v = base + q * T;
                if (v >= n) continue;
                const uint32_t tg = tgs[q];
                my_digest += mix64((static_cast<unsigned long long>(v) << 32) | tg);
                // isolated vertices (bitmap from the vertex records) are roots in
                // every tree: their root and draw counts for all the job's trees
                // are added at once, by the workgroup that samples its first tree
                const bool iso = (isw[q] >> (v & 31u)) & 1u;
                if (tg == n) {
                    ++my_roots;
                    if (!iso) atomicAdd(&job.root_counts[v], 1u);
                    else if (ti == 0) atomicAdd(&job.root_counts[v], job.tree_count);
                }
                if (job.parents)
                    job.parents[static_cast<size_t>(ti) * n + v] = static_cast<int32_t>(tg);
                if (want_k) {
                    const uint64_t kv = kk[v];
                    const uint32_t k = hi32(kv) == epoch ? lo32(kv) : 1u;
                    if (job.visit_counts) {
                        if (!iso) atomicAdd(&job.visit_counts[v], static_cast<unsigned long long>(k));
                        else if (ti == 0)
                            atomicAdd(&job.visit_counts[v],
                                      static_cast<unsigned long long>(job.tree_count));
                    }
                    if (job.tree_visits) job.tree_visits[static_cast<size_t>(ti) * n + v] = k;
                }
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

size_t coop_lds_bytes(uint32_t n) { return 4u * ((static_cast<size_t>(n) + 31u) >> 5); }

template <bool kLds, typename W, bool kIn, bool kWt>
hipError_t launch_one(const CoopArgs &a, uint32_t threads, uint32_t repop_words, hipStream_t stream) {
    const size_t lds = (kLds ? (kIn ? 2 : 1) * coop_lds_bytes(a.n_max) : 0) + 4u * repop_words;
    wilson_coop_kernel<kLds, W, kIn, kWt><<<a.slots, threads, lds, stream>>>(a, repop_words);
    return hipGetLastError();
}

template <typename W, bool kWt>
const void *kernel_of(bool lds_bits, bool in_bits) {
    if (!lds_bits) return reinterpret_cast<const void *>(&wilson_coop_kernel<false, W, false, kWt>);
    return in_bits ? reinterpret_cast<const void *>(&wilson_coop_kernel<true, W, true, kWt>)
                   : reinterpret_cast<const void *>(&wilson_coop_kernel<true, W, false, kWt>);
}

template <bool kWt>
const void *kernel_of(bool lds_bits, bool in_bits, bool word32) {
    return word32 ? kernel_of<uint32_t, kWt>(lds_bits, in_bits)
                  : kernel_of<unsigned long long, kWt>(lds_bits, in_bits);
}

int coop_max_active(uint32_t threads, bool lds_bits, bool in_bits, bool word32, uint32_t n_max,
                    bool weighted, uint32_t repop_words) {
    const size_t lds = (lds_bits ? (in_bits ? 2 : 1) * coop_lds_bytes(n_max) : 0) + 4u * repop_words;
    const void *f = weighted ? kernel_of<true>(lds_bits, in_bits, word32)
                             : kernel_of<false>(lds_bits, in_bits, word32);
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, static_cast<int>(threads), lds) !=
        hipSuccess)
        return 0;
    return blocks;
}

hipError_t coop_set_lds_limit(size_t bytes) {
    const int lim = static_cast<int>(bytes);
    for (int m = 0; m < 12; ++m) {
        const bool lds_bits = (m % 3) != 0, in_bits = (m % 3) == 2, word32 = (m / 3) % 2 == 0;
        const void *f = m < 6 ? kernel_of<false>(lds_bits, in_bits, word32)
                              : kernel_of<true>(lds_bits, in_bits, word32);
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <bool kWt>
hipError_t launch_coop(const CoopArgs &a, uint32_t threads, bool lds_bits, bool in_bits,
                       bool word32, uint32_t rw, hipStream_t stream) {
    if (lds_bits && in_bits)
        return word32 ? launch_one<true, uint32_t, true, kWt>(a, threads, rw, stream)
                      : launch_one<true, unsigned long long, true, kWt>(a, threads, rw, stream);
    if (lds_bits)
        return word32 ? launch_one<true, uint32_t, false, kWt>(a, threads, rw, stream)
                      : launch_one<true, unsigned long long, false, kWt>(a, threads, rw, stream);
    return word32 ? launch_one<false, uint32_t, false, kWt>(a, threads, rw, stream)
                  : launch_one<false, unsigned long long, false, kWt>(a, threads, rw, stream);
}

hipError_t launch_wilson_coop(const CoopArgs &a, uint32_t threads, bool lds_bits, bool in_bits,
                              bool word32, bool weighted, uint32_t repop_words, hipStream_t stream) {
    if (a.n_max == 0 || a.item_count == 0 || a.slots == 0) return hipSuccess;
    if (repop_words & (repop_words - 1u)) return hipErrorInvalidValue;  // a power of two or 0
    return weighted ? launch_coop<true>(a, threads, lds_bits, in_bits, word32, repop_words, stream)
                    : launch_coop<false>(a, threads, lds_bits, in_bits, word32, repop_words, stream);
}

}  // namespace fc
