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
//            (merged into the first-arrow pass in round 0)
//   level 0  v with cnt[v] == 0 starts the peel list
//   peel     a peeled x decrements cnt[target(x)]; the one that drops it to 0
//            appends (target, its own target) to the list (a global load of
//            the target's tree word); levels of at most 64 vertices (the long
//            tail) are peeled by one wave without workgroup barriers
//   sweep    peel levels in reverse: x is settled when its target is, else it
//            hangs off a cycle, keeps its arrow and joins the next U
//   cycles   unsettled vertices with cnt[v] != 0 (found by scanning the
//            settled bitmap and the fields) were never peeled: they lie on a
//            cycle and draw their next arrow (cnt[v] back to 0)
// A count is exact for every unsettled vertex: after the peel, peeled
// vertices are at 0 and cycle vertices at 1 (one arrow from the cycle, a
// functional graph's leftover after Kahn peeling is a union of cycles), so
// the redraw pass leaves all unsettled counts at 0 before the next count.
// Counts of settled vertices are never read again; they stay at most the
// degree, so no field overflows into its neighbour.
//
// Ids fit in 18 bits (a tree whose fields fit in LDS has n < 2^18), which
// leaves room to carry each vertex's draw count k_v with its arrow:
//   word[v]  u64 global  internal target | original target << 18 | k_v << 36
//                        (u* = n in both numberings)
//   lists    u64 global  v | internal target << 18: two unsettled lists and
//                        the peel order (reused for the cycle list)
//   levels   u32 global  peel level boundaries
//   LDS      count fields (4/8/16/32 bits by class), then the settled bitmap
// so redrawing a cycle vertex touches no per-vertex array besides its word
// (whose k_v it reads, except in round 0, where every k_v is 1).
// Isolated vertices (internal ids [n3, n)) take no part in the rounds: only
// the output visits them.
#include "fc_kernels.hpp"
#include "fc_wave.hpp"

namespace fc {

namespace {

constexpr uint32_t kIdBits = kRelabelIdBits;
constexpr uint32_t kIdMask = (1u << kIdBits) - 1u;
constexpr uint32_t kKShift = 2 * kIdBits;
constexpr uint32_t kKMax = (1u << (64 - kKShift)) - 1u;  // largest draw count a word holds

// Makes x live at this point: its first use is here, not earlier (an empty
// asm statement; it reads and writes no memory).
__device__ __forceinline__ void hold_u64(uint64_t &x) { asm volatile("" : "+v"(x)); }

// list entry / tree word fields
__device__ __forceinline__ uint32_t f_lo(uint64_t w) { return static_cast<uint32_t>(w) & kIdMask; }
__device__ __forceinline__ uint32_t f_mid(uint64_t w) {
    return static_cast<uint32_t>(w >> kIdBits) & kIdMask;
}
__device__ __forceinline__ uint32_t f_k(uint64_t w) { return static_cast<uint32_t>(w >> kKShift); }
__device__ __forceinline__ uint64_t pack(uint32_t lo, uint32_t mid, uint32_t k) {
    return static_cast<uint64_t>(lo) | (static_cast<uint64_t>(mid) << kIdBits) |
           (static_cast<uint64_t>(k) << kKShift);
}

// Per-phase clock sums: first arrows, in-arrow count + peel level 0, wide peel
// levels, narrow (single-wave) peel levels, reverse sweep (with the next
// unsettled list), cycle scan, cycle popping, output.
enum Phase : int { kPhDraw0 = 0, kPhLevel0, kPhPeel, kPhTail, kPhSweep, kPhSplit, kPhCycles,
                   kPhOutput, kPhCount };

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

// Arrow number k (0-based) of the vertex with record r in tree t: its tree
// word with draw count k + 1 (internal | original target; u* = n in both).
// kWeighted: the job may carry running weight sums (weighted step).
template <bool kWeighted>
__device__ __forceinline__ uint64_t draw(const CoopJob &j, const VRec &r, uint32_t key0,
                                         uint32_t key1, uint32_t k, uint32_t t) {
    const uint32_t orig = r.always_root & 0x7FFFFFFFu;
    const Philox4 x = philox4x32_10(orig, k, t, j.stream_id, key0, key1);
    const uint64_t kbits = static_cast<uint64_t>(k + 1u) << kKShift;
    if ((r.always_root >> 31) || x.x0 < r.thr) return pack(j.n, j.n, 0u) | kbits;
    const uint32_t idx = neighbour_entry<kWeighted>(r, x.x1, j.wsum, j.wthr);
    return j.adj[r.start + static_cast<int32_t>(idx)] | kbits;
}

// Items per lane per pass iteration (independent loads in flight per lane):
// streaming passes (R), wide peel levels, where each item may add a random
// load (RP), passes that also draw arrows (RD, RC: more registers each);
// middle peel levels (more than one wave's worth, at most Slots per thread)
// keep their entries in registers; registers per lane that hold a window of
// narrow peel levels for the sweep (up to 64 TailRegs entries); vertices per
// thread whose loads the output pass keeps in flight (O).  The lean
// shape (workgroups of at most 512 threads) holds fewer, so that its
// registers leave room for six waves per SIMD instead of four.
template <bool kLean> struct LdsShape {
    static constexpr int R = 8, RP = 4, RD = 2, RC = 2, Slots = 2, TailRegs = 6, O = 8;
};
template <> struct LdsShape<true> {
    static constexpr int R = 2, RP = 2, RD = 1, RC = 1, Slots = 1, TailRegs = 3, O = 4;
};

// Passes of the re-formed 2-cycle pops per round (an optimisation that may
// stop at any pass: the next round pops what is left).
constexpr uint32_t kRepopPasses = 32;

template <bool kWeighted, bool kRepop, bool kLean>
__global__ __launch_bounds__(kLean ? 512 : 1024) __attribute__((amdgpu_waves_per_eu(kLean ? 6 : 1)))
void wilson_lds_kernel(CoopArgs a) {
    constexpr int kR = LdsShape<kLean>::R;
    constexpr int kRP = LdsShape<kLean>::RP;
    constexpr int kRD = LdsShape<kLean>::RD;
    constexpr int kRC = LdsShape<kLean>::RC;
    constexpr int kSlots = LdsShape<kLean>::Slots;
    constexpr int kTailRegs = LdsShape<kLean>::TailRegs;
    extern __shared__ uint32_t s_lds[];
    __shared__ uint32_t s_item, s_u, s_p, s_cycles, s_over, s_nlev, s_rp, s_rp_over;
    __shared__ unsigned long long s_digest, s_roots;
    __shared__ unsigned long long s_ph[kPhCount + 1];

    const uint32_t T = blockDim.x;
    const uint32_t tid = threadIdx.x;
    const uint32_t wave_base = tid & ~63u;
    const uint32_t lane = tid & 63u;
    const size_t slot = blockIdx.x;
    const size_t stride = a.n_max;
    uint64_t *const slot_word = a.word ? static_cast<uint64_t *>(a.word) + slot * stride : nullptr;
    uint64_t *__restrict__ listA = a.lists + slot * (3ull * stride);
    uint64_t *__restrict__ listB = listA + stride;
    uint64_t *__restrict__ peel = listB + stride;
    uint32_t *__restrict__ lvl = a.levels + slot * (stride + 2);
    unsigned int err = 0;

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
        const uint32_t n = job.n;    // also the id of u*
        const uint32_t nl = job.n3;  // vertices that are not isolated: ids [0, nl)
        // the tree's words: its own pre-drawn array, or the slot's
        uint64_t *__restrict__ word = a.pre ? a.pre + static_cast<size_t>(item) * stride : slot_word;
        const CountLayout L = count_layout(nl, job.n0, job.n1, job.n2);
        const Classes C{job.n0, job.n1, job.n2, L.o1, L.o2, L.o3};
        uint32_t *__restrict__ bits = s_lds + L.ob;

        // targets are u* or vertices in [0, nl): isolated vertices have no in-arrows
        auto is_settled = [&](uint32_t v) -> bool {
            return v >= nl || ((bits[v >> 5] >> (v & 31u)) & 1u);
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
        if (a.pre) {  // arrows drawn already: stream them
            for (uint32_t base = wave_base; base < nl; base += kR * T) {
                uint64_t w[kR];
                bool live[kR];
#pragma unroll
                for (int q = 0; q < kR; ++q) {
                    const uint32_t v = base + q * T + lane;
                    w[q] = v < nl ? word[v] : pack(n, n, 0u);
                }
#pragma unroll
                for (int q = 0; q < kR; ++q) {
                    const uint32_t v = base + q * T + lane;
                    live[q] = v < nl && f_lo(w[q]) != n;
                    if (v < nl) {
                        if (live[q]) count_add(f_lo(w[q]));
                        else set_settled(v);
                    }
                    w[q] = pack(v, f_lo(w[q]), 0u);
                }
                wave_append_many<kR>(listA, &s_u, n, &s_over, w, live);
            }
        } else {
        // (records are loaded one iteration ahead, so each iteration waits for
        // one global load, the neighbour gather, instead of two in a row)
        VRec r[kRD] = {};
#pragma unroll
        for (int q = 0; q < kRD; ++q) {
            const uint32_t v = wave_base + q * T + lane;
            if (v < nl) r[q] = load_vrec(job.vrec, v);
        }
        for (uint32_t base = wave_base; base < nl; base += kRD * T) {
            VRec rn[kRD] = {};
            uint64_t w[kRD];
#pragma unroll
            for (int q = 0; q < kRD; ++q) {
                const uint32_t v = base + (kRD + q) * T + lane;
                if (v < nl) rn[q] = load_vrec(job.vrec, v);
            }
#pragma unroll
            for (int q = 0; q < kRD; ++q) {
                const uint32_t v = base + q * T + lane;
                w[q] = v < nl ? draw<kWeighted>(job, r[q], a.key0, a.key1, 0u, t)
                              : pack(n, n, 0u);
            }
            bool live[kRD];
#pragma unroll
            for (int q = 0; q < kRD; ++q) {
                const uint32_t v = base + q * T + lane;
                live[q] = v < nl && f_lo(w[q]) != n;
                if (v < nl) {
                    word[v] = w[q];
                    if (live[q]) count_add(f_lo(w[q]));
                    else set_settled(v);
                }
                w[q] = pack(v, f_lo(w[q]), 0u);
            }
            wave_append_many<kRD>(listA, &s_u, n, &s_over, w, live);
#pragma unroll
            for (int q = 0; q < kRD; ++q) r[q] = rn[q];
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
            const bool first = rounds == 1;
            if (!first) {
                for (uint32_t base = tid; base < ucount; base += kR * T) {
                    uint32_t tg[kR];
#pragma unroll
                    for (int q = 0; q < kR; ++q) {
                        const uint32_t i = base + q * T;
                        tg[q] = i < ucount ? f_mid(U[i]) : n;
                    }
#pragma unroll
                    for (int q = 0; q < kR; ++q)
                        if (!is_settled(tg[q])) count_add(tg[q]);
                }
                __syncthreads();
            }
            // level 0 of the peel: no in-arrows (s_p is 0 here: reset at the
            // tree's start and before the sweep, both followed by a barrier)
            for (uint32_t base = wave_base; base < ucount; base += kR * T) {
                uint64_t it[kR];
                bool leaf[kR];
#pragma unroll
                for (int q = 0; q < kR; ++q) {
                    const uint32_t i = base + q * T + lane;
                    it[q] = i < ucount ? U[i] : pack(n, n, 0u);
                }
#pragma unroll
                for (int q = 0; q < kR; ++q) {
                    const uint32_t v = f_lo(it[q]);
                    leaf[q] = v < nl && count_of(v) == 0u;
                }
                wave_append_many<kR>(peel, &s_p, n, &s_over, it, leaf);
            }
            __syncthreads();
            mark(kPhLevel0);
            uint32_t lo = 0, hi = min(uniform(s_p), n), nlev = 0;
            if (tid == 0) lvl[0] = 0;
            while (hi - lo > kSlots * T) {
                if (tid == 0) lvl[nlev + 1] = hi;
                // (the level's entries are loaded one iteration ahead; entries
                // appended meanwhile lie beyond hi)
                uint32_t tg[kRP];
#pragma unroll
                for (int q = 0; q < kRP; ++q) {
                    const uint32_t i = lo + wave_base + q * T + lane;
                    tg[q] = i < hi ? f_mid(peel[i]) : n;
                }
                for (uint32_t base = lo + wave_base; base < hi; base += kRP * T) {
                    uint32_t tgn[kRP];
                    bool push[kRP];
                    uint64_t nx[kRP];
#pragma unroll
                    for (int q = 0; q < kRP; ++q) {
                        const uint32_t i = base + (kRP + q) * T + lane;
                        tgn[q] = i < hi ? f_mid(peel[i]) : n;
                        push[q] = false;
                    }
#pragma unroll
                    for (int q = 0; q < kRP; ++q)
                        if (!is_settled(tg[q])) push[q] = count_dec(tg[q]) == 1u;
#pragma unroll
                    for (int q = 0; q < kRP; ++q) nx[q] = push[q] ? word[tg[q]] : 0ull;
#pragma unroll
                    for (int q = 0; q < kRP; ++q) nx[q] = pack(tg[q], f_lo(nx[q]), 0u);
                    wave_append_many<kRP>(peel, &s_p, n, &s_over, nx, push);
#pragma unroll
                    for (int q = 0; q < kRP; ++q) tg[q] = tgn[q];
                }
                __syncthreads();
                ++nlev;
                lo = hi;
                hi = min(uniform(s_p), n);
                __syncthreads();  // every wave has read s_p before the next level appends
            }
            // Levels of at most kSlots entries per thread (and more than one
            // wave's worth): the frontier stays in registers, in the threads that
            // freed it, so no level reloads its entries from the list, and the
            // barriers between levels order LDS accesses only (the list and the
            // level bounds are read after the full barrier that ends this part).
            // Each pushed entry's target word is loaded right away, a level ahead
            // of its use, so that the load overlaps the appends and barriers.
            const uint32_t tA = nlev;
            if (hi - lo > 64u) {
                uint64_t it[kSlots], wt[kSlots];
                bool have[kSlots];
#pragma unroll
                for (int q = 0; q < kSlots; ++q) {
                    const uint32_t i = lo + q * T + tid;
                    have[q] = i < hi;
                    it[q] = have[q] ? peel[i] : 0ull;
                }
#pragma unroll
                for (int q = 0; q < kSlots; ++q) {
                    const uint32_t tg = f_mid(it[q]);
                    wt[q] = word[have[q] && tg < nl ? tg : 0u];
                }
                for (;;) {
                    if (tid == 0) lvl[nlev + 1] = hi;
                    bool push[kSlots];
#pragma unroll
                    for (int q = 0; q < kSlots; ++q) {
                        const uint32_t tg = f_mid(it[q]);
                        push[q] = false;
                        if (have[q] && !is_settled(tg)) push[q] = count_dec(tg) == 1u;
                    }
                    uint64_t nx[kSlots];
#pragma unroll
                    for (int q = 0; q < kSlots; ++q) {
                        hold_u64(wt[q]);
                        nx[q] = push[q] ? pack(f_mid(it[q]), f_lo(wt[q]), 0u) : 0ull;
                    }
#pragma unroll
                    for (int q = 0; q < kSlots; ++q) {
                        const uint32_t tg = f_mid(nx[q]);
                        wt[q] = word[push[q] && tg < nl ? tg : 0u];
                    }
                    wave_append_many<kSlots>(peel, &s_p, n, &s_over, nx, push);
                    lds_barrier();
                    ++nlev;
                    lo = hi;
                    hi = min(uniform(s_p), n);
                    lds_barrier();  // every wave has read s_p before the next level appends
#pragma unroll
                    for (int q = 0; q < kSlots; ++q) {
                        it[q] = nx[q];
                        have[q] = push[q];
                    }
                    if (hi - lo <= 64u) break;
                }
                __syncthreads();  // the list's entries are read below
            }
            // No level is larger than the one before it (a peeled vertex frees at
            // most its own target), so once a level fits in one wave, wave 0 peels
            // the rest alone, without workgroup barriers.  Each lane frees at most
            // one vertex per level, so the frontier stays in the lanes that freed
            // it (no compaction); it is also appended to the list for the sweep.
            const uint32_t tail0 = nlev;
            mark(kPhPeel);
            if (lo < hi) {
                if (wave_base == 0) {
                    uint32_t pos = hi, lv = nlev;  // lv: the level being peeled
                    bool have = lane < hi - lo;
                    uint64_t it = have ? peel[lo + lane] : 0ull;
                    hold_u64(it);  // waited for here, not at every level's start
                    const uint64_t below = (1ull << lane) - 1ull;
                    while (__ballot(have) != 0ull) {
                        const uint32_t tg = f_mid(it);
                        // the target's word is loaded (by every lane, in bounds)
                        // before its count is known to drop to 0, and first used
                        // after the two LDS accesses, which its load then overlaps
                        uint64_t wt = word[have && tg < nl ? tg : 0u];
                        if (lane == 0) lvl[lv + 1] = pos;
                        bool push = false;
                        if (have && !is_settled(tg)) push = count_dec(tg) == 1u;
                        hold_u64(wt);
                        const uint64_t nx = push ? pack(tg, f_lo(wt), 0u) : 0ull;
                        const uint64_t mask = __ballot(push);
                        const uint32_t m = static_cast<uint32_t>(__popcll(mask));
                        if (pos + m > n) {
                            if (lane == 0) s_over = 1u;
                            break;
                        }
                        if (push) peel[pos + static_cast<uint32_t>(__popcll(mask & below))] = nx;
                        it = nx;
                        have = push;
                        pos += m;
                        ++lv;
                    }
                    if (lane == 0) {
                        s_p = pos;
                        s_nlev = lv;
                    }
                }
                __syncthreads();
                hi = uniform(s_p);
                nlev = uniform(s_nlev);
            }
            const uint32_t peeled = hi;
            mark(kPhTail);
            if (peeled == ucount) {  // no cycle: every unsettled vertex reaches u*
                ucount = 0;
                break;
            }
            // every wave has read s_p and s_nlev: reset the list tails (the next
            // unsettled list, the cycle list, the next round's peel)
            __syncthreads();
            if (tid == 0) {
                s_u = 0;
                s_cycles = 0;
                s_p = 0;
            }
            __syncthreads();
            // reverse sweep: a peeled vertex is settled when its target is; the
            // others hang off a cycle, keep their arrow and go to the next
            // unsettled list.  The narrow tail levels first, by wave 0 alone
            // (level boundaries fetched 63 at a time), then the wide ones.
            // The tail's list tail is kept in a register (s_u is 0 and no other
            // wave appends until the barrier after it).  The tail levels are
            // taken in windows of consecutive levels with at most 64 kTailRegs
            // entries: a window's entries are loaded into registers at once
            // (entry A + 64 q + lane in buf[q]), its levels settled with LDS
            // accesses only, and its hanging entries appended after it (a load
            // or store inside the level loop would make each level wait for the
            // level before's store: loads and stores share one counter).
            if (wave_base == 0 && nlev > tail0) {
                uint32_t ut = 0;
                const uint64_t below = (1ull << lane) - 1ull;
                for (int32_t top = static_cast<int32_t>(nlev) - 1; top >= static_cast<int32_t>(tail0);
                     top -= 63) {
                    const int32_t li = top + 1 - static_cast<int32_t>(lane);  // lane j: lvl[top + 1 - j]
                    const uint32_t bnd = li >= static_cast<int32_t>(tail0) ? lvl[li] : 0u;
                    const int32_t levels = min(63, top - static_cast<int32_t>(tail0) + 1);
                    for (int32_t j = 0; j < levels;) {
                        // levels j .. je - 1 of the batch (level j has at most 64
                        // entries, so the window holds at least one level)
                        const uint32_t B = lane_of(bnd, j);
                        const int32_t ln = static_cast<int32_t>(lane);
                        const uint64_t fit =
                            __ballot(ln > j && ln <= levels && B - bnd <= 64u * kTailRegs);
                        const int32_t je = fit ? 63 - __builtin_clzll(fit) : j + 1;
                        const uint32_t A = lane_of(bnd, je);
                        uint64_t buf[kTailRegs];
#pragma unroll
                        for (int q = 0; q < kTailRegs; ++q) {
                            const uint32_t i = A + 64u * q + lane;
                            buf[q] = i < B ? peel[i] : 0ull;
                        }
                        uint32_t hm = 0;  // bit q: buf[q] hangs
                        for (; j < je; ++j) {
                            const uint32_t a1 = lane_of(bnd, j), a0 = lane_of(bnd, j + 1);
                            // a level has at most 64 entries: one per lane at most
                            uint64_t p = 0;
                            int sel = -1;
#pragma unroll
                            for (int q = 0; q < kTailRegs; ++q) {
                                const uint32_t i = A + 64u * q + lane;
                                if (i >= a0 && i < a1) {
                                    p = buf[q];
                                    sel = q;
                                }
                            }
                            if (sel >= 0) {
                                if (is_settled(f_mid(p))) set_settled(f_lo(p));
                                else hm |= 1u << sel;
                            }
                        }
#pragma unroll
                        for (int q = 0; q < kTailRegs; ++q) {
                            const bool hang = (hm >> q) & 1u;
                            const uint64_t mask = __ballot(hang);
                            if (hang) {
                                const uint32_t at = ut + static_cast<uint32_t>(__popcll(mask & below));
                                if (at < n) Unext[at] = buf[q];
                            }
                            ut += static_cast<uint32_t>(__popcll(mask));
                        }
                    }
                }
                if (lane == 0) {
                    s_u = ut;
                    if (ut > n) s_over = 1u;
                }
            }
            __syncthreads();
            // the middle levels [tA, tail0): at most kSlots entries per thread;
            // each thread loads its entries of the next level while it settles
            // the current one, and the barriers between levels order LDS only
            // (the next unsettled list is read after a full barrier)
            if (tail0 > tA) {
                const int32_t ta = static_cast<int32_t>(tA);
                for (int32_t top = static_cast<int32_t>(tail0) - 1; top >= ta; top -= 63) {
                    const int32_t li = top + 1 - static_cast<int32_t>(lane);  // lane j: lvl[top + 1 - j]
                    const uint32_t bnd = li >= ta ? lvl[li] : 0u;
                    const int32_t levels = min(63, top - ta + 1);
                    // level top - j: [bnd of lane j + 1, bnd of lane j)
                    uint64_t p[kSlots];
                    {
                        const uint32_t a1 = lane_of(bnd, 0), a0 = lane_of(bnd, 1);
#pragma unroll
                        for (int q = 0; q < kSlots; ++q) {
                            const uint32_t i = a0 + q * T + tid;
                            p[q] = i < a1 ? peel[i] : pack(n, n, 0u);
                        }
                    }
                    for (int32_t j = 0; j < levels; ++j) {
                        uint64_t cur[kSlots];
#pragma unroll
                        for (int q = 0; q < kSlots; ++q) cur[q] = p[q];
                        if (j + 1 < levels) {
                            const uint32_t a1 = lane_of(bnd, j + 1), a0 = lane_of(bnd, j + 2);
#pragma unroll
                            for (int q = 0; q < kSlots; ++q) {
                                const uint32_t i = a0 + q * T + tid;
                                p[q] = i < a1 ? peel[i] : pack(n, n, 0u);
                            }
                        }
                        bool hang[kSlots];
#pragma unroll
                        for (int q = 0; q < kSlots; ++q) {
                            hang[q] = false;
                            if (f_lo(cur[q]) < n) {
                                if (is_settled(f_mid(cur[q]))) set_settled(f_lo(cur[q]));
                                else hang[q] = true;
                            }
                        }
                        wave_append_many<kSlots>(Unext, &s_u, n, &s_over, cur, hang);
                        lds_barrier();
                    }
                }
            }
            for (int32_t Lv = static_cast<int32_t>(tA) - 1; Lv >= 0; --Lv) {
                const uint32_t a0 = uniform(lvl[Lv]), a1 = uniform(lvl[Lv + 1]);
                for (uint32_t base = a0 + wave_base; base < a1; base += kR * T) {
                    uint64_t p[kR];
                    bool hang[kR];
#pragma unroll
                    for (int q = 0; q < kR; ++q) {
                        const uint32_t i = base + q * T + lane;
                        p[q] = i < a1 ? peel[i] : pack(n, n, 0u);
                    }
#pragma unroll
                    for (int q = 0; q < kR; ++q) {
                        hang[q] = false;
                        if (f_lo(p[q]) < n) {
                            if (is_settled(f_mid(p[q]))) set_settled(f_lo(p[q]));
                            else hang[q] = true;
                        }
                    }
                    wave_append_many<kR>(Unext, &s_u, n, &s_over, p, hang);
                }
                __syncthreads();
            }
            mark(kPhSweep);
            // the cycle vertices: unsettled and never peeled, i.e. an in-arrow
            // count left (1: the arrow of the cycle predecessor), found by a scan
            // of the settled bitmap and the fields, in id order, into the dead
            // peel buffer
            uint64_t *__restrict__ cyc = peel;
            const uint32_t nbw = (nl + 31u) >> 5;
            for (uint32_t wb = wave_base; wb < nbw; wb += T) {
                const uint32_t wi = wb + lane;
                uint32_t m = 0;
                if (wi < nbw) {
                    m = ~bits[wi];
                    if (wi == nbw - 1u && (nl & 31u)) m &= (1u << (nl & 31u)) - 1u;
                }
                while (__ballot(m != 0u)) {
                    uint64_t e[kR];
                    bool pop[kR];
#pragma unroll
                    for (int q = 0; q < kR; ++q) {
                        const uint32_t v = m != 0u ? (wi << 5) + static_cast<uint32_t>(__builtin_ctz(m)) : 0u;
                        pop[q] = m != 0u && count_of(v) != 0u;
                        e[q] = pack(v, 0u, 0u);
                        m &= m - 1u;
                    }
                    wave_append_many<kR>(cyc, &s_cycles, n, &s_over, e, pop);
                }
            }
            const uint32_t u_hang = uniform(s_u);  // the sweep's entries (final since its barrier)
            __syncthreads();
            mark(kPhSplit);
            // pop every cycle: each cycle vertex draws its next arrow (in round 0
            // every vertex has drawn once; later the count is in its word)
            const uint32_t ccount = min(uniform(s_cycles), n);
            for (uint32_t base = wave_base; base < ccount; base += kRC * T) {
                uint32_t v[kRC], k[kRC];
                VRec r[kRC];
                uint64_t w[kRC];
#pragma unroll
                for (int q = 0; q < kRC; ++q) {
                    const uint32_t i = base + q * T + lane;
                    v[q] = i < ccount ? f_lo(cyc[i]) : n;
                    k[q] = 1u;
                    if (v[q] < n) {
                        r[q] = load_vrec(job.vrec, v[q]);
                        if (!first) k[q] = f_k(word[v[q]]);
                    }
                }
#pragma unroll
                for (int q = 0; q < kRC; ++q) {
                    if (v[q] < n && k[q] >= min(kKMax, a.k_limit)) {  // count past the limit
                        err |= kErrVisitOverflow;
                        v[q] = n;
                    }
                    w[q] = v[q] < n ? draw<kWeighted>(job, r[q], a.key0, a.key1, k[q], t)
                                    : pack(n, n, 0u);
                }
                bool live[kRC];
#pragma unroll
                for (int q = 0; q < kRC; ++q) {
                    live[q] = v[q] < n && f_lo(w[q]) != n;
                    if (v[q] < n) {
                        (void)count_dec(v[q]);  // the cycle's arrow into v is gone
                        word[v[q]] = w[q];
                        if (!live[q]) set_settled(v[q]);
                    }
                    // (the entry carries the new draw count for the re-pop passes)
                    w[q] = pack(v[q], f_lo(w[q]), f_k(w[q]));
                }
                wave_append_many<kRC>(Unext, &s_u, n, &s_over, w, live);
            }
            __syncthreads();
            // Re-formed 2-cycles: a redrawn vertex u whose new arrow goes to an
            // unsettled tg whose arrow goes back to u closes a cycle of the current
            // arrows, which may be popped at once (any cycle may be popped at any
            // time) instead of a round later with everything that hangs off it.
            // The pair is popped by u's lane, or by the smaller id's when both were
            // redrawn in the same pass.  In-arrow fields, all 0 here for unsettled
            // vertices, mark "redrawn in this pass" (+1, cleared after the
            // detection) and "popped again this round" (+2).  The popped vertices are
            // already in the next list, with their old targets: a pass over that
            // list re-reads the target of every entry marked +2 and clears the mark.
            // The pass lists carry each vertex's draw count (from its new word, or
            // from the partner's word read for the detection), so a redraw reads
            // no tree word.
            // A pass's pops go to one half of the dead peel buffer; a pass that
            // would overflow it ends the loop.
            if (kRepop) {
                const uint32_t cap = n >> 1;
                const uint32_t u_end = min(uniform(s_u), n), u_beg = min(u_hang, u_end);
                const uint64_t *cur = Unext + u_beg;
                uint32_t ccur = u_end - u_beg;
                bool any = false;
                for (uint32_t pass = 0; ccur > 0u && pass < kRepopPasses; ++pass) {
                    uint64_t *nxt = peel + ((pass & 1u) ? cap : 0u);
                    for (uint32_t i = tid; i < ccur; i += T) count_add(f_lo(cur[i]));
                    if (tid == 0) {
                        s_rp = 0;
                        s_rp_over = 0;
                    }
                    __syncthreads();
                    for (uint32_t base = wave_base; base < ccur; base += T) {
                        const uint32_t i = base + lane;
                        uint64_t e[2] = {0ull, 0ull};
                        bool pp[2] = {false, false};
                        if (i < ccur) {
                            const uint64_t c = cur[i];
                            const uint32_t u = f_lo(c), tg = f_mid(c);
                            if (tg < nl && !is_settled(tg)) {
                                const uint64_t wt = word[tg];
                                if (f_lo(wt) == u && ((count_of(tg) & 1u) == 0u || u < tg)) {
                                    // both ends with their draw counts so far
                                    e[0] = pack(u, 0u, f_k(c));
                                    e[1] = pack(tg, 0u, f_k(wt));
                                    pp[0] = pp[1] = true;
                                }
                            }
                        }
                        wave_append_many<2>(nxt, &s_rp, cap, &s_rp_over, e, pp);
                    }
                    __syncthreads();
                    for (uint32_t i = tid; i < ccur; i += T) (void)count_dec(f_lo(cur[i]));
                    const uint32_t cn = uniform(s_rp);
                    if (uniform(s_rp_over) != 0u || cn == 0u) break;
                    for (uint32_t i = tid; i < cn; i += T) {
                        const uint32_t v = f_lo(nxt[i]);
                        const uint32_t k = f_k(nxt[i]);
                        if (k >= min(kKMax, a.k_limit)) {  // count past the limit
                            err |= kErrVisitOverflow;
                            nxt[i] = pack(v, n, 0u);
                            continue;
                        }
                        const uint64_t nw = draw<kWeighted>(job, load_vrec(job.vrec, v), a.key0,
                                                            a.key1, k, t);
                        word[v] = nw;
                        if (f_lo(nw) == n) set_settled(v);
                        nxt[i] = pack(v, f_lo(nw), f_k(nw));
                        if ((count_of(v) & 2u) == 0u) {  // first pop this round: mark it
                            const Field f = field_of(C, v);
                            atomicAdd(&s_lds[f.w], 2u << f.sh);
                        }
                    }
                    draws += cn;
                    any = true;
                    cur = nxt;
                    ccur = cn;
                    __syncthreads();
                }
                if (any) {
                    const uint32_t nu = min(uniform(s_u), n);
                    for (uint32_t i = tid; i < nu; i += T) {
                        const uint32_t v = f_lo(Unext[i]);
                        if (count_of(v) & 2u) {
                            Unext[i] = pack(v, f_lo(word[v]), 0u);
                            const Field f = field_of(C, v);
                            atomicAdd(&s_lds[f.w], 0u - (2u << f.sh));
                        }
                    }
                }
                __syncthreads();
            }
            mark(kPhCycles);
            draws += ccount;
            ucount = min(uniform(s_u), n);
            uint64_t *tmp = U;
            U = Unext;
            Unext = tmp;
        }
        __syncthreads();
        if (err & kErrStepCap) break;

        unsigned long long my_digest = 0, my_roots = 0;
        const bool want_k = job.visit_counts || job.tree_visits;
        constexpr int kO = LdsShape<kLean>::O;
        for (uint32_t base = tid; base < nl; base += kO * T) {
            uint64_t ws[kO];
            uint32_t ovs[kO];
#pragma unroll
            for (int q = 0; q < kO; ++q) {
                const uint32_t v = base + q * T;
                ws[q] = v < nl ? word[v] : 0ull;
                ovs[q] = v < nl ? job.orig[v] : 0u;
            }
#pragma unroll
            for (int q = 0; q < kO; ++q) {
                if (base + q * T >= nl) continue;
                const uint64_t w = ws[q];
                const uint32_t ov = ovs[q];
                const uint32_t otg = f_mid(w);
                my_digest += mix64((static_cast<unsigned long long>(ov) << 32) | otg);
                if (f_lo(w) == n) {
                    ++my_roots;
                    atomicAdd(&job.root_counts[ov], 1u);
                }
                if (job.parents)
                    job.parents[static_cast<size_t>(ti) * n + ov] = static_cast<int32_t>(otg);
                if (want_k) {
                    const uint32_t k = f_k(w);
                    if (job.visit_counts)
                        atomicAdd(&job.visit_counts[ov], static_cast<unsigned long long>(k));
                    if (job.tree_visits) job.tree_visits[static_cast<size_t>(ti) * n + ov] = k;
                }
            }
        }
        // isolated vertices: a root after one draw in every tree.  Their digest
        // terms are added per tree; their root and draw counts for all the job's
        // trees at once, by the workgroup that samples its first tree.
        for (uint32_t base = nl + tid; base < n; base += kO * T) {
            uint32_t ovs[kO];
#pragma unroll
            for (int q = 0; q < kO; ++q) {
                const uint32_t v = base + q * T;
                ovs[q] = v < n ? job.orig[v] : 0u;
            }
#pragma unroll
            for (int q = 0; q < kO; ++q) {
                if (base + q * T >= n) continue;
                const uint32_t ov = ovs[q];
                my_digest += mix64((static_cast<unsigned long long>(ov) << 32) | n);
                ++my_roots;
                if (job.parents)
                    job.parents[static_cast<size_t>(ti) * n + ov] = static_cast<int32_t>(n);
                if (job.tree_visits) job.tree_visits[static_cast<size_t>(ti) * n + ov] = 1u;
                if (ti == 0) {
                    atomicAdd(&job.root_counts[ov], job.tree_count);
                    if (job.visit_counts)
                        atomicAdd(&job.visit_counts[ov], static_cast<unsigned long long>(job.tree_count));
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

// Trees per workgroup of the pre-draw kernel (each thread owns one vertex and
// draws its first arrow in that many trees).
constexpr uint32_t kPreTrees = 16;
constexpr uint32_t kPreThreads = 256;

// First arrow of a weighted graph's vertex in tree t, given the first chunk
// of its row's step thresholds (loaded once for all of the vertex's trees):
// the same word as draw<true>(j, r, key0, key1, 0, t).
__device__ __forceinline__ uint64_t draw_first_w(const CoopJob &j, const VRec &r,
                                                 const uint32_t (&t0)[kWeightedScan],
                                                 uint32_t key0, uint32_t key1, uint32_t t) {
    const uint32_t orig = r.always_root & 0x7FFFFFFFu;
    const Philox4 x = philox4x32_10(orig, 0u, t, j.stream_id, key0, key1);
    const uint64_t kbits = 1ull << kKShift;
    if ((r.always_root >> 31) || x.x0 < r.thr) return pack(j.n, j.n, 0u) | kbits;
    const uint32_t m = r.deg - 1;
    const uint32_t idx = (x.x1 - 1u >= 0xFFFFFFFEu || m > kWeightedScan)
                             ? weighted_entry(j.wsum + r.start, j.wthr + r.start, r.deg, x.x1)
                             : weighted_chunk_count(t0, 0u, m, x.x1);
    return j.adj[r.start + static_cast<int32_t>(idx)] | kbits;
}

template <bool kWeighted>
__global__ __launch_bounds__(kPreThreads) void lds_predraw_kernel(CoopArgs a, uint32_t groups) {
    const CoopJob &job = a.single;
    const uint32_t v = blockIdx.x * kPreThreads + threadIdx.x;
    if (v >= job.n3) return;
    const VRec r = load_vrec(job.vrec, v);
    uint32_t t0[kWeightedScan];
    if (kWeighted) load_chunk(job.wthr + r.start, t0);  // padded table: in bounds
    for (uint32_t g = blockIdx.y; g < groups; g += gridDim.y) {
        const uint32_t i0 = g * kPreTrees;
#pragma unroll
        for (uint32_t q = 0; q < kPreTrees; ++q) {
            const uint32_t item = i0 + q;
            if (item < a.item_count)
                a.pre[static_cast<size_t>(item) * a.n_max + v] =
                    kWeighted ? draw_first_w(job, r, t0, a.key0, a.key1, job.tree_begin + item)
                              : draw<false>(job, r, a.key0, a.key1, 0u, job.tree_begin + item);
        }
    }
}

}  // namespace

hipError_t launch_lds_predraw(const CoopArgs &a, hipStream_t stream) {
    if (!a.pre || a.single.n3 == 0 || a.item_count == 0) return hipSuccess;
    // vertex tiles a multiple of 8 wide: block b of every tree group then runs on
    // XCD b mod 8, whose L2 keeps that tile's records and adjacency rows
    uint32_t tiles = (a.single.n3 + kPreThreads - 1) / kPreThreads;
    tiles = (tiles + 7u) & ~7u;
    const uint32_t groups = (a.item_count + kPreTrees - 1) / kPreTrees;
    const dim3 grid(tiles, groups < 65535u ? groups : 65535u);
    if (a.single.wsum) lds_predraw_kernel<true><<<grid, kPreThreads, 0, stream>>>(a, groups);
    else lds_predraw_kernel<false><<<grid, kPreThreads, 0, stream>>>(a, groups);
    return hipGetLastError();
}

namespace {
const void *lds_kernel_of(bool weighted, bool repop, bool lean) {
    if (lean) {
        if (weighted)
            return repop ? reinterpret_cast<const void *>(&wilson_lds_kernel<true, true, true>)
                         : reinterpret_cast<const void *>(&wilson_lds_kernel<true, false, true>);
        return repop ? reinterpret_cast<const void *>(&wilson_lds_kernel<false, true, true>)
                     : reinterpret_cast<const void *>(&wilson_lds_kernel<false, false, true>);
    }
    if (weighted)
        return repop ? reinterpret_cast<const void *>(&wilson_lds_kernel<true, true, false>)
                     : reinterpret_cast<const void *>(&wilson_lds_kernel<true, false, false>);
    return repop ? reinterpret_cast<const void *>(&wilson_lds_kernel<false, true, false>)
                 : reinterpret_cast<const void *>(&wilson_lds_kernel<false, false, false>);
}
}  // namespace

hipError_t lds_set_limit(size_t bytes) {
    for (int m = 0; m < 8; ++m) {
        const hipError_t e = hipFuncSetAttribute(lds_kernel_of(m & 1, m & 2, m & 4),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 static_cast<int>(bytes));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int lds_max_active(uint32_t threads, uint32_t lds_words, bool weighted, bool repop, bool lean) {
    int blocks = 0;
    const void *f = lds_kernel_of(weighted, repop, lean && threads <= 512u);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, static_cast<int>(threads),
                                                     4u * static_cast<size_t>(lds_words)) !=
        hipSuccess)
        return 0;
    return blocks;
}

hipError_t launch_wilson_lds(const CoopArgs &a, uint32_t threads, uint32_t lds_words,
                             bool weighted, bool repop, bool lean, hipStream_t stream) {
    if (a.n_max == 0 || a.item_count == 0 || a.slots == 0) return hipSuccess;
    const size_t lds = 4u * static_cast<size_t>(lds_words);
    const void *f = lds_kernel_of(weighted, repop, lean && threads <= 512u);
    void *args[] = {const_cast<CoopArgs *>(&a)};
    return hipLaunchKernel(f, dim3(a.slots), dim3(threads), args, lds, stream);
}

}  // namespace fc
