// Workgroup-per-tree sampler for graphs whose counters do not all fit in LDS.
//
// Same round-synchronous cycle popping as the other workgroup samplers
// (Wilson's theorem makes the tree and every per-vertex arrow count
// independent of the popping order).  Vertices are relabelled widest degree
// class first (relabel.hip), so the lowest internal ids are the vertices of
// highest degree -- the ones that receive most arrows.  A prefix [0, hot) of
// the ids keeps its in-arrow counter (a field of 4, 8, 16 or 32 bits by degree
// class) and its settled bit in LDS; the remaining ids keep the counter in the
// high half of their global tree word and the settled bit in a global bitmap.
// Isolated vertices (ids [n3, n)) take no part in the rounds.
//
// Memory per tree (slot), n vertices:
//   word[v]   u64 global  internal target | settled << 31 | in-arrow count << 32
//                         (settled flag and count used for ids >= hot only;
//                         for ids >= hot only)
//   origt[v]  u32 global  original id of the target (outputs)
//   kk[v]     u64 global  (epoch << 32) | k_v for redrawn vertices
//   lists     u64 global  (v, internal target) pairs: two unsettled lists and
//                         the peel order; peel level boundaries (u32)
//   LDS                   fields of the ids < hot, then their settled bitmap
#include "fc_kernels.hpp"
#include "fc_wave.hpp"

namespace fc {

namespace {

__device__ __forceinline__ uint32_t lo32(uint64_t w) { return static_cast<uint32_t>(w); }
__device__ __forceinline__ uint32_t hi32(uint64_t w) { return static_cast<uint32_t>(w >> 32); }
__device__ __forceinline__ uint64_t pair(uint32_t v, uint32_t tg) {
    return static_cast<uint64_t>(v) | (static_cast<uint64_t>(tg) << 32);
}

// Per-tree global arrays belong to one workgroup for the whole launch:
// workgroup-scope atomics suffice.
__device__ __forceinline__ uint64_t wg_add(uint64_t *p, uint64_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Items per lane per pass iteration: streaming passes, wide peel levels (each
// item may add a global atomic or load), passes that draw arrows.
constexpr int kR = 8;
constexpr int kRP = 4;
constexpr int kRD = 2;
constexpr uint64_t kCntOne = 1ull << 32;
// settled flag of an id >= hot: bit 31 of its tree word (targets are < 2^31)
constexpr uint32_t kSettled = 1u << 31;
__device__ __forceinline__ uint32_t tgt_of(uint64_t w) { return lo32(w) & ~kSettled; }

enum Phase : int { kPhDraw0 = 0, kPhIndeg, kPhLevel0, kPhPeel, kPhSweep, kPhRedraw, kPhOutput,
                   kPhCount };

// LDS field of hot id x (< hot): classes 32-, 16-, 8-, 4-bit, ending at e3, e2,
// e1 (and n3); the layout covers only ids below hot.
struct Field {
    uint32_t w, sh, mask;
};
struct HotClasses {
    uint32_t e3, e2, e1, o2, o1, o0;
};
// (selects rather than branches: a branch chain over the class bounds is
// turned into an indexed private-memory table by the compiler)
__device__ __forceinline__ Field hot_field(const HotClasses c, uint32_t x) {
    const bool c3 = x < c.e3, c2 = x < c.e2, c1 = x < c.e1;
    const uint32_t start = c3 ? 0u : c2 ? c.e3 : c1 ? c.e2 : c.e1;
    const uint32_t off = c3 ? 0u : c2 ? c.o2 : c1 ? c.o1 : c.o0;
    const uint32_t lg = c3 ? 0u : c2 ? 1u : c1 ? 2u : 3u;  // log2 of the fields per word
    const uint32_t j = x - start;
    Field f;
    f.w = off + (j >> lg);
    f.sh = (j & ((1u << lg) - 1u)) << (5u - lg);  // field width 32 >> lg
    f.mask = lg == 0u ? 0xFFFFFFFFu : (1u << (32u >> lg)) - 1u;
    return f;
}

// Arrow number k of the vertex with (relabelled) record r in tree t:
// internal | original target (u* = n in both).  kWeighted: the job carries
// running weight sums (weighted step).
template <bool kWeighted>
__device__ __forceinline__ uint64_t draw(const CoopJob &j, VRec r, uint32_t key0,
                                         uint32_t key1, uint32_t k, uint32_t t) {
    hold_vrec(r);
    if (r.always_root >> 31) return pair(j.n, j.n);
    const uint32_t orig = r.always_root & 0x7FFFFFFFu;
    const Philox4 x = philox4x32_10(orig, k, t, j.stream_id, key0, key1);
    if (x.x0 < r.thr) return pair(j.n, j.n);
    const uint32_t idx = neighbour_entry<kWeighted>(r, x.x1, j.wsum, j.wthr);
    return j.adj[r.start + static_cast<int32_t>(idx)];
}

template <bool kWeighted>
__global__ __launch_bounds__(1024) void wilson_hyb_kernel(CoopArgs a) {
    extern __shared__ uint32_t s_lds[];
    __shared__ uint32_t s_item, s_u, s_p, s_cycles, s_over, s_nlev;
    __shared__ uint64_t s_tail[64];
    __shared__ unsigned long long s_digest, s_roots;
    __shared__ unsigned long long s_ph[kPhCount + 1];

    const uint32_t T = blockDim.x;
    const uint32_t tid = threadIdx.x;
    const uint32_t wave_base = tid & ~63u;
    const uint32_t lane = tid & 63u;
    const size_t slot = blockIdx.x;
    const size_t stride = a.n_max;
    uint64_t *__restrict__ word = static_cast<uint64_t *>(a.word) + slot * stride;
    uint32_t *__restrict__ origt = a.origt + slot * stride;
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
        const uint32_t n = job.n;     // also the id of u*
        const uint32_t nl = job.n3;   // ids [0, nl) are not isolated
        const uint32_t hot = job.hot; // ids [0, hot) have their counter in LDS
        const HotLayout H = hot_layout(hot, job.n0, job.n1, job.n2);
        const HotClasses C{uniform(job.n0), uniform(job.n1), uniform(job.n2), uniform(H.o2),
                           uniform(H.o1), uniform(H.o0)};
        uint32_t *__restrict__ hbits = s_lds + H.ob;

        // Settled state: an LDS bit for ids < hot, bit 31 of the tree word for
        // the others.  Counts of settled vertices are never read, so a count
        // may change after its vertex settles: the count pass adds to ids >= hot
        // without checking, and a peel decrement learns from the word it gets
        // back whether the vertex had settled (the count field wraps harmlessly
        // above the flag).
        auto hot_settled = [&](uint32_t v) -> bool { return (hbits[v >> 5] >> (v & 31u)) & 1u; };
        auto is_settled = [&](uint32_t v) -> bool {
            if (v >= nl) return true;
            if (v < hot) return hot_settled(v);
            return (lo32(word[v]) & kSettled) != 0u;
        };
        // x (peeled, so its count is 0) settles; tx is its target
        auto settle = [&](uint32_t x, uint32_t tx) {
            if (x < hot) atomicOr(&hbits[x >> 5], 1u << (x & 31u));
            else word[x] = tx | kSettled;
        };
        // an in-arrow into t from an unsettled vertex
        auto count_arrow = [&](uint32_t t) {
            if (t < hot) {
                if (!hot_settled(t)) {
                    const Field f = hot_field(C, t);
                    atomicAdd(&s_lds[f.w], 1u << f.sh);
                }
            } else if (t < nl) {
                (void)wg_add(&word[t], kCntOne);
            }
        };
        // one in-arrow of t removed: when t is unsettled and that was its last,
        // returns the peel entry (t, target of t), else 0 (no entry is 0: t is
        // never its own target)
        auto peel_dec = [&](uint32_t t) -> uint64_t {
            if (t < hot) {
                if (hot_settled(t)) return 0ull;
                const Field f = hot_field(C, t);
                const uint32_t old = (atomicAdd(&s_lds[f.w], 0u - (1u << f.sh)) >> f.sh) & f.mask;
                return old == 1u ? pair(t, tgt_of(word[t])) : 0ull;
            }
            if (t >= nl) return 0ull;
            const uint64_t old = wg_add(&word[t], 0ull - kCntOne);
            return (lo32(old) & kSettled) == 0u && hi32(old) == 1u ? pair(t, tgt_of(old)) : 0ull;
        };
        // whether unsettled v still has an in-arrow (a cycle vertex after the peel)
        // and whether it is settled, from one look at its state
        auto live_count = [&](uint32_t v, bool &live) -> uint32_t {
            if (v < hot) {
                live = !hot_settled(v);
                const Field f = hot_field(C, v);
                return (s_lds[f.w] >> f.sh) & f.mask;
            }
            const uint64_t w = word[v];
            live = (lo32(w) & kSettled) == 0u;
            return hi32(w);
        };

        ++epoch;
        if (tid == 0) {
            s_u = 0;
            s_p = 0;
            s_digest = 0;
            s_roots = 0;
        }
        for (uint32_t i = tid; i < H.words; i += T) s_lds[i] = 0u;
        __syncthreads();

        // round 0: the first arrow of every vertex that is not isolated (records
        // loaded one iteration ahead: one dependent global load per iteration)
        VRec r[kRD] = {};
#pragma unroll
        for (int q = 0; q < kRD; ++q) {
            const uint32_t v = wave_base + q * T + lane;
            if (v < nl) r[q] = load_vrec(job.vrec, v);
        }
        for (uint32_t base = wave_base; base < nl; base += kRD * T) {
            uint64_t w[kRD];
            bool live[kRD];
            VRec rn[kRD] = {};
#pragma unroll
            for (int q = 0; q < kRD; ++q) {
                const uint32_t v = base + (kRD + q) * T + lane;
                if (v < nl) rn[q] = load_vrec(job.vrec, v);
            }
#pragma unroll
            for (int q = 0; q < kRD; ++q) {
                const uint32_t v = base + q * T + lane;
                w[q] = pair(n, n);
                if (v < nl) w[q] = draw<kWeighted>(job, r[q], a.key0, a.key1, 0u, t);
            }
#pragma unroll
            for (int q = 0; q < kRD; ++q) {
                const uint32_t v = base + q * T + lane;
                if (v < nl) {
                    const bool root = lo32(w[q]) == n;
                    word[v] = lo32(w[q]) | (root ? kSettled : 0u);
                    origt[v] = hi32(w[q]);
                    if (root && v < hot) atomicOr(&hbits[v >> 5], 1u << (v & 31u));
                }
                live[q] = v < nl && lo32(w[q]) != n;
                w[q] = pair(v, lo32(w[q]));
            }
            wave_append_many<kRD>(listA, &s_u, n, &s_over, w, live);
#pragma unroll
            for (int q = 0; q < kRD; ++q) r[q] = rn[q];
        }
        __syncthreads();
        mark(kPhDraw0);
        uint32_t ucount = min(uniform(s_u), n);
        uint64_t *U = listA, *Unext = listB;
        unsigned long long draws = n;
        uint32_t rounds = 0;

        while (ucount > 0) {
            if (++rounds > a.max_rounds || draws > job.step_cap || s_over) {
                err |= kErrStepCap;
                break;
            }
            // in-arrows of unsettled targets from unsettled vertices
            for (uint32_t base = tid; base < ucount; base += kR * T) {
                uint32_t tg[kR];
#pragma unroll
                for (int q = 0; q < kR; ++q) {
                    const uint32_t i = base + q * T;
                    tg[q] = i < ucount ? hi32(U[i]) : n;
                }
#pragma unroll
                for (int q = 0; q < kR; ++q)
                    count_arrow(tg[q]);
            }
            if (tid == 0) s_p = 0;
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
                }
#pragma unroll
                for (int q = 0; q < kR; ++q) {
                    const uint32_t i = base + q * T + lane;
                    bool live = false;
                    leaf[q] = i < ucount && live_count(lo32(it[q]), live) == 0u;
                }
                wave_append_many<kR>(peel, &s_p, n, &s_over, it, leaf);
            }
            __syncthreads();
            mark(kPhLevel0);
            uint32_t lo = 0, hi = min(uniform(s_p), n), nlev = 0;
            if (tid == 0) lvl[0] = 0;
            while (hi - lo > 64u) {
                if (tid == 0) lvl[nlev + 1] = hi;
                // (entries loaded one iteration ahead; those appended meanwhile
                // lie beyond hi)
                uint32_t tg[kRP];
#pragma unroll
                for (int q = 0; q < kRP; ++q) {
                    const uint32_t i = lo + wave_base + q * T + lane;
                    tg[q] = i < hi ? hi32(peel[i]) : n;
                }
                for (uint32_t base = lo + wave_base; base < hi; base += kRP * T) {
                    uint32_t tgn[kRP];
                    uint64_t nx[kRP];
                    bool push[kRP];
#pragma unroll
                    for (int q = 0; q < kRP; ++q) {
                        const uint32_t i = base + (kRP + q) * T + lane;
                        tgn[q] = i < hi ? hi32(peel[i]) : n;
                    }
#pragma unroll
                    for (int q = 0; q < kRP; ++q) {
                        nx[q] = peel_dec(tg[q]);
                        push[q] = nx[q] != 0ull;
                    }
                    wave_append_many<kRP>(peel, &s_p, n, &s_over, nx, push);
#pragma unroll
                    for (int q = 0; q < kRP; ++q) tg[q] = tgn[q];
                }
                __syncthreads();
                ++nlev;
                lo = hi;
                hi = min(uniform(s_p), n);
                __syncthreads();
            }
            // narrow tail levels: wave 0 alone (levels never grow)
            const uint32_t tail0 = nlev;
            if (lo < hi) {
                if (wave_base == 0) {
                    uint32_t cnt = hi - lo, pos = hi, nl2 = nlev;
                    uint64_t it = lane < cnt ? peel[lo + lane] : 0ull;
                    while (cnt > 0) {
                        if (lane == 0) lvl[nl2 + 1] = pos;
                        const uint32_t tg = hi32(it);
                        uint64_t nx = 0ull;
                        if (lane < cnt) nx = peel_dec(tg);
                        const bool push = nx != 0ull;
                        const uint64_t mask = __ballot(push);
                        const uint32_t m = static_cast<uint32_t>(__popcll(mask));
                        if (pos + m > n) {
                            if (lane == 0) s_over = 1u;
                            break;
                        }
                        if (push) {
                            const uint32_t r =
                                static_cast<uint32_t>(__popcll(mask & ((1ull << lane) - 1ull)));
                            s_tail[r] = nx;
                            peel[pos + r] = nx;
                        }
                        wave_sync();
                        it = lane < m ? s_tail[lane] : 0ull;
                        wave_sync();
                        pos += m;
                        cnt = m;
                        ++nl2;
                    }
                    if (lane == 0) {
                        s_p = pos;
                        s_nlev = nl2;
                    }
                }
                __syncthreads();
                hi = uniform(s_p);
                nlev = uniform(s_nlev);
            }
            const uint32_t peeled = hi;
            mark(kPhPeel);
            if (peeled == ucount) {
                ucount = 0;
                break;
            }
            // reverse sweep: tail levels by wave 0, then the wide ones
            if (wave_base == 0 && nlev > tail0) {
                for (int32_t top = static_cast<int32_t>(nlev) - 1; top >= static_cast<int32_t>(tail0);
                     top -= 63) {
                    const int32_t li = top + 1 - static_cast<int32_t>(lane);
                    const uint32_t bnd = li >= static_cast<int32_t>(tail0) ? lvl[li] : 0u;
                    const int32_t levels = min(63, top - static_cast<int32_t>(tail0) + 1);
                    for (int32_t j = 0; j < levels; ++j) {
                        const uint32_t a1 = __shfl(bnd, j, 64), a0 = __shfl(bnd, j + 1, 64);
                        if (lane < a1 - a0) {
                            const uint64_t p = peel[a0 + lane];
                            if (is_settled(hi32(p))) settle(lo32(p), hi32(p));
                        }
                        wave_sync();
                    }
                }
            }
            __syncthreads();
            for (int32_t L = static_cast<int32_t>(tail0) - 1; L >= 0; --L) {
                const uint32_t a0 = uniform(lvl[L]), a1 = uniform(lvl[L + 1]);
                for (uint32_t base = a0 + tid; base < a1; base += kR * T) {
                    uint64_t p[kR];
#pragma unroll
                    for (int q = 0; q < kR; ++q) {
                        const uint32_t i = base + q * T;
                        p[q] = i < a1 ? peel[i] : pair(n, n);
                    }
#pragma unroll
                    for (int q = 0; q < kR; ++q)
                        if (lo32(p[q]) < n && is_settled(hi32(p[q]))) settle(lo32(p[q]), hi32(p[q]));
                }
                __syncthreads();
            }
            mark(kPhSweep);
            // split: hanging vertices keep their arrow, cycle vertices (count 1
            // left: the arrow of the cycle predecessor) go to the cycle list
            if (tid == 0) {
                s_u = 0;
                s_cycles = 0;
            }
            __syncthreads();
            uint64_t *__restrict__ cyc = peel;
            for (uint32_t base = wave_base; base < ucount; base += kR * T) {
                uint64_t it[kR];
                bool keep[kR], pop[kR];
#pragma unroll
                for (int q = 0; q < kR; ++q) {
                    const uint32_t i = base + q * T + lane;
                    it[q] = i < ucount ? U[i] : pair(n, n);
                }
#pragma unroll
                for (int q = 0; q < kR; ++q) {
                    const uint32_t v = lo32(it[q]);
                    bool live = false;
                    const uint32_t c = v < nl ? live_count(v, live) : 0u;
                    pop[q] = live && c != 0u;
                    keep[q] = live && !pop[q];
                }
                wave_append_many<kR>(Unext, &s_u, n, &s_over, it, keep);
                wave_append_many<kR>(cyc, &s_cycles, n, &s_over, it, pop);
            }
            __syncthreads();
            // pop every cycle: each cycle vertex draws its next arrow
            const uint32_t ccount = min(uniform(s_cycles), n);
            for (uint32_t base = wave_base; base < ccount; base += kRD * T) {
                uint32_t v[kRD], k[kRD];
                uint64_t w[kRD];
                VRec r[kRD] = {};
#pragma unroll
                for (int q = 0; q < kRD; ++q) {
                    const uint32_t i = base + q * T + lane;
                    v[q] = i < ccount ? lo32(cyc[i]) : n;
                    k[q] = 1u;
                    if (v[q] < n) {
                        // (the record is loaded beside the draw count, not after it)
                        r[q] = load_vrec(job.vrec, v[q]);
                        const uint64_t kv = kk[v[q]];
                        if (hi32(kv) == epoch) k[q] = lo32(kv);
                    }
                }
#pragma unroll
                for (int q = 0; q < kRD; ++q)
                    w[q] = v[q] < n ? draw<kWeighted>(job, r[q], a.key0, a.key1, k[q], t)
                                    : pair(n, n);
#pragma unroll
                for (int q = 0; q < kRD; ++q) {
                    if (v[q] < n) {
                        if (k[q] + 1u > a.k_limit) err |= kErrVisitOverflow;
                        kk[v[q]] = (static_cast<uint64_t>(epoch) << 32) | (k[q] + 1u);
                        if (v[q] < hot) {  // the cycle's arrow into v is gone
                            const Field f = hot_field(C, v[q]);
                            atomicAdd(&s_lds[f.w], 0u - (1u << f.sh));
                        }
                        const bool root = lo32(w[q]) == n;
                        // (a global counter goes back to 0 with it)
                        word[v[q]] = lo32(w[q]) | (root ? kSettled : 0u);
                        origt[v[q]] = hi32(w[q]);
                        if (root && v[q] < hot) atomicOr(&hbits[v[q] >> 5], 1u << (v[q] & 31u));
                    }
                }
                bool live[kRD];
#pragma unroll
                for (int q = 0; q < kRD; ++q) {
                    live[q] = v[q] < n && lo32(w[q]) != n;
                    w[q] = pair(v[q], lo32(w[q]));
                }
                wave_append_many<kRD>(Unext, &s_u, n, &s_over, w, live);
            }
            __syncthreads();
            mark(kPhRedraw);
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
        constexpr int kO = 8;  // vertices whose loads each thread keeps in flight
        for (uint32_t base = tid; base < nl; base += kO * T) {
            uint32_t tgs[kO], ovs[kO], otgs[kO];
#pragma unroll
            for (int q = 0; q < kO; ++q) {
                const uint32_t v = base + q * T;
                tgs[q] = v < nl ? tgt_of(word[v]) : 0u;
                ovs[q] = v < nl ? job.orig[v] : 0u;
                otgs[q] = v < nl ? origt[v] : 0u;
            }
#pragma unroll
            for (int q = 0; q < kO; ++q) {
                const uint32_t v = base + q * T;
                if (v >= nl) continue;
                const uint32_t tg = tgs[q], ov = ovs[q], otg = otgs[q];
                my_digest += mix64((static_cast<unsigned long long>(ov) << 32) | otg);
                if (tg == n) {
                    ++my_roots;
                    atomicAdd(&job.root_counts[ov], 1u);
                }
                if (job.parents)
                    job.parents[static_cast<size_t>(ti) * n + ov] = static_cast<int32_t>(otg);
                if (want_k) {
                    const uint64_t kv = kk[v];
                    const uint32_t k = hi32(kv) == epoch ? lo32(kv) : 1u;
                    if (job.visit_counts)
                        atomicAdd(&job.visit_counts[ov], static_cast<unsigned long long>(k));
                    if (job.tree_visits) job.tree_visits[static_cast<size_t>(ti) * n + ov] = k;
                }
            }
        }
        // isolated vertices: per-tree digest terms; totals once per job
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

}  // namespace

hipError_t hyb_set_limit(size_t bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&wilson_hyb_kernel<false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(bytes));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&wilson_hyb_kernel<true>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

int hyb_max_active(uint32_t threads, uint32_t lds_words, bool weighted) {
    int blocks = 0;
    const void *f = weighted ? reinterpret_cast<const void *>(&wilson_hyb_kernel<true>)
                             : reinterpret_cast<const void *>(&wilson_hyb_kernel<false>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, static_cast<int>(threads),
                                                     4u * static_cast<size_t>(lds_words)) !=
        hipSuccess)
        return 0;
    return blocks;
}

hipError_t launch_wilson_hyb(const CoopArgs &a, uint32_t threads, uint32_t lds_words,
                             hipStream_t stream) {
    if (a.n_max == 0 || a.item_count == 0 || a.slots == 0) return hipSuccess;
    const size_t lds = 4u * static_cast<size_t>(lds_words);
    if (a.single.wsum) wilson_hyb_kernel<true><<<a.slots, threads, lds, stream>>>(a);
    else wilson_hyb_kernel<false><<<a.slots, threads, lds, stream>>>(a);
    return hipGetLastError();
}

}  // namespace fc
