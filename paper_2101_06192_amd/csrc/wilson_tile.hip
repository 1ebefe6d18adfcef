// Workgroup-per-tree sampler for graphs whose vertex ids are local (road
// networks, grids: most edges join ids that are close), by tile-local cycle
// popping.
//
// Wilson's cycle-popping theorem (the tree and every per-vertex arrow count
// are the same whatever order the cycles of the top arrows are popped in)
// lets one workgroup pop a tree's cycles in any grouping.  Here:
//
// 1. Tiles.  The ids are cut into tiles of B consecutive vertices, handled
//    one after another.  A tile's arrows are loaded into LDS as tile-local
//    targets; an arrow to u* or out of the tile ends a path there.  Round
//    after round, the cycles that lie inside the tile are found (in-arrow
//    counts in LDS, Kahn peel, reverse sweep) and popped, until none is
//    left; after the first round only the vertices still unresolved are
//    scanned (they are listed each round).  Every vertex of the tile then
//    has an exit: the last tile vertex on its path (whose arrow leaves the
//    tile), or "settled" when the path reaches u* inside the tile.
// 2. Exit graph.  On the exit vertices the map u -> ex[target(u)] is a
//    functional graph whose cycles are exactly the arrows' cycles that cross
//    tiles.  A Kahn peel over the exits (global counters; only exits take
//    part) and a reverse sweep find which exits reach u*.
// 3. Residual.  A vertex is settled exactly when its exit is.  The few
//    vertices that are not (on a crossing cycle or hanging off one) finish
//    as one more LDS set like a tile (numbered in list order, a target
//    settled before counting as u*) once they fit the tile arrays; until
//    then, with the ordinary round-synchronous popping: a settled bitmap (LDS
//    when it fits), global in-arrow counters and lists, only for them.
// No global atomic touches a vertex outside the exit graph and the residual.
//
// LDS during the tiles:
//   lt[i]  u16  tile-local target of tile vertex i, or kRoot (u*) / kExt (a
//               vertex of another tile)
//   st[i]  u16  resolved: the tile-local id of its exit, or kSettled;
//               unresolved: kUnres | in-arrow count of the current round
//   tp     u16  peel order of the current round
//   lvs    u16  the first kLvLds peel level bounds (the rest in global lv)
// and, once the tiles are done, the exit bitmap and then the settled bitmap,
// when n/8 bytes fit.
// Global, per tree slot:
//   tw[v]  u32  the top arrow's target (u* = n): the tree's own pre-drawn
//               array, or the slot's
//   kk[v]  u64  (epoch << 32) | arrows drawn, written when v draws again
//   ex[v]  u16  tile-local id of v's exit, or kSettled
//   exl    u32  each tile's exit vertices, at offset tile * B; ecnt[tile]
//   pc, sc u32  in-counts (exit graph, residual; zero between uses) and exit
//               successors
//   bl     u32  lists: exits / residual, next residual, peel order (during
//               the tiles: each round's unresolved vertices, two lists)
//   lv     u32  peel level bounds
//   xb          exits whose chain reaches u* (LDS when n/8 bytes fit)
//   bits        settled bitmap of the residual rounds (copied into LDS when it
//               fits)
#include "fc_kernels.hpp"
#include "fc_wave.hpp"

namespace fc {

namespace {

constexpr uint32_t kRoot = 0xFFFFu;     // lt: the arrow goes to u*
constexpr uint32_t kExt = 0xFFFEu;      // lt: the arrow leaves the tile
constexpr uint32_t kUnres = 0x8000u;    // st: unresolved (low 15 bits: in-arrow count)
constexpr uint32_t kSettled = 0x7FFFu;  // st: the path reaches u* inside the tile
constexpr uint32_t kCountMask = 0x7FFFu;
constexpr uint32_t kLvLds = 2048;       // peel level bounds kept in LDS per round

// Per-phase clock sums (tid 0 of each workgroup): tile loads, in-arrow counts
// with peel level 0, peel levels with the reverse sweep, cycle pops, the tiles'
// exits, the exit graph, the residual rounds, the output.
enum Phase : int { kPhLoad = 0, kPhCount, kPhPeel, kPhPop, kPhExits, kPhExit, kPhResidual,
                   kPhOutput, kPhNum };

// One arrow of v in tree t with draw index k (original ids; kWeighted: the
// graph may carry running weight sums).
template <bool kWeighted>
__device__ __forceinline__ uint32_t tile_draw(const TileArgs &a, uint32_t v, uint32_t k,
                                              uint32_t t) {
    VRec r = load_vrec(a.vrec, v);
    hold_vrec(r);
    if (r.always_root) return a.n;
    const Philox4 x = philox4x32_10(v, k, t, a.stream_id, a.key0, a.key1);
    return arrow_target<kWeighted>(r, x.x0, x.x1, a.col_idx, a.wsum, a.wthr, a.n);
}

// Appends `item` to a list whose tail counter is in LDS when `pred` holds (one
// LDS atomic per wave); items at or past `cap` are dropped and reported through
// *over.  The position is relative to `base` (list[base + tail]).  Every lane
// of the wave must reach the call.
template <typename T>
__device__ __forceinline__ void wave_push(T *__restrict__ list, uint32_t base, uint32_t *tail,
                                          uint32_t cap, uint32_t *over, T item, bool pred) {
    const uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    const uint32_t lane = __lane_id();
    const uint32_t cnt = static_cast<uint32_t>(__popcll(mask));
    const uint32_t leader = static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(mask))) - 1u;
    uint32_t off = 0;
    if (lane == leader) {
        off = atomicAdd(tail, cnt);
        if (base + off + cnt > cap) atomicOr(over, 1u);
    }
    off = __shfl(off, static_cast<int>(leader), 64);
    if (pred) {
        const uint32_t at = base + off + static_cast<uint32_t>(__popcll(mask & ((1ull << lane) - 1ull)));
        if (at < cap) list[at] = item;
    }
}

template <bool kWeighted>
__global__ __launch_bounds__(1024) void wilson_tile_kernel(TileArgs a) {
    extern __shared__ uint32_t s_dyn[];
    // s_lc: three rotating tail counters, so that one barrier per peel level
    // suffices (level k appends with counter (k + 1) % 3 while thread 0 clears
    // counter (k + 2) % 3, which everyone read a level ago)
    __shared__ uint32_t s_item, s_u, s_c, s_over, s_rover, s_nlev, s_pos, s_nc, s_lc[3];
    __shared__ uint32_t s_tail[64];
    __shared__ unsigned long long s_digest, s_roots, s_draws;
    __shared__ unsigned long long s_ph[kPhNum + 1];

    const uint32_t T = blockDim.x;
    const uint32_t tid = threadIdx.x;
    const uint32_t wave_base = tid & ~63u;
    const uint32_t lane = tid & 63u;
    const size_t slot = blockIdx.x;
    const uint32_t n = a.n;
    const uint32_t B = a.B;
    const uint32_t Bp = a.Bp;  // B rounded up to a multiple of 64
    const uint32_t ntiles = a.ntiles;
    const size_t nn = n;
    const uint32_t nw = (n + 31u) >> 5;

    uint16_t *__restrict__ lt = reinterpret_cast<uint16_t *>(s_dyn);
    uint32_t *__restrict__ st32 = s_dyn + (Bp >> 1);
    uint16_t *__restrict__ st16 = reinterpret_cast<uint16_t *>(st32);
    uint16_t *__restrict__ tp = reinterpret_cast<uint16_t *>(s_dyn + Bp);
    uint16_t *__restrict__ lvs = reinterpret_cast<uint16_t *>(s_dyn + Bp + (Bp >> 1));
    uint32_t *const gbits = a.bits + slot * static_cast<size_t>(nw);
    uint32_t *__restrict__ bits = a.bits_lds ? s_dyn : gbits;
    uint32_t *__restrict__ xb = a.xb ? a.xb + slot * static_cast<size_t>(nw) : s_dyn;

    uint32_t *const slot_tw = a.tw ? a.tw + slot * nn : nullptr;
    uint64_t *__restrict__ kk = a.kk + slot * nn;
    uint16_t *__restrict__ ex = a.ex + slot * nn;
    uint32_t *__restrict__ exl = a.exl + slot * nn;
    uint32_t *__restrict__ ecnt = a.ecnt + slot * static_cast<size_t>(ntiles);
    uint32_t *__restrict__ pc = a.pc + slot * nn;
    uint32_t *__restrict__ sc = a.sc + slot * nn;
    uint32_t *__restrict__ bU = a.bl + slot * (3ull * nn);
    uint32_t *__restrict__ bN = bU + nn;
    uint32_t *__restrict__ bP = bN + nn;
    uint32_t *__restrict__ lvg = a.lv + slot * (nn + 2u);

    unsigned int err = 0;
    uint32_t epoch = 0;  // per-slot tree sequence number of this launch (kk is zeroed per launch)
    const bool timing = a.phase_ticks != nullptr;
    if (tid == 0) {
        s_over = 0;
        s_lc[0] = s_lc[1] = s_lc[2] = 0;
    }
    if (timing && tid == 0) {
        for (int i = 0; i < kPhNum; ++i) s_ph[i] = 0;
        s_ph[kPhNum] = wall_clock64();
    }
    auto mark = [&](int which) {
        if (timing && tid == 0) {
            const unsigned long long now = wall_clock64();
            s_ph[which] += now - s_ph[kPhNum];
            s_ph[kPhNum] = now;
        }
    };
    auto st_get = [&](uint32_t i) -> uint32_t { return (st32[i >> 1] >> ((i & 1u) << 4)) & 0xFFFFu; };
    auto st_inc = [&](uint32_t i) { atomicAdd(&st32[i >> 1], 1u << ((i & 1u) << 4)); };
    // decrement an unresolved count (>= 1); returns the field before
    auto st_dec = [&](uint32_t i) -> uint32_t {
        const uint32_t sh = (i & 1u) << 4;
        return (atomicAdd(&st32[i >> 1], 0u - (1u << sh)) >> sh) & 0xFFFFu;
    };
    // tile peel level bounds: LDS first, global beyond
    auto lv_set = [&](uint32_t i, uint32_t v) {
        if (i < kLvLds) lvs[i] = static_cast<uint16_t>(v);
        else lvg[i] = v;
    };
    auto lv_get = [&](uint32_t i) -> uint32_t { return i < kLvLds ? lvs[i] : lvg[i]; };
    auto is_settled = [&](uint32_t v) -> bool {
        return v >= n || ((bits[v >> 5] >> (v & 31u)) & 1u);
    };
    auto set_settled = [&](uint32_t v) { atomicOr(&bits[v >> 5], 1u << (v & 31u)); };

    for (;;) {
        __syncthreads();
        if (tid == 0) s_item = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t item = uniform(s_item);
        if (item >= a.tree_count) break;
        const uint32_t t = a.tree_begin + item;
        uint32_t *__restrict__ tw = a.pre ? a.pre + static_cast<size_t>(item) * nn : slot_tw;
        ++epoch;
        if (tid == 0) {
            s_digest = 0;
            s_roots = 0;
            s_draws = n;
        }
        // first arrows, when no pre-draw kernel drew them
        if (!a.pre) {
            for (uint32_t v = tid; v < n; v += T) tw[v] = tile_draw<kWeighted>(a, v, 0u, t);
        }
        auto pop = [&](uint32_t v) -> uint32_t {  // v draws its next arrow
            const uint64_t kv = kk[v];
            const uint32_t k = static_cast<uint32_t>(kv >> 32) == epoch ? static_cast<uint32_t>(kv) : 1u;
            if (k + 1u > a.k_limit) err |= kErrVisitOverflow;
            const uint32_t tg = tile_draw<kWeighted>(a, v, k, t);
            kk[v] = (static_cast<uint64_t>(epoch) << 32) | (k + 1u);
            tw[v] = tg;
            return tg;
        };

        // Cycle popping inside a vertex set held in LDS (a tile, or the
        // residual): set vertex i is global id vid(i); an arrow's target becomes
        // a set-local code: kRoot when it reaches u* (u* itself, or a vertex
        // settled before), kExt for a vertex of another tile, else its local id.
        // Rounds until every vertex of the set is resolved (settled, or its
        // exit known).
        // (the residual set: its id list and a list buffer apart from it and bP)
        uint32_t *res_list = bU, *res_l0 = bN;
        auto pop_rounds = [&](uint32_t b, uint32_t lo, bool res, int ph_count, int ph_peel,
                              int ph_pop) {
            auto vid = [&](uint32_t i) -> uint32_t { return res ? res_list[i] : lo + i; };
            auto code_of = [&](uint32_t tg) -> uint32_t {
                if (tg == n) return kRoot;
                if (res) return ((gbits[tg >> 5] >> (tg & 31u)) & 1u) ? kRoot : sc[tg];
                return tg - lo < b ? tg - lo : kExt;
            };
            // After the first round (which scans the whole set) only the vertices
            // left hanging off a cycle by the sweep and the cycle vertices
            // themselves can be unresolved: each round lists them (global, per
            // slot, in lists the tiles do not use otherwise), and later rounds
            // scan that list instead of the set.
            uint32_t *Lcur = res ? res_l0 : bN + lo;
            uint32_t *Lnext = res ? bP : bP + lo;
            uint32_t lcount = 0;
            bool full = true;
            uint32_t rounds = 0;
            for (;;) {
                if (++rounds > a.max_rounds || s_over) {
                    err |= kErrStepCap;
                    break;
                }
                // in-arrows between unresolved vertices (every unresolved vertex
                // has an internal target and a zero count here); count them
                if (tid == 0) {
                    s_u = 0;
                    s_c = 0;
                    s_nc = 0;
                    s_lc[0] = 0;
                    s_lc[1] = 0;
                }
                __syncthreads();
                const uint32_t scan = full ? b : lcount;  // candidates: the set, or the list
                uint32_t mine = 0;
                for (uint32_t j = tid; j < scan; j += T) {
                    const uint32_t i = full ? j : Lcur[j];
                    if (st_get(i) & kUnres) {
                        ++mine;
                        const uint32_t tg = lt[i];
                        if (st_get(tg) & kUnres) st_inc(tg);
                    }
                }
                wave_count(&s_u, mine);
                __syncthreads();
                const uint32_t ucount = uniform(s_u);
                if (ucount == 0) break;  // every vertex of the set resolved
                // peel level 0: unresolved with no in-arrow (level k appends
                // with counter (k + 1) % 3)
                for (uint32_t j = wave_base; j < scan; j += T) {
                    const uint32_t lj = j + lane;
                    uint32_t li = 0;
                    bool leaf = false;
                    if (lj < scan) {
                        li = full ? lj : Lcur[lj];
                        leaf = st_get(li) == kUnres;
                    }
                    wave_push<uint16_t>(tp, 0u, &s_lc[0], Bp, &s_over, static_cast<uint16_t>(li), leaf);
                }
                __syncthreads();
                mark(ph_count);
                uint32_t plo = 0, phi = min(uniform(s_lc[0]), b), nlev = 0;
                if (tid == 0) lv_set(0, 0);
                while (phi - plo > 64u) {
                    const uint32_t cn = (nlev + 1u) % 3u, cz = (nlev + 2u) % 3u;
                    if (tid == 0) {
                        lv_set(nlev + 1, phi);
                        s_lc[cz] = 0;
                    }
                    for (uint32_t i = plo + wave_base; i < phi; i += T) {
                        const uint32_t li = i + lane;
                        uint32_t tg = 0;
                        bool push = false;
                        if (li < phi) {
                            tg = lt[tp[li]];
                            if (st_get(tg) & kUnres) push = (st_dec(tg) & kCountMask) == 1u;
                        }
                        wave_push<uint16_t>(tp, phi, &s_lc[cn], Bp, &s_over, static_cast<uint16_t>(tg), push);
                    }
                    __syncthreads();
                    ++nlev;
                    plo = phi;
                    phi = min(phi + uniform(s_lc[cn]), b);
                }
                const uint32_t tail0 = nlev;
                if (plo < phi) {  // narrow levels: wave 0 alone, frontier in registers
                    if (wave_base == 0) {
                        uint32_t cnt = phi - plo, pos = phi, nl = nlev;
                        uint32_t x = lane < cnt ? tp[plo + lane] : 0u;
                        while (cnt > 0) {
                            if (lane == 0) lv_set(nl + 1, pos);
                            bool push = false;
                            uint32_t tg = 0;
                            if (lane < cnt) {
                                tg = lt[x];
                                if (st_get(tg) & kUnres) push = (st_dec(tg) & kCountMask) == 1u;
                            }
                            const uint64_t mask = __ballot(push);
                            const uint32_t m = static_cast<uint32_t>(__popcll(mask));
                            if (pos + m > b) {
                                if (lane == 0) s_over = 1u;
                                break;
                            }
                            if (push) {
                                const uint32_t r = static_cast<uint32_t>(
                                    __popcll(mask & ((1ull << lane) - 1ull)));
                                s_tail[r] = tg;
                                tp[pos + r] = static_cast<uint16_t>(tg);
                            }
                            wave_sync();
                            x = lane < m ? s_tail[lane] : 0u;
                            wave_sync();
                            pos += m;
                            cnt = m;
                            ++nl;
                        }
                        if (lane == 0) {
                            s_pos = pos;
                            s_nlev = nl;
                        }
                    }
                    __syncthreads();
                    phi = min(uniform(s_pos), b);
                    nlev = uniform(s_nlev);
                }
                const uint32_t peeled = phi;
                // reverse sweep: a peeled vertex takes its target's exit when the
                // target is resolved; otherwise it hangs off a cycle and stays
                // unresolved (count 0) for the next round
                if (wave_base == 0 && nlev > tail0) {
                    for (uint32_t L = nlev; L > tail0; --L) {
                        const uint32_t a0 = lv_get(L - 1), a1 = L == nlev ? peeled : lv_get(L);
                        if (lane < a1 - a0) {
                            const uint32_t x = tp[a0 + lane];
                            const uint32_t s = st_get(lt[x]);
                            if (!(s & kUnres)) st16[x] = static_cast<uint16_t>(s);
                        }
                        wave_sync();
                    }
                }
                __syncthreads();
                for (uint32_t L = tail0; L > 0; --L) {
                    const uint32_t a0 = lv_get(L - 1), a1 = lv_get(L);
                    for (uint32_t i = a0 + tid; i < a1; i += T) {
                        const uint32_t x = tp[i];
                        const uint32_t s = st_get(lt[x]);
                        if (!(s & kUnres)) st16[x] = static_cast<uint16_t>(s);
                    }
                    __syncthreads();
                }
                mark(ph_peel);
                if (peeled == ucount) break;  // no cycle: every unresolved vertex resolved
                // pop the set's cycles: unresolved vertices with an in-arrow left
                // (exactly one, from the cycle) draw their next arrow.  They are
                // listed first (the peel order is spent), so that the draws'
                // global loads go out together.
                // The same scan lists every vertex still unresolved (hanging off a
                // cycle, or on one) for the next round: no other can be then.
                // When every thread scans at most one entry, a cycle vertex is
                // popped right there (the cycles are disjoint: popping them all at
                // once is popping them one after another), saving a barrier and
                // overlapping the draws with the scan.
                const uint32_t half = Bp >> 1;
                const bool inline_pop = scan <= T && scan <= half;
                if (tid == 0) s_lc[0] = 0;  // the first re-pop pass's tail (the peel's counters are spent)
                for (uint32_t j = wave_base; j < scan; j += T) {
                    const uint32_t lj = j + lane;
                    uint32_t li = 0;
                    bool cyc = false, unres = false;
                    if (lj < scan) {
                        li = full ? lj : Lcur[lj];
                        const uint32_t s = st_get(li);
                        unres = (s & kUnres) != 0u;
                        cyc = unres && (s & kCountMask);
                    }
                    wave_push<uint16_t>(tp, 0u, &s_c, Bp, &s_over, static_cast<uint16_t>(li), cyc);
                    wave_push<uint32_t>(Lnext, 0u, &s_nc, b, &s_over, li, unres);
                    if (inline_pop && cyc) {  // (npop <= half here: the re-pops run when enabled)
                        const uint32_t tg = pop(vid(li));
                        const uint32_t code = code_of(tg);
                        lt[li] = static_cast<uint16_t>(code);
                        st16[li] = static_cast<uint16_t>(code == kRoot ? kSettled
                                                         : code == kExt ? li
                                                         : a.repop ? kUnres | 1u : kUnres);
                    }
                }
                __syncthreads();
                const uint32_t npop = min(uniform(s_c), b);
                const uint32_t next_count = min(uniform(s_nc), b);
                // with the re-pops, vertices redrawn to an unresolved target carry
                // the mark "redrawn in this pass" (count 1) into the first pass
                const bool repop = a.repop && npop <= half;
                const uint32_t fresh = repop ? kUnres | 1u : kUnres;
                if (!inline_pop) {
                    for (uint32_t j = tid; j < npop; j += T) {
                        const uint32_t i = tp[j];
                        const uint32_t tg = pop(vid(i));
                        const uint32_t code = code_of(tg);
                        lt[i] = static_cast<uint16_t>(code);
                        st16[i] = static_cast<uint16_t>(code == kRoot ? kSettled : code == kExt ? i : fresh);
                    }
                    __syncthreads();
                }
                if (tid == 0) s_draws += npop;
                // Re-formed 2-cycles: a redrawn vertex u whose new arrow goes to an
                // unresolved t whose arrow comes back to u closes a cycle of the
                // current arrows, popped at once (any cycle may be popped at any
                // time) instead of a round later.  The pair is popped by u's lane,
                // or by the smaller id's when both were redrawn in this pass
                // (both marked).  Passes alternate between the halves of the peel
                // list; one that would overflow its half pops nothing and ends them.
                if (repop) {
                    uint32_t cur = 0, ncur = npop;
                    for (uint32_t pass = 0; ncur > 0; ++pass) {
                        const uint32_t nxt = cur ? 0u : half;
                        const uint32_t cp = pass % 2u;  // tail counter of this pass
                        if (tid == 0) s_lc[cp ^ 1u] = 0;
                        for (uint32_t j = wave_base; j < ncur; j += T) {
                            const uint32_t lj = j + lane;
                            uint32_t u = 0, tg = 0;
                            bool lead = false;
                            if (lj < ncur && pass < 32u) {
                                u = tp[cur + lj];
                                if (st_get(u) & kUnres) {
                                    tg = lt[u];
                                    if (tg < b) {
                                        const uint32_t sv = st_get(tg);
                                        lead = (sv & kUnres) && lt[tg] == u &&
                                               ((sv & kCountMask) == 0u || u < tg);
                                    }
                                }
                            }
                            wave_push<uint16_t>(tp, nxt, &s_lc[cp], nxt + half, &s_rover,
                                                static_cast<uint16_t>(u), lead);
                            wave_push<uint16_t>(tp, nxt, &s_lc[cp], nxt + half, &s_rover,
                                                static_cast<uint16_t>(tg), lead);
                        }
                        __syncthreads();
                        for (uint32_t j = tid; j < ncur; j += T) {  // clear the marks
                            const uint32_t u = tp[cur + j];
                            if (st_get(u) == (kUnres | 1u)) st16[u] = static_cast<uint16_t>(kUnres);
                        }
                        const uint32_t nn = uniform(s_lc[cp]);
                        __syncthreads();
                        // no pair, or the half overflowed (then nothing is popped: the next
                        // round finds those cycles)
                        if (nn == 0u || nn > half) break;
                        for (uint32_t j = tid; j < nn; j += T) {
                            const uint32_t i = tp[nxt + j];
                            const uint32_t tg = pop(vid(i));
                            const uint32_t code = code_of(tg);
                            lt[i] = static_cast<uint16_t>(code);
                            st16[i] = static_cast<uint16_t>(code == kRoot ? kSettled
                                                            : code == kExt ? i : kUnres | 1u);
                        }
                        __syncthreads();
                        if (tid == 0) s_draws += nn;
                        cur = nxt;
                        ncur = nn;
                    }
                }
                mark(ph_pop);
                uint32_t *const spent = Lcur;
                Lcur = Lnext;
                Lnext = spent;
                lcount = next_count;
                full = false;
            }
        };

        // -------------------------------------------------------------------
        // 1. tiles: their own cycles, then every vertex's exit
        // -------------------------------------------------------------------
        for (uint32_t tile = 0; tile < ntiles && !(err & kErrStepCap); ++tile) {
            const uint32_t lo = tile * B;
            const uint32_t b = min(B, n - lo);
            __syncthreads();
            {
                constexpr int kL = 8;  // loads in flight per thread
                for (uint32_t i0 = tid; i0 < b; i0 += kL * T) {
                    uint32_t tg[kL];
#pragma unroll
                    for (int q = 0; q < kL; ++q) {
                        const uint32_t i = i0 + q * T;
                        tg[q] = i < b ? tw[lo + i] : n;
                    }
#pragma unroll
                    for (int q = 0; q < kL; ++q) {
                        const uint32_t i = i0 + q * T;
                        if (i < b) {
                            const uint32_t code = tg[q] == n ? kRoot : (tg[q] - lo < b ? tg[q] - lo : kExt);
                            lt[i] = static_cast<uint16_t>(code);
                            st16[i] = static_cast<uint16_t>(code == kRoot ? kSettled
                                                            : code == kExt ? i : kUnres);
                        }
                    }
                }
            }
            mark(kPhLoad);
            pop_rounds(b, lo, false, kPhCount, kPhPeel, kPhPop);
            if (err & kErrStepCap) break;
            // every vertex's exit, and the tile's exit list
            if (tid == 0) s_c = 0;
            __syncthreads();
            for (uint32_t i = wave_base; i < b; i += T) {
                const uint32_t li = i + lane;
                bool isx = false;
                if (li < b) {
                    ex[lo + li] = static_cast<uint16_t>(st_get(li));
                    isx = lt[li] == kExt;
                }
                wave_push<uint32_t>(exl, lo, &s_c, lo + b, &s_over, lo + li, isx);
            }
            __syncthreads();
            if (tid == 0) ecnt[tile] = min(s_c, b);
            mark(kPhExits);
        }
        __syncthreads();
        if (err & kErrStepCap) break;

        // -------------------------------------------------------------------
        // 2. the exit graph: u -> ex[target(u)] over the exit vertices
        // -------------------------------------------------------------------
        if (tid == 0) {
            s_u = 0;
            s_lc[0] = s_lc[1] = s_lc[2] = 0;
        }
        for (uint32_t i = tid; i < nw; i += T) xb[i] = 0u;
        __syncthreads();
        for (uint32_t tile = wave_base >> 6; tile < ntiles; tile += T >> 6) {
            const uint32_t c = ecnt[tile];
            const uint32_t *seg = exl + static_cast<size_t>(tile) * B;
            for (uint32_t i = 0; i < c; i += 64) {
                const bool ok = i + lane < c;
                wave_push<uint32_t>(bU, 0u, &s_u, n, &s_over, ok ? seg[i + lane] : 0u, ok);
            }
        }
        __syncthreads();
        const uint32_t m = min(uniform(s_u), n);
        bool residual = false;
        if (m > 0) {
            for (uint32_t i = tid; i < m; i += T) {
                const uint32_t u = bU[i];
                const uint32_t x = tw[u];
                const uint32_t e = ex[x];
                const uint32_t s = e == kSettled ? n : x - x % B + e;
                sc[u] = s;
                if (s < n) atomicAdd(&pc[s], 1u);
            }
            __syncthreads();
            for (uint32_t i = wave_base; i < m; i += T) {
                const uint32_t li = i + lane;
                uint32_t u = 0;
                bool leaf = false;
                if (li < m) {
                    u = bU[li];
                    leaf = pc[u] == 0u;
                }
                wave_push<uint32_t>(bP, 0u, &s_lc[0], n, &s_over, u, leaf);
            }
            __syncthreads();
            uint32_t plo = 0, phi = min(uniform(s_lc[0]), n), nlev = 0;
            if (tid == 0) lvg[0] = 0;
            while (phi > plo) {
                const uint32_t cn = (nlev + 1u) % 3u, cz = (nlev + 2u) % 3u;
                if (tid == 0) {
                    lvg[nlev + 1] = phi;
                    s_lc[cz] = 0;
                }
                for (uint32_t i = plo + wave_base; i < phi; i += T) {
                    const uint32_t li = i + lane;
                    uint32_t s = 0;
                    bool push = false;
                    if (li < phi) {
                        s = sc[bP[li]];
                        if (s < n) push = atomicSub(&pc[s], 1u) == 1u;
                    }
                    wave_push<uint32_t>(bP, phi, &s_lc[cn], n, &s_over, s, push);
                }
                __syncthreads();
                ++nlev;
                plo = phi;
                phi = min(phi + uniform(s_lc[cn]), n);
            }
            // reverse sweep: an exit reaches u* when its successor does (bit in xb)
            for (uint32_t L = nlev; L > 0; --L) {
                const uint32_t a0 = lvg[L - 1], a1 = lvg[L];
                for (uint32_t i = a0 + tid; i < a1; i += T) {
                    const uint32_t u = bP[i];
                    const uint32_t s = sc[u];
                    if (s >= n || ((xb[s >> 5] >> (s & 31u)) & 1u)) atomicOr(&xb[u >> 5], 1u << (u & 31u));
                }
                __syncthreads();
            }
            residual = plo < m;  // exits left unpeeled lie on crossing cycles
        }
        mark(kPhExit);

        // -------------------------------------------------------------------
        // 3. the residual: vertices whose exit does not reach u*
        // -------------------------------------------------------------------
        if (residual) {
            if (tid == 0) s_u = 0;
            // exits on crossing cycles keep one in-arrow count: clear it
            for (uint32_t i = tid; i < m; i += T) pc[bU[i]] = 0u;
            __syncthreads();
            // settled bitmap (global first) and the residual list: v is settled iff
            // its path reaches u* inside its tile or its exit's chain does
            {
                constexpr int kS = 4;  // vertices per lane in flight
                for (uint32_t base0 = wave_base; base0 < n; base0 += kS * T) {
                    uint32_t e[kS];
#pragma unroll
                    for (int q = 0; q < kS; ++q) {
                        const uint32_t v = base0 + q * T + lane;
                        e[q] = v < n ? ex[v] : kSettled;
                    }
#pragma unroll
                    for (int q = 0; q < kS; ++q) {
                        const uint32_t base = base0 + q * T;
                        const uint32_t v = base + lane;
                        bool done = true;
                        if (v < n && e[q] != kSettled) {
                            const uint32_t x = v - v % B + e[q];
                            done = (xb[x >> 5] >> (x & 31u)) & 1u;
                        }
                        const uint64_t mask = __ballot(done);
                        if (base < n) {
                            if (lane == 0) gbits[base >> 5] = static_cast<uint32_t>(mask);
                            if (lane == 32 && (base >> 5) + 1u < nw)
                                gbits[(base >> 5) + 1u] = static_cast<uint32_t>(mask >> 32);
                        }
                        wave_push<uint32_t>(bU, 0u, &s_u, n, &s_over, v, !done);
                    }
                }
            }
            __syncthreads();
            uint32_t ucount = min(uniform(s_u), n);
            if (ucount > B && a.bits_lds) {  // the global rounds test the bitmap in LDS
                for (uint32_t i = tid; i < nw; i += T) s_dyn[i] = gbits[i];
                __syncthreads();
            }
            uint32_t *U = bU, *Un = bN;
            uint32_t rounds = 0;
            while (ucount > 0) {
                if (ucount <= B) {
                    // What is left fits the tiles' LDS arrays: pop it as one more
                    // set, its vertices numbered in list order (sc, spent since the
                    // exit graph, maps an id to that number); targets settled
                    // before count as u*.
                    if (rounds > 0 && a.bits_lds) {  // the settled bitmap back to global
                        for (uint32_t i = tid; i < nw; i += T) gbits[i] = s_dyn[i];
                        __syncthreads();
                    }
                    for (uint32_t i = tid; i < ucount; i += T) sc[U[i]] = i;
                    __syncthreads();
                    for (uint32_t i = tid; i < ucount; i += T) {
                        const uint32_t tg = tw[U[i]];
                        const uint32_t code =
                            tg == n || ((gbits[tg >> 5] >> (tg & 31u)) & 1u) ? kRoot : sc[tg];
                        lt[i] = static_cast<uint16_t>(code);
                        st16[i] = static_cast<uint16_t>(code == kRoot ? kSettled : kUnres);
                    }
                    res_list = U;
                    res_l0 = U == bU ? bN : bU;
                    pop_rounds(ucount, 0u, true, kPhResidual, kPhResidual, kPhResidual);
                    break;
                }
                if (++rounds > a.max_rounds || s_over) {
                    err |= kErrStepCap;
                    break;
                }
                if (tid == 0) {
                    s_lc[0] = s_lc[1] = s_lc[2] = 0;
                    s_c = 0;
                }
                for (uint32_t i = tid; i < ucount; i += T) {
                    const uint32_t tg = tw[U[i]];
                    if (!is_settled(tg)) atomicAdd(&pc[tg], 1u);
                }
                __syncthreads();
                for (uint32_t i = wave_base; i < ucount; i += T) {
                    const uint32_t li = i + lane;
                    uint32_t x = 0;
                    bool leaf = false;
                    if (li < ucount) {
                        x = U[li];
                        leaf = pc[x] == 0u;
                    }
                    wave_push<uint32_t>(bP, 0u, &s_lc[0], n, &s_over, x, leaf);
                }
                __syncthreads();
                uint32_t plo = 0, phi = min(uniform(s_lc[0]), n), nlev = 0;
                if (tid == 0) lvg[0] = 0;
                while (phi > plo) {
                    const uint32_t cn = (nlev + 1u) % 3u, cz = (nlev + 2u) % 3u;
                    if (tid == 0) {
                        lvg[nlev + 1] = phi;
                        s_lc[cz] = 0;
                    }
                    for (uint32_t i = plo + wave_base; i < phi; i += T) {
                        const uint32_t li = i + lane;
                        uint32_t tg = 0;
                        bool push = false;
                        if (li < phi) {
                            tg = tw[bP[li]];
                            if (!is_settled(tg)) push = atomicSub(&pc[tg], 1u) == 1u;
                        }
                        wave_push<uint32_t>(bP, phi, &s_lc[cn], n, &s_over, tg, push);
                    }
                    __syncthreads();
                    ++nlev;
                    plo = phi;
                    phi = min(phi + uniform(s_lc[cn]), n);
                }
                const uint32_t peeled = phi;
                if (tid == 0) s_u = 0;  // every thread read it before the level-0 barrier
                // reverse sweep: settled when the target is; the others hang off a
                // cycle and stay listed
                for (uint32_t L = nlev; L > 0; --L) {
                    const uint32_t a0 = lvg[L - 1], a1 = lvg[L];
                    for (uint32_t i = a0 + wave_base; i < a1; i += T) {
                        const uint32_t li = i + lane;
                        uint32_t x = 0;
                        bool hang = false;
                        if (li < a1) {
                            x = bP[li];
                            if (is_settled(tw[x])) set_settled(x);
                            else hang = true;
                        }
                        wave_push<uint32_t>(Un, 0u, &s_u, n, &s_over, x, hang);
                    }
                    __syncthreads();
                }
                if (peeled == ucount) break;  // no cycle left
                // pop the cycles: listed vertices never peeled (one in-arrow left)
                uint32_t pops = 0;
                for (uint32_t i = wave_base; i < ucount; i += T) {
                    const uint32_t li = i + lane;
                    uint32_t x = 0;
                    bool live = false;
                    if (li < ucount) {
                        x = U[li];
                        if (!is_settled(x) && pc[x] != 0u) {
                            pc[x] = 0u;
                            const uint32_t tg = pop(x);
                            if (tg == n) set_settled(x);
                            else live = true;
                            ++pops;
                        }
                    }
                    wave_push<uint32_t>(Un, 0u, &s_u, n, &s_over, x, live);
                }
                wave_count(&s_c, pops);
                __syncthreads();
                if (tid == 0) s_draws += s_c;
                ucount = min(uniform(s_u), n);
                uint32_t *tmp = U;
                U = Un;
                Un = tmp;
            }
            __syncthreads();
            if (err & kErrStepCap) break;
        }
        mark(kPhResidual);
        {
            const unsigned long long drawn = s_draws;  // final since the last barrier
            if (drawn > a.step_cap) {
                err |= kErrStepCap;
                break;
            }
        }

        // the tree: top arrows; R, digest, optional per-tree dumps
        unsigned long long my_digest = 0, my_roots = 0;
        const bool want_k = a.visit_counts || a.tree_visits;
        constexpr int kO = 16;  // targets whose loads each thread keeps in flight
        for (uint32_t base = tid; base < n; base += kO * T) {
            uint32_t tgs[kO];
#pragma unroll
            for (int q = 0; q < kO; ++q) {
                const uint32_t v = base + q * T;
                tgs[q] = v < n ? tw[v] : 0u;
            }
#pragma unroll
            for (int q = 0; q < kO; ++q) {
                const uint32_t v = base + q * T;
                if (v >= n) continue;
                const uint32_t tg = tgs[q];
                my_digest += mix64((static_cast<unsigned long long>(v) << 32) | tg);
                if (tg == n) {
                    ++my_roots;
                    atomicAdd(&a.root_counts[v], 1u);
                }
                if (a.parents) a.parents[static_cast<size_t>(item) * nn + v] = static_cast<int32_t>(tg);
                if (want_k) {
                    const uint64_t kv = kk[v];
                    const uint32_t k =
                        static_cast<uint32_t>(kv >> 32) == epoch ? static_cast<uint32_t>(kv) : 1u;
                    if (a.visit_counts) atomicAdd(&a.visit_counts[v], static_cast<unsigned long long>(k));
                    if (a.tree_visits) a.tree_visits[static_cast<size_t>(item) * nn + v] = k;
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
            if (a.tree_digests) a.tree_digests[item] = s_digest;
            if (a.tree_steps) a.tree_steps[item] = s_draws;
            atomicAdd(&a.totals->walk_steps, s_draws);
            atomicAdd(&a.totals->roots, s_roots);
            atomicAdd(&a.totals->digest_sum, s_digest);
        }
        mark(kPhOutput);
    }
    if (timing && tid == 0)
        for (int i = 0; i < kPhNum; ++i) atomicAdd(&a.phase_ticks[i], s_ph[i]);
    if (s_over) err |= kErrStepCap;
    if (err) atomicOr(&a.totals->error, err);
}

// Trees per workgroup of the pre-draw kernel (each thread owns one vertex and
// draws its first arrow in that many trees).
constexpr uint32_t kPreTrees = 16;
constexpr uint32_t kPreThreads = 256;

template <bool kWeighted>
__global__ __launch_bounds__(kPreThreads) void tile_predraw_kernel(TileArgs a, uint32_t groups) {
    const uint32_t v = blockIdx.x * kPreThreads + threadIdx.x;
    if (v >= a.n) return;
    const VRec r = load_vrec(a.vrec, v);
    for (uint32_t g = blockIdx.y; g < groups; g += gridDim.y) {
        const uint32_t i0 = g * kPreTrees;
#pragma unroll 4
        for (uint32_t q = 0; q < kPreTrees; ++q) {
            const uint32_t item = i0 + q;
            if (item >= a.tree_count) break;
            uint32_t tg = a.n;
            if (!r.always_root) {
                const Philox4 x = philox4x32_10(v, 0u, a.tree_begin + item, a.stream_id, a.key0, a.key1);
                tg = arrow_target<kWeighted>(r, x.x0, x.x1, a.col_idx, a.wsum, a.wthr, a.n);
            }
            a.pre[static_cast<size_t>(item) * a.n + v] = tg;
        }
    }
}

// Entries of the CSR whose two ends lie in different tiles of B ids (one
// atomic per block).
__global__ __launch_bounds__(256) void count_cross_kernel(const int32_t *__restrict__ row_ptr,
                                                          const int32_t *__restrict__ col_idx,
                                                          uint32_t n, uint32_t B,
                                                          unsigned long long *out) {
    __shared__ unsigned long long s_sum;
    if (threadIdx.x == 0) s_sum = 0;
    __syncthreads();
    unsigned long long c = 0;
    for (uint32_t v = blockIdx.x * 256u + threadIdx.x; v < n; v += gridDim.x * 256u) {
        const uint32_t tv = v / B;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
            c += static_cast<uint32_t>(col_idx[e]) / B != tv ? 1u : 0u;
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
    if ((threadIdx.x & 63u) == 0) atomicAdd(&s_sum, c);
    __syncthreads();
    if (threadIdx.x == 0 && s_sum) atomicAdd(out, s_sum);
}

}  // namespace

hipError_t launch_count_cross(const int32_t *row_ptr, const int32_t *col_idx, uint32_t n,
                              uint32_t B, unsigned long long *out, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    uint32_t blocks = (n + 255u) / 256u;
    blocks = blocks < 4096u ? blocks : 4096u;
    count_cross_kernel<<<blocks, 256, 0, stream>>>(row_ptr, col_idx, n, B, out);
    return hipGetLastError();
}

hipError_t launch_tile_predraw(const TileArgs &a, hipStream_t stream) {
    if (!a.pre || a.n == 0 || a.tree_count == 0) return hipSuccess;
    // vertex tiles a multiple of 8 wide: block b of every tree group then runs on
    // XCD b mod 8, whose L2 keeps that tile's records and adjacency rows
    uint32_t tiles = (a.n + kPreThreads - 1) / kPreThreads;
    tiles = (tiles + 7u) & ~7u;
    const uint32_t groups = (a.tree_count + kPreTrees - 1) / kPreTrees;
    const dim3 grid(tiles, groups < 65535u ? groups : 65535u);
    if (a.wsum) tile_predraw_kernel<true><<<grid, kPreThreads, 0, stream>>>(a, groups);
    else tile_predraw_kernel<false><<<grid, kPreThreads, 0, stream>>>(a, groups);
    return hipGetLastError();
}

size_t tile_lds_bytes(uint32_t B) {
    const size_t Bp = (static_cast<size_t>(B) + 63u) & ~static_cast<size_t>(63u);
    return 6u * Bp + 2u * kLvLds;
}

hipError_t tile_set_limit(size_t bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&wilson_tile_kernel<false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(bytes));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&wilson_tile_kernel<true>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

int tile_max_active(uint32_t threads, size_t lds, bool weighted) {
    int blocks = 0;
    const void *f = weighted ? reinterpret_cast<const void *>(&wilson_tile_kernel<true>)
                             : reinterpret_cast<const void *>(&wilson_tile_kernel<false>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, static_cast<int>(threads), lds) !=
        hipSuccess)
        return 0;
    return blocks;
}

hipError_t launch_wilson_tile(const TileArgs &a, uint32_t threads, size_t lds, hipStream_t stream) {
    if (a.n == 0 || a.tree_count == 0 || a.slots == 0) return hipSuccess;
    if (a.B == 0 || a.B > kTileMax || a.Bp % 64u || a.Bp < a.B) return hipErrorInvalidValue;
    if (lds < tile_lds_bytes(a.B)) return hipErrorInvalidValue;
    const size_t bw = 4u * static_cast<size_t>((a.n + 31u) >> 5);
    if ((a.bits_lds || !a.xb) && bw > lds) return hipErrorInvalidValue;
    if (a.wsum) wilson_tile_kernel<true><<<a.slots, threads, lds, stream>>>(a);
    else wilson_tile_kernel<false><<<a.slots, threads, lds, stream>>>(a);
    return hipGetLastError();
}

}  // namespace fc
