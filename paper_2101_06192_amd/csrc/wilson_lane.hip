// Lane-per-tree Wilson sampler (Algorithm 3 of the paper on G*, rooted at u*).
//
// Each active lane owns one slot of per-tree state (n packed 64-bit words,
// see fc_device.hpp) and samples whole trees one after another, taking tree
// indices from a device queue.  Within a tree the lane runs Wilson's walk in
// the "overwrite next[]" form: the last arrow drawn at a vertex replaces the
// earlier ones, which erases loops chronologically, and a retrace from the
// start vertex adds the loop-erased path to the tree.  Vertices are started
// in a rotated identity order instead of ascending degree: by Wilson's
// cycle-popping theorem the tree and the per-vertex arrow counts do not
// depend on the start order, because arrows are keyed by (vertex, arrow
// index, tree, stream).
//
// Control flow is one loop with a per-lane mode (SCAN / WALK / RETRACE) so a
// wave keeps all lanes busy whatever mode each is in; every iteration makes
// one dependent load of the current vertex's state word.
#include "fc_kernels.hpp"

namespace fc {

namespace {

enum : uint32_t { kScan = 0, kWalk = 1, kRetrace = 2 };

template <bool kWeighted>
__global__ __launch_bounds__(64) void wilson_lane_kernel(LaneArgs a) {
    const uint32_t lane = threadIdx.x;
    if (lane >= a.lanes_per_wave) return;
    const uint32_t slot = blockIdx.x * a.lanes_per_wave + lane;
    if (slot >= a.slots) return;

    const uint32_t n = a.n;
    uint64_t *__restrict__ st = a.state + static_cast<size_t>(slot) * n;
    const int32_t *__restrict__ col = a.col_idx;
    const VRec *__restrict__ vrec = a.vrec;

    uint32_t ep = 0;  // the slot's words start zeroed: epoch 0 means fresh for tree 1
    unsigned long long lane_steps = 0, lane_roots = 0, lane_digest = 0;
    unsigned int err = 0;

    for (;;) {
        const uint32_t ti = atomicAdd(a.queue, 1u);
        if (ti >= a.tree_count) break;
        ep ^= 1u;
        const uint32_t t = a.tree_begin + ti;

        // start scanning at a tree-dependent offset so concurrent trees touch
        // different rows of R at different times
        uint32_t s = static_cast<uint32_t>(
            (static_cast<unsigned long long>(mix64(t) >> 32) * n) >> 32);
        uint32_t scanned = 0;
        uint32_t cur = s;
        uint32_t mode = kScan;
        unsigned long long steps = 0, digest = 0;
        uint32_t roots = 0;

        while (true) {
            const uint64_t w = (cur < n) ? st[cur] : 0ull;
            const bool intree = (cur >= n) || sw::in_tree(w, ep);
            if (mode == kScan) {
                if (intree) {
                    if (++scanned == n) break;
                    s = (s + 1 == n) ? 0u : s + 1;
                    cur = s;
                    continue;
                }
                mode = kWalk;
            }
            if (mode == kWalk) {
                if (intree) {  // the walk reached T (or u*): add its loop erasure
                    mode = kRetrace;
                    cur = s;
                    continue;
                }
                const uint32_t k = sw::visits(w, ep);
                const VRec r = load_vrec(vrec, cur);
                const Philox4 x = philox4x32_10(cur, k, t, a.stream_id, a.key0, a.key1);
                const uint32_t nxt = arrow_target<kWeighted>(r, x.x0, x.x1, col, a.wsum, a.wthr, n);
                if (k + 1 > a.k_limit) err |= kErrVisitOverflow;
                st[cur] = sw::pack(nxt, k + 1, ep);
                if (++steps > a.step_cap) {  // never reached by a valid walk; keeps the kernel finite
                    err |= kErrStepCap;
                    break;
                }
                cur = nxt;
                continue;
            }
            // kRetrace: cur is on the loop-erased path, not yet in T
            if (intree) {
                mode = kScan;
                cur = s;
                continue;
            }
            const uint32_t nxt = sw::next(w);
            st[cur] = w | sw::kInTree;
            digest += mix64((static_cast<unsigned long long>(cur) << 32) | nxt);
            if (nxt == n) {
                atomicAdd(&a.root_counts[cur], 1u);
                ++roots;
            }
            if (a.visit_counts) atomicAdd(&a.visit_counts[cur], static_cast<unsigned long long>(sw::visits(w, ep)));
            cur = nxt;
        }
        if (err & kErrStepCap) break;  // the call fails; stop this lane

        if (a.tree_digests) a.tree_digests[ti] = digest;
        if (a.tree_steps) a.tree_steps[ti] = steps;
        if (a.parents || a.tree_visits) {
            for (uint32_t v = 0; v < n; ++v) {
                const uint64_t w = st[v];
                if (a.parents) a.parents[static_cast<size_t>(ti) * n + v] = static_cast<int32_t>(sw::next(w));
                if (a.tree_visits) a.tree_visits[static_cast<size_t>(ti) * n + v] = sw::visits(w, ep);
            }
        }
        lane_steps += steps;
        lane_roots += roots;
        lane_digest += digest;
    }
    if (lane_steps) {
        atomicAdd(&a.totals->walk_steps, lane_steps);
        atomicAdd(&a.totals->roots, lane_roots);
        atomicAdd(&a.totals->digest_sum, lane_digest);
    }
    if (err) atomicOr(&a.totals->error, err);
}

}  // namespace

hipError_t launch_wilson_lane(const LaneArgs &a, hipStream_t stream) {
    if (a.n == 0 || a.tree_count == 0 || a.slots == 0) return hipSuccess;
    const uint32_t lpw = a.lanes_per_wave;
    const uint32_t blocks = (a.slots + lpw - 1) / lpw;
    if (a.wsum) wilson_lane_kernel<true><<<blocks, 64, 0, stream>>>(a);
    else wilson_lane_kernel<false><<<blocks, 64, 0, stream>>>(a);
    return hipGetLastError();
}

}  // namespace fc
