// Persistent counting kernel for gfx950.
//
// What it computes: the number of embeddings of a pattern under one
// configuration (schedule + restriction closure), i.e. the nested-loop search
// of Section II-B / IV-B with candidate sets formed by intersecting sorted
// neighbor lists and cut by the restrictions (the generated code of Fig.
// pseudocode_performance), with every level's injectivity enforced
// (Section II-A requires a bijection).
//
// How it maps to the machine:
//   * Tasks are root edges (v0, v1) = the first two loops fused, taken from a
//     device-wide atomic queue in chunks (the fine-grained task partitioning
//     of Section IV-E, as a lock-free queue instead of a master thread). Root
//     arrays are ordered by their smaller (higher-degree) endpoint, so hubs
//     go first, and the heaviest roots can be split over their level-2
//     candidates into several tasks.
//   * A group of G lanes (G in {64, 32, 16, 8}) of one wavefront shares one
//     search path. Intersections are group-cooperative (each lane
//     binary-searches one element of the smaller list in the larger one;
//     ballot + popcount compact the hits). G < 64 runs 64/G independent paths
//     per wavefront, which pays on graphs whose lists are short.
//   * Intersection results ("tmp" sets) live in a per-group scratch region in
//     HBM; they are written and re-read while hot in L2.
//   * The second-to-last level is spread over the lanes (leaf mode 1: each
//     lane counts the last level for its own candidate), walked with the
//     group counting each last level together (leaf mode 2), flattened with
//     the level above it into one balanced batch (leaf mode 3), or spread over
//     the lanes with long hub-tested lists walked by the whole group (leaf
//     mode 4).
//   * Hub vertices carry dense neighbor bitmaps: a membership test against a
//     hub's list is one word load.
//   * The last level is never enumerated: its count is
//     |C ∩ [lo, hi)| minus the earlier bound vertices that fall in it.
//   * Counts: uint64 per lane, wavefront tree reduction with carry detection,
//     one atomic per wavefront; wrap-around sets the overflow flag.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "sets.hpp"

namespace gpcount {

using namespace gpdev;

constexpr int kBlock = 256;

// Kernel modes: plain count, per-root counts, or accounting of the
// algorithmic bytes of the paper's cost model (never timed).
enum { MODE_PLAIN = 0, MODE_PER_ROOT = 1, MODE_ACCOUNT = 2 };

struct CountArgs {
    const int64_t* row_ptr;
    const int32_t* col;
    const int2* roots;
    int64_t n_roots;      // sampled roots: roots[root_offset + r * root_stride], r < n_roots
    int64_t root_offset;
    int64_t root_stride;
    // The first split_roots sampled roots (the heaviest: root arrays are
    // ordered by their hub endpoint) are each split into split_ways tasks, the
    // j-th of which binds only every split_ways-th level-2 candidate from j on.
    // Tasks: split_roots * split_ways split ones, then one per remaining root.
    int64_t n_tasks;
    int64_t split_roots;
    int32_t split_ways;
    const uint32_t* hub_bits;  // n_hubs dense bitmaps of hub_words words
    int64_t hub_words;
    int32_t n_hubs;
    int32_t* scratch;
    int64_t buf_cap;
    unsigned long long* queue;
    unsigned long long* result;    // {count, overflow, algorithmic bytes}
    unsigned long long* per_root;  // optional, indexed by CSR entry of (v0, v1)
    // optional {sum over wavefronts of active clock ticks, wavefronts, longest
    // chunk of tasks in ticks}: the balanced run time of a sample and its tail
    unsigned long long* busy;
    // with busy: stop taking tasks once a wavefront has run this many clock
    // ticks (0: no limit); the count is then incomplete and flagged (bit 2)
    uint64_t budget_ticks;
    // optional (leaf mode 4, plans the host found eligible): per group,
    // n_hubs words {root tag, |N(x) & pre & cut|} for hub candidates x
    unsigned long long* memo;
    int32_t chunk;
};

typedef void (*KernelFn)(GpPlanDesc, CountArgs);

// Batched launch: one entry per plan, in task order.
constexpr int kBatchMaxPlans = 64;

struct BatchPlan {
    const int2* roots;    // this plan's whole root array (cut already applied)
    int64_t n_tasks;      // tasks of this plan in the launch
    int64_t task_begin;   // first global task index of this plan
    int64_t task_offset;  // where in the plan's own task space the launch starts
    int64_t split_roots;  // as in CountArgs: the first split_roots roots run as
    int32_t split_ways;   // split_ways tasks each
    int32_t leaf;         // 1 or 3 (flattened last two levels)
};

// Root of task t, and the level-2 slice it binds: the first split_roots roots
// are split_ways tasks each, the rest one task each.
__device__ __forceinline__ int64_t task_root(int64_t t, int64_t split_roots, int32_t split_ways, int32_t& sj,
                                             int32_t& sJ) {
    const int64_t split_tasks = split_roots * (int64_t)split_ways;
    if (t < split_tasks) {
        const int64_t r = t / split_ways;
        sj = (int32_t)(t - r * split_ways);
        sJ = split_ways;
        return r;
    }
    sj = 0;
    sJ = 1;
    return t - split_tasks + split_roots;
}

struct BatchArgs {
    const int64_t* row_ptr;
    const int32_t* col;
    const GpPlanDesc* descs;  // device, np entries
    const BatchPlan* plans;   // device, np entries
    int32_t np;
    int64_t total_tasks;
    const uint32_t* hub_bits;
    int64_t hub_words;
    int32_t n_hubs;
    int32_t* scratch;
    int64_t buf_cap;
    int32_t nbuf;  // buffer slots per group (max over plans)
    unsigned long long* queue;
    unsigned long long* result;  // {count, overflow, busy clock ticks} per plan
    int32_t chunk;
};

typedef void (*BatchFn)(BatchArgs);

// Values equal in every lane of a group. With 64-lane groups they are
// wavefront-uniform: readfirstlane lets the compiler keep them, and what is
// computed from them (bound vertices, set bounds, loop counters), in scalar
// registers, which leaves vector registers for more resident wavefronts.
template <int G>
__device__ __forceinline__ int32_t uni(int32_t x) {
    if constexpr (G == 64) return __builtin_amdgcn_readfirstlane(x);
    else return x;
}
template <int G>
__device__ __forceinline__ int64_t uni64(int64_t x) {
    if constexpr (G == 64) {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)x);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)x >> 32));
        return (int64_t)(((uint64_t)hi << 32) | lo);
    } else {
        return x;
    }
}
// Cut a group-uniform set to [lo, hi) (lo, hi group-uniform).
template <int G>
__device__ __forceinline__ Set trim_u(Set s, int32_t lo, int32_t hi) {
    int32_t b = lo > 0 ? uni<G>(lower_bound(s.p, s.n, lo)) : 0;
    int32_t e = hi < 0x7fffffff ? uni<G>(lower_bound(s.p, s.n, hi)) : s.n;
    if (e < b) e = b;
    return Set{s.p + b, e - b, s.bits};
}

template <int G>
struct Ctx {
    const int64_t* row_ptr;
    const int32_t* col;
    int32_t* bufs;
    int64_t cap;
    int32_t* lens;  // LDS: length per buffer slot
    uint64_t* bytes;  // accounting mode: per-lane algorithmic bytes
    const uint32_t* hub_bits;
    int64_t hub_words;
    int32_t n_hubs;
    int32_t sj, sJ;     // level-2 slice of the current task: candidates sj, sj + sJ, ...
    uint64_t deadline;  // clock tick after which every search loop stops (0: none)
    unsigned long long* memo;  // this group's last-level memo (null: none)
    uint32_t tag;              // current root + 1, the memo's validity tag
    Group<G> g;

    __device__ __forceinline__ bool expired() const {
        return deadline != 0 && wall_clock64() > deadline;
    }

    __device__ __forceinline__ Set nbr(int32_t v) const {
        int64_t b = row_ptr[v], e = row_ptr[v + 1];
        return Set{col + b, (int32_t)(e - b), v < n_hubs ? hub_bits + (int64_t)v * hub_words : nullptr};
    }
    __device__ __forceinline__ Set buf(int slot) const {
        return Set{bufs + (int64_t)slot * cap, lens[slot], nullptr};
    }
    // the same for a group-uniform vertex or slot
    __device__ __forceinline__ Set nbr_u(int32_t v) const {
        const int64_t b = uni64<G>(row_ptr[v]), e = uni64<G>(row_ptr[v + 1]);
        return Set{col + b, (int32_t)(e - b), v < n_hubs ? hub_bits + (int64_t)v * hub_words : nullptr};
    }
    __device__ __forceinline__ Set buf_u(int slot) const {
        return Set{bufs + (int64_t)slot * cap, uni<G>(lens[slot]), nullptr};
    }
};

// v[idx] for a runtime idx without dynamic register indexing.
template <int K>
__device__ __forceinline__ int32_t pick(const int32_t (&v)[K], int idx) {
    int32_t r = v[0];
#pragma unroll
    for (int j = 1; j < K; ++j) r = (idx == j) ? v[j] : r;
    return r;
}

template <int K>
__device__ __forceinline__ void bounds(uint32_t hi_src, uint32_t lo_src, const int32_t (&v)[K],
                                       int32_t& lo, int32_t& hi) {
    lo = 0;
    hi = 0x7fffffff;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if ((hi_src >> j) & 1u) hi = min(hi, v[j]);
        if ((lo_src >> j) & 1u) lo = max(lo, v[j] + 1);
    }
}

template <int K>
__device__ __forceinline__ bool inj_hit(uint32_t inj, const int32_t (&v)[K], int32_t x) {
    bool hit = false;
#pragma unroll
    for (int j = 0; j < K; ++j)
        if ((inj >> j) & 1u) hit |= (v[j] == x);
    return hit;
}

__device__ __forceinline__ void add_count(uint64_t& acc, uint64_t c, bool& ovf) {
    uint64_t s = acc + c;
    ovf |= (s < acc);
    acc = s;
}

// Algorithmic bytes of one binary search in a sorted list of n int32.
__device__ __forceinline__ uint64_t probe_bytes(int32_t n) {
    return 4ull * (uint64_t)(32 - __clz(n > 0 ? n : 1));
}

__device__ __forceinline__ void group_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Builds scheduled right after level h is bound.
template <int K, int G, int MODE>
__device__ __forceinline__ void run_builds(const GpPlanDesc& d, const Ctx<G>& c, int h,
                                           const int32_t (&v)[K]) {
    const int b0 = d.build_begin[h], b1 = d.build_end[h];
    for (int t = b0; t < b1; ++t) {
        const GpBuild& b = d.b[t];
        int32_t lo, hi;
        bounds<K>(b.hi_src, b.lo_src, v, lo, hi);
        Set A = b.src_buf >= 0 ? c.buf_u(b.src_buf) : c.nbr_u(pick<K>(v, b.src_list));
        Set B = c.nbr_u(pick<K>(v, b.with_list));
        A = trim_u<G>(A, lo, hi);
        B = trim_u<G>(B, lo, hi);
        if constexpr (MODE == MODE_ACCOUNT)
            if (c.g.gl == 0) *c.bytes += 4ull * (uint64_t)(A.n + B.n);
        int32_t n = uni<G>(intersect_into<G>(c.g, A, B, c.bufs + (int64_t)b.dst * c.cap));
        group_fence();
        c.lens[b.dst] = n;
        group_fence();
    }
}

// Count of the last level for bound values v[0..K-2], by one lane.
template <int K, int G, int MODE>
__device__ __forceinline__ uint32_t leaf_serial(const GpPlanDesc& d, const Ctx<G>& c,
                                                const int32_t (&v)[K]) {
    const GpLevel& lv = d.lv[K - 1];
    int32_t lo, hi;
    bounds<K>(lv.hi_src, lv.lo_src, v, lo, hi);
    if (lv.last_list < 0) {
        Set S = lv.list >= 0 ? c.nbr(pick<K>(v, lv.list)) : c.buf(lv.buf);
        if constexpr (MODE == MODE_ACCOUNT)
            *c.bytes += probe_bytes(S.n) * (uint64_t)((lo > 0) + (hi < 0x7fffffff));
        S = trim(S, lo, hi);
        uint32_t cnt = (uint32_t)S.n;
#pragma unroll
        for (int j = 0; j < K - 1; ++j) {
            if ((lv.inj >> j) & 1u) {
                int32_t y = v[j];
                if (y >= lo && y < hi) {
                    if constexpr (MODE == MODE_ACCOUNT) *c.bytes += probe_bytes(S.n);
                    if (member(S, y)) --cnt;
                }
            }
        }
        return cnt;
    }
    Set A = lv.pre_buf >= 0 ? c.buf(lv.pre_buf) : c.nbr(pick<K>(v, lv.pre_list));
    Set B = c.nbr(pick<K>(v, lv.last_list));
    // injectivity folded into the intersection: matches equal to an earlier
    // image are not counted
    const uint32_t inj = lv.inj;
    auto skip = [&](int32_t x) { return inj_hit<K>(inj, v, x); };
    // a hub operand is tested by bits, so only the other operand is cut
    if constexpr (MODE != MODE_ACCOUNT) {
        if (B.bits && A.n <= kShortList && A.n * 4 <= B.n) return count_bits_range(A, lo, hi, B.bits, skip);
        if (A.bits && B.n <= kShortList && B.n * 4 <= A.n) return count_bits_range(B, lo, hi, A.bits, skip);
    }
    if (B.bits) {
        const Set Ac = trim(A, lo, hi);
        if (Ac.n * 4 <= B.n) {
            if constexpr (MODE == MODE_ACCOUNT) *c.bytes += 4ull * (uint64_t)(Ac.n + trim(B, lo, hi).n);
            return count_bits(Ac, B.bits, skip);
        }
    } else if (A.bits) {
        const Set Bc = trim(B, lo, hi);
        if (Bc.n * 4 <= A.n) {
            if constexpr (MODE == MODE_ACCOUNT) *c.bytes += 4ull * (uint64_t)(Bc.n + trim(A, lo, hi).n);
            return count_bits(Bc, A.bits, skip);
        }
    }
    A = trim(A, lo, hi);
    B = trim(B, lo, hi);
    if constexpr (MODE == MODE_ACCOUNT) *c.bytes += 4ull * (uint64_t)(A.n + B.n);
    return intersect_count_serial(A, B, skip);
}

// Count of the last level, computed by the whole group (same value in every lane).
template <int K, int G, int MODE>
__device__ __forceinline__ uint32_t leaf_group(const GpPlanDesc& d, const Ctx<G>& c,
                                               const int32_t (&v)[K]) {
    const GpLevel& lv = d.lv[K - 1];
    if (lv.last_list < 0) {
        // every lane computes the same count; only lane 0 keeps the bytes
        uint64_t keep = 0;
        if constexpr (MODE == MODE_ACCOUNT) keep = *c.bytes;
        uint32_t r = leaf_serial<K, G, MODE>(d, c, v);
        if constexpr (MODE == MODE_ACCOUNT)
            if (c.g.gl != 0) *c.bytes = keep;
        return r;
    }
    int32_t lo, hi;
    bounds<K>(lv.hi_src, lv.lo_src, v, lo, hi);
    Set A = lv.pre_buf >= 0 ? c.buf_u(lv.pre_buf) : c.nbr_u(pick<K>(v, lv.pre_list));
    Set B = c.nbr_u(pick<K>(v, lv.last_list));
    A = trim_u<G>(A, lo, hi);
    B = trim_u<G>(B, lo, hi);
    if constexpr (MODE == MODE_ACCOUNT)
        if (c.g.gl == 0) *c.bytes += 4ull * (uint64_t)(A.n + B.n);
    const uint32_t inj = lv.inj;
    return intersect_count_group<G>(c.g, A, B, [&](int32_t x) { return inj_hit<K>(inj, v, x); });
}

// Counting with inclusion-exclusion over the last two levels (Section IV-D,
// k = 2 inner sets): for bound values v[0..K-3], the number of pairs (y, z)
// with y in S1, z in S2, y != z, where S1, S2 are the candidate sets of
// levels K-2 and K-1 (outer images removed): |S1| |S2| - |S1 & S2|. By one
// lane.
template <int K, int G, int MODE>
__device__ __forceinline__ uint64_t iep_leaf_serial(const GpPlanDesc& d, const Ctx<G>& c,
                                                    const int32_t (&v)[K]) {
    const GpLevel& l1 = d.lv[K - 2];
    const GpLevel& l2 = d.lv[K - 1];
    int32_t lo1, hi1, lo2, hi2;
    bounds<K>(l1.hi_src, l1.lo_src, v, lo1, hi1);
    bounds<K>(l2.hi_src, l2.lo_src, v, lo2, hi2);
    const Set S1 = l1.list >= 0 ? c.nbr(pick<K>(v, l1.list)) : c.buf(l1.buf);
    const Set S2 = l2.list >= 0 ? c.nbr(pick<K>(v, l2.list)) : c.buf(l2.buf);
    const Set A = trim(S1, lo1, hi1);
    const Set B = trim(S2, lo2, hi2);
    uint64_t c1 = (uint64_t)A.n, c2 = (uint64_t)B.n;
#pragma unroll
    for (int j = 0; j < K - 2; ++j) {
        const int32_t y = v[j];
        if (((l1.inj >> j) & 1u) && y >= lo1 && y < hi1 && member(A, y)) --c1;
        if (((l2.inj >> j) & 1u) && y >= lo2 && y < hi2 && member(B, y)) --c2;
    }
    const int32_t lo = max(lo1, lo2), hi = min(hi1, hi2);
    const Set A12 = trim(A, lo, hi), B12 = trim(B, lo, hi);
    const uint32_t inj = (uint32_t)l1.inj | (uint32_t)l2.inj;
    const uint32_t c12 = intersect_count_serial(A12, B12, [&](int32_t x) { return inj_hit<K>(inj, v, x); });
    if constexpr (MODE == MODE_ACCOUNT)
        *c.bytes += 2 * probe_bytes(S1.n) + 2 * probe_bytes(S2.n) + 4ull * (uint64_t)(A12.n + B12.n);
    return c1 * c2 - c12;
}

// The same computed by the whole group (same value in every lane).
template <int K, int G, int MODE>
__device__ __forceinline__ uint64_t iep_leaf_group(const GpPlanDesc& d, const Ctx<G>& c,
                                                   const int32_t (&v)[K]) {
    const GpLevel& l1 = d.lv[K - 2];
    const GpLevel& l2 = d.lv[K - 1];
    int32_t lo1, hi1, lo2, hi2;
    bounds<K>(l1.hi_src, l1.lo_src, v, lo1, hi1);
    bounds<K>(l2.hi_src, l2.lo_src, v, lo2, hi2);
    const Set S1 = l1.list >= 0 ? c.nbr_u(pick<K>(v, l1.list)) : c.buf_u(l1.buf);
    const Set S2 = l2.list >= 0 ? c.nbr_u(pick<K>(v, l2.list)) : c.buf_u(l2.buf);
    const Set A = trim_u<G>(S1, lo1, hi1);
    const Set B = trim_u<G>(S2, lo2, hi2);
    uint64_t c1 = (uint64_t)A.n, c2 = (uint64_t)B.n;
#pragma unroll
    for (int j = 0; j < K - 2; ++j) {
        const int32_t y = v[j];
        if (((l1.inj >> j) & 1u) && y >= lo1 && y < hi1 && member(A, y)) --c1;
        if (((l2.inj >> j) & 1u) && y >= lo2 && y < hi2 && member(B, y)) --c2;
    }
    const int32_t lo = max(lo1, lo2), hi = min(hi1, hi2);
    const Set A12 = trim_u<G>(A, lo, hi), B12 = trim_u<G>(B, lo, hi);
    const uint32_t inj = (uint32_t)l1.inj | (uint32_t)l2.inj;
    const uint32_t c12 =
        intersect_count_group<G>(c.g, A12, B12, [&](int32_t x) { return inj_hit<K>(inj, v, x); });
    if constexpr (MODE == MODE_ACCOUNT)
        if (c.g.gl == 0)
            *c.bytes += 2 * probe_bytes(S1.n) + 2 * probe_bytes(S2.n) + 4ull * (uint64_t)(A12.n + B12.n);
    return c1 * c2 - c12;
}

// The last two enumerated levels flattened into one load-balanced batch
// (leaf mode 3): each lane takes a candidate x of level K-3 and cuts its
// level-(K-2) candidate list; a group prefix sum over the list lengths then
// deals every (x, y) pair to a lane, which counts the last level alone. This
// keeps all G lanes busy when the per-candidate lists are short (sparse
// graphs), where leaf mode 1 leaves most lanes idle. Only used when no build
// runs after level K-3 is bound.
template <int K, int G, int MODE>
__device__ void flat_leaf(const GpPlanDesc& d, const Ctx<G>& c, const int32_t (&v)[K], Set S,
                          int32_t st, uint32_t inj_l, uint64_t& acc, bool& ovf) {
    constexpr int L = K - 3;
    const GpLevel& l2 = d.lv[K - 2];
    for (int32_t base = 0; base < S.n; base += G) {
        if (c.expired()) break;
        const int32_t i = base + c.g.gl;
        int32_t x2 = 0;
        Set C{nullptr, 0, nullptr};
        if (i < S.n) {
            x2 = S.p[(int64_t)i * st];
            if (!inj_hit<K>(inj_l, v, x2)) {
                int32_t w[K];
#pragma unroll
                for (int j = 0; j < K; ++j) w[j] = v[j];
                w[L] = x2;
                int32_t lo, hi;
                bounds<K>(l2.hi_src, l2.lo_src, w, lo, hi);
                C = l2.list >= 0 ? c.nbr(pick<K>(w, l2.list)) : c.buf(l2.buf);
                C = trim(C, lo, hi);
            }
        }
        // inclusive prefix sum of the list lengths over the group
        int32_t incl = C.n;
#pragma unroll
        for (int off = 1; off < G; off <<= 1) {
            int32_t t = __shfl_up(incl, off, G);
            if (c.g.gl >= off) incl += t;
        }
        const int32_t total = __shfl(incl, G - 1, G);
        const int32_t excl = incl - C.n;
        const long long cp = (long long)C.p;
        if constexpr (MODE == MODE_ACCOUNT)
            if (c.g.gl == 0) *c.bytes += 4ull * (uint64_t)total;
        for (int32_t t0 = 0; t0 < total; t0 += G) {
            const int32_t item = t0 + c.g.gl;
            // owner: the last lane whose exclusive prefix is <= item
            int32_t o = 0;
#pragma unroll
            for (int step = G / 2; step >= 1; step >>= 1) {
                const int32_t e2 = __shfl(excl, o + step, G);
                if (e2 <= item) o += step;
            }
            const int32_t ox = __shfl(x2, o, G);
            const int32_t oex = __shfl(excl, o, G);
            const int32_t* op = (const int32_t*)__shfl(cp, o, G);
            if (item < total) {
                const int32_t y = op[item - oex];
                int32_t w[K];
#pragma unroll
                for (int j = 0; j < K; ++j) w[j] = v[j];
                w[L] = ox;
                if (!inj_hit<K>(l2.inj, w, y)) {
                    w[K - 2] = y;
                    add_count(acc, leaf_serial<K, G, MODE>(d, c, w), ovf);
                }
            }
        }
    }
}

// Leaf mode 4: lanes take different second-to-last candidates x as in leaf
// mode 1, except that where the last level is pre & N(x) with a group-uniform
// pre that is a hub bitmap, a long N(x) (more than kCoopList elements after the
// cut) is walked by the whole group: one hub candidate otherwise keeps one
// lane busy for thousands of elements while the other lanes of its wavefront
// idle. The group takes the long lists one after another (ballot), each lane
// every G-th element (coalesced loads), and each element costs one bit test
// in the shared bitmap. Returns false (nothing done) when the last level has
// another form; the caller then counts it as in leaf mode 1.
//
// With a memo (c.memo), the count |N(x) & pre & [lo, hi)| of a hub candidate
// x is kept per root edge: the host enables it only when pre and the cut come
// from the two root levels, so for one root they are fixed and the count
// depends on x alone, however the levels between were bound (split tasks of
// one root that a group takes in a row share it). The earlier
// images the last level must avoid are then all parents of x, so each lies
// in N(x), and whether it falls in the set is its pre bit and the cut: they
// are subtracted per lane.
constexpr int32_t kCoopList = 64;

template <int K, int G, int MODE>
__device__ bool coop_bits_leaf(const GpPlanDesc& d, const Ctx<G>& c, const int32_t (&v)[K], Set S, int32_t st,
                               uint32_t inj_l, uint64_t& acc, bool& ovf) {
    const GpLevel& ll = d.lv[K - 1];
    if (ll.last_list != K - 2) return false;
    const Set A = ll.pre_buf >= 0 ? c.buf_u(ll.pre_buf) : c.nbr_u(pick<K>(v, ll.pre_list));
    if (!A.bits) return false;
    const uint32_t* bits = A.bits;
    for (int32_t base = 0; base < S.n; base += G) {
        if (c.expired()) break;
        const int32_t i = base + c.g.gl;
        int32_t x = -1;
        Set B{nullptr, 0, nullptr};
        bool longl = false;
        if (i < S.n) {
            x = S.p[(int64_t)i * st];
            if (!inj_hit<K>(inj_l, v, x)) {
                int32_t w[K];
#pragma unroll
                for (int j = 0; j < K; ++j) w[j] = v[j];
                w[K - 2] = x;
                int32_t lo, hi;
                bounds<K>(ll.hi_src, ll.lo_src, w, lo, hi);
                auto skip = [&](int32_t y) { return inj_hit<K>(ll.inj, w, y); };
                if (c.memo && x < c.n_hubs) {
                    // earlier images in the set: parents of x, so in N(x)
                    uint32_t corr = 0;
#pragma unroll
                    for (int j = 0; j < K - 1; ++j)
                        if ((ll.inj >> j) & 1u) {
                            const int32_t y = w[j];
                            corr += (y >= lo && y < hi && ((bits[y >> 5] >> (y & 31)) & 1u)) ? 1u : 0u;
                        }
                    const unsigned long long e = c.memo[x];
                    if ((uint32_t)(e >> 32) == c.tag) {
                        add_count(acc, (uint32_t)e - corr, ovf);
                    } else {
                        B = trim(c.nbr(x), lo, hi);
                        if (B.n <= kCoopList) {
                            const uint32_t all = count_bits(B, bits, [](int32_t) { return false; });
                            c.memo[x] = ((unsigned long long)c.tag << 32) | all;
                            add_count(acc, all - corr, ovf);
                        } else {
                            longl = true;
                        }
                    }
                } else {
                    B = c.nbr(x);
                    if (B.n <= kShortList) {
                        add_count(acc, count_bits_range(B, lo, hi, bits, skip), ovf);
                    } else {
                        B = trim(B, lo, hi);
                        if (B.n <= kCoopList) add_count(acc, count_bits(B, bits, skip), ovf);
                        else longl = true;
                    }
                }
            }
        }
        uint64_t m = c.g.ballot(longl);
        while (m) {
            const int o = __builtin_ctzll(m);
            m &= m - 1;
            const int32_t ox = __shfl(x, o, G);
            const int32_t on = __shfl(B.n, o, G);
            const int32_t* op = (const int32_t*)__shfl((long long)B.p, o, G);
            int32_t w[K];
#pragma unroll
            for (int j = 0; j < K; ++j) w[j] = v[j];
            w[K - 2] = ox;
            uint32_t cnt = 0, all = 0;
            for (int32_t j = c.g.gl; j < on; j += G) {
                const int32_t y = op[j];
                if ((bits[y >> 5] >> (y & 31)) & 1u) {
                    ++all;
                    cnt += !inj_hit<K>(ll.inj, w, y);
                }
            }
            add_count(acc, cnt, ovf);
            if (c.memo && ox < c.n_hubs) {
                // the long list of a hub candidate: keep its whole count
                const uint32_t tot = (uint32_t)c.g.sum(all);
                if (c.g.gl == 0) c.memo[ox] = ((unsigned long long)c.tag << 32) | tot;
            }
        }
    }
    return true;
}

template <int K, int L, int G, int LEAF, int MODE, bool IEP>
__device__ void search(const GpPlanDesc& d, const Ctx<G>& c, int32_t (&v)[K], uint64_t& acc,
                       bool& ovf) {
    const GpLevel& lv = d.lv[L];
    int32_t lo, hi;
    bounds<K>(lv.hi_src, lv.lo_src, v, lo, hi);
    Set S = lv.list >= 0 ? c.nbr_u(pick<K>(v, lv.list)) : c.buf_u(lv.buf);
    S = trim_u<G>(S, lo, hi);
    if constexpr (MODE == MODE_ACCOUNT)
        if (c.g.gl == 0) *c.bytes += 4ull * (uint64_t)S.n;
    // a split task binds only its slice of the level-2 candidates
    int32_t st = 1;
    if constexpr (L == 2) {
        if (c.sJ > 1) {
            S.n = S.n > c.sj ? (S.n - c.sj + c.sJ - 1) / c.sJ : 0;
            S.p += c.sj;
            st = c.sJ;
        }
    }
    if constexpr (IEP && L == K - 3) {
        // last outer level: every candidate adds its inclusion-exclusion count
        if (d.build_begin[L] == d.build_end[L]) {
            for (int32_t base = 0; base < S.n; base += G) {
                if (c.expired()) break;
                const int32_t i = base + c.g.gl;
                if (i < S.n) {
                    const int32_t x = S.p[(int64_t)i * st];
                    if (!inj_hit<K>(lv.inj, v, x)) {
                        int32_t w[K];
#pragma unroll
                        for (int j = 0; j < K; ++j) w[j] = v[j];
                        w[L] = x;
                        add_count(acc, iep_leaf_serial<K, G, MODE>(d, c, w), ovf);
                    }
                }
            }
        } else {
            for (int32_t t = 0; t < S.n; ++t) {
                if (c.expired()) break;
                const int32_t x = uni<G>(S.p[(int64_t)t * st]);
                if (inj_hit<K>(lv.inj, v, x)) continue;
                v[L] = x;
                run_builds<K, G, MODE>(d, c, L, v);
                const uint64_t cnt = iep_leaf_group<K, G, MODE>(d, c, v);
                if (c.g.gl == 0) add_count(acc, cnt, ovf);
            }
        }
    } else if constexpr (L == K - 2) {
        if constexpr (LEAF == 4 && MODE != MODE_ACCOUNT)
            if (coop_bits_leaf<K, G, MODE>(d, c, v, S, st, lv.inj, acc, ovf)) return;
        if constexpr (LEAF != 2) {
            for (int32_t base = 0; base < S.n; base += G) {
                if (c.expired()) break;
                int32_t i = base + c.g.gl;
                if (i < S.n) {
                    int32_t x = S.p[(int64_t)i * st];
                    if (!inj_hit<K>(lv.inj, v, x)) {
                        int32_t w[K];
#pragma unroll
                        for (int j = 0; j < K; ++j) w[j] = v[j];
                        w[K - 2] = x;
                        add_count(acc, leaf_serial<K, G, MODE>(d, c, w), ovf);
                    }
                }
            }
        } else {
            for (int32_t t = 0; t < S.n; ++t) {
                if (c.expired()) break;
                const int32_t x = uni<G>(S.p[(int64_t)t * st]);
                if (inj_hit<K>(lv.inj, v, x)) continue;
                v[K - 2] = x;
                uint32_t cnt = leaf_group<K, G, MODE>(d, c, v);
                if (c.g.gl == 0) add_count(acc, cnt, ovf);
            }
        }
    } else {
        if constexpr (LEAF == 3 && L == K - 3 && !IEP) {
            if (d.build_begin[L] == d.build_end[L]) {
                flat_leaf<K, G, MODE>(d, c, v, S, st, lv.inj, acc, ovf);
                return;
            }
        }
        for (int32_t t = 0; t < S.n; ++t) {
            if (c.expired()) break;
            const int32_t x = uni<G>(S.p[(int64_t)t * st]);
            if (inj_hit<K>(lv.inj, v, x)) continue;
            v[L] = x;
            run_builds<K, G, MODE>(d, c, L, v);
            search<K, L + 1, G, LEAF, MODE, IEP>(d, c, v, acc, ovf);
        }
    }
}

__device__ __forceinline__ int64_t entry_index(const int64_t* row_ptr, const int32_t* col,
                                               int32_t v0, int32_t v1) {
    int64_t b = row_ptr[v0];
    return b + lower_bound(col + b, (int32_t)(row_ptr[v0 + 1] - b), v1);
}

// Wavefronts per SIMD the compiler is asked to keep resident (it trims
// registers, spilling a few if it must). The searches are bound by the
// latency of scattered loads, so more resident wavefronts pay even against
// some spills. Measured on R-MAT 17 for k = 5 (64-lane groups with lanes on
// separate candidates: 8, others 6) and on Chung-Lu 7000 for k = 6 (64-lane
// groups 6, others 5); k >= 7 keeps the compiler's choice.
constexpr int occupancy_target(int K, int G, int LEAF) {
    return K > 6 ? 1 : K == 6 ? (G == 64 ? 6 : 5) : (G == 64 && (LEAF == 1 || LEAF == 4) ? 8 : 6);
}

template <int K, int G, int LEAF, int MODE, bool IEP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(occupancy_target(K, G, LEAF)))) void count_kernel(GpPlanDesc d, CountArgs a) {
    constexpr bool PER_ROOT = MODE == MODE_PER_ROOT;
    __shared__ int32_t s_len[kBlock / G][GP_DESC_MAX_BUILDS];
    Ctx<G> c;
    c.row_ptr = a.row_ptr;
    c.col = a.col;
    c.cap = a.buf_cap;
    c.hub_bits = a.hub_bits;
    c.hub_words = a.hub_words;
    c.n_hubs = a.n_hubs;
    const int grp = threadIdx.x / G;
    const int64_t group_id = (int64_t)blockIdx.x * (kBlock / G) + grp;
    c.bufs = a.scratch ? a.scratch + group_id * (int64_t)d.nbuf * a.buf_cap : nullptr;
    c.lens = s_len[grp];
    uint64_t bytes = 0;
    c.bytes = &bytes;
    c.sj = 0;
    c.sJ = 1;
    c.memo = a.memo ? a.memo + group_id * (int64_t)a.n_hubs : nullptr;
    c.tag = 0;
    const uint64_t t_begin = a.busy ? wall_clock64() : 0;
    c.deadline = a.busy && a.budget_ticks ? t_begin + a.budget_ticks : 0;
    uint64_t chunk_max = 0;
    bool stopped = false;

    uint64_t acc = 0;
    bool ovf = false;
    const int64_t chunk = a.chunk;

    for (;;) {
        unsigned long long t0 = 0;
        if (c.g.gl == 0) t0 = atomicAdd(a.queue, (unsigned long long)chunk);
        t0 = (unsigned long long)uni64<G>((int64_t)c.g.bcast(t0, 0));
        if ((int64_t)t0 >= a.n_tasks) break;
        const int64_t t1 = min((int64_t)t0 + chunk, a.n_tasks);
        const uint64_t t_chunk = a.busy ? wall_clock64() : 0;
        if constexpr (IEP && K == 4) {
            // the root is the last outer level
            if (d.build_begin[1] == d.build_end[1]) {
                for (int64_t base = (int64_t)t0; base < t1; base += G) {
                    const int64_t r = base + c.g.gl;
                    if (r < t1) {
                        const int2 e = a.roots[a.root_offset + r * a.root_stride];
                        if constexpr (MODE == MODE_ACCOUNT) bytes += 8;
                        int32_t w[K] = {e.x, e.y, 0, 0};
                        const uint64_t cnt = iep_leaf_serial<K, G, MODE>(d, c, w);
                        add_count(acc, cnt, ovf);
                        if constexpr (PER_ROOT) a.per_root[entry_index(a.row_ptr, a.col, e.x, e.y)] = cnt;
                    }
                }
            } else {
                for (int64_t r = (int64_t)t0; r < t1; ++r) {
                    int2 e = a.roots[a.root_offset + r * a.root_stride];
                    e.x = uni<G>(e.x);
                    e.y = uni<G>(e.y);
                    if constexpr (MODE == MODE_ACCOUNT)
                        if (c.g.gl == 0) bytes += 8;
                    int32_t v[K] = {e.x, e.y, 0, 0};
                    run_builds<K, G, MODE>(d, c, 1, v);
                    const uint64_t cnt = iep_leaf_group<K, G, MODE>(d, c, v);
                    if (c.g.gl == 0) add_count(acc, cnt, ovf);
                    if constexpr (PER_ROOT)
                        if (c.g.gl == 0) a.per_root[entry_index(a.row_ptr, a.col, e.x, e.y)] = cnt;
                }
            }
        } else if constexpr (K <= 3 && LEAF != 2) {
            // lanes take different roots
            for (int64_t base = (int64_t)t0; base < t1; base += G) {
                int64_t r = base + c.g.gl;
                if (r < t1) {
                    int2 e = a.roots[a.root_offset + r * a.root_stride];
                    uint64_t cnt = 1;
                    if constexpr (MODE == MODE_ACCOUNT) bytes += 8;
                    if constexpr (K == 3) {
                        int32_t w[K] = {e.x, e.y, 0};
                        cnt = leaf_serial<K, G, MODE>(d, c, w);
                    }
                    add_count(acc, cnt, ovf);
                    if constexpr (PER_ROOT)
                        a.per_root[entry_index(a.row_ptr, a.col, e.x, e.y)] = cnt;
                }
            }
        } else {
            for (int64_t t = (int64_t)t0; t < t1; ++t) {
                const int64_t r = task_root(t, a.split_roots, a.split_ways, c.sj, c.sJ);
                c.tag = (uint32_t)(r + 1);
                int2 e = a.roots[a.root_offset + r * a.root_stride];
                e.x = uni<G>(e.x);
                e.y = uni<G>(e.y);
                const uint64_t before = acc;
                if constexpr (MODE == MODE_ACCOUNT)
                    if (c.g.gl == 0) bytes += 8;
                if constexpr (K <= 3) {
                    uint64_t cnt = 1;
                    if constexpr (K == 3) {
                        int32_t w[K] = {e.x, e.y, 0};
                        cnt = leaf_group<K, G, MODE>(d, c, w);
                    }
                    if (c.g.gl == 0) add_count(acc, cnt, ovf);
                } else {
                    int32_t v[K];
#pragma unroll
                    for (int j = 0; j < K; ++j) v[j] = 0;
                    v[0] = e.x;
                    v[1] = e.y;
                    run_builds<K, G, MODE>(d, c, 1, v);
                    search<K, 2, G, LEAF, MODE, IEP>(d, c, v, acc, ovf);
                }
                if constexpr (PER_ROOT) {
                    uint64_t mine = c.g.sum(acc - before);
                    if (c.g.gl == 0) a.per_root[entry_index(a.row_ptr, a.col, e.x, e.y)] = mine;
                }
            }
        }
        if (a.busy) {
            const uint64_t now = wall_clock64();
            chunk_max = max(chunk_max, now - t_chunk);
            if (c.deadline && now > c.deadline) {
                stopped = true;
                break;
            }
        }
    }

    // wavefront reduction with carry detection, one atomic per wavefront
    uint64_t s = acc;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        uint64_t t = __shfl_xor(s, off, 64);
        uint64_t u = s + t;
        ovf |= (u < s);
        s = u;
    }
    const bool any_ovf = __ballot(ovf) != 0;
    if constexpr (MODE == MODE_ACCOUNT) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) bytes += __shfl_xor(bytes, off, 64);
    }
    uint64_t cm = chunk_max;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) cm = max(cm, (uint64_t)__shfl_xor(cm, off, 64));
    const bool any_stop = __ballot(stopped) != 0;
    if (__lane_id() == 0) {
        unsigned long long old = atomicAdd(&a.result[0], (unsigned long long)s);
        if (any_ovf || old + s < old) atomicOr(&a.result[1], 1ull);
        if (any_stop) atomicOr(&a.result[1], 4ull);
        if constexpr (MODE == MODE_ACCOUNT) atomicAdd(&a.result[2], (unsigned long long)bytes);
        if (a.busy) {
            atomicAdd(&a.busy[0], (unsigned long long)(wall_clock64() - t_begin));
            atomicAdd(&a.busy[1], 1ull);
            atomicMax(&a.busy[2], (unsigned long long)cm);
        }
    }
}

}  // namespace gpcount
