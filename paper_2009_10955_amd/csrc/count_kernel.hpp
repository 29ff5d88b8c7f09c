// Persistent counting kernel for gfx950.
//
// What it computes: the number of embeddings of a pattern under one
// configuration (schedule + restriction closure), i.e. the nested-loop search
// of Section II-B / IV-B with candidate sets formed by intersecting sorted
// neighbor lists and cut by the restrictions (the generated code of Fig.
// pseudocode_performance), with every level's injectivity enforced
// (Section II-A requires a bijection). Optionally the innermost 2 to 4
// pairwise non-adjacent levels are not enumerated but counted by
// inclusion-exclusion (Section IV-D, Algorithm 2).
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
//     HBM; they are written and re-read while hot in L2. (A variant with the
//     buffers in LDS was measured slower and turned every buffer access into
//     a flat access; it is not kept.)
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
//   * Counts: a 64-bit total and a carry count per lane, an exact 128-bit
//     wavefront sum, one pair of atomics per wavefront into a 128-bit device
//     total; a last step divides it by the IEP over-count and flags a
//     quotient that does not fit in 64 bits.
//   * Byte accounting (MODE_ACCOUNT) is the same search, leaf mode and memo
//     with a per-lane byte counter added where memory is touched: it measures
//     the bytes of the path the timed launch takes.
#pragma once
#include <hip/hip_runtime.h>

#include <utility>

#include "internal.hpp"
#include "sets.hpp"

namespace gpcount {

using namespace gpdev;

constexpr int kBlock = 256;

// Kernel modes: plain count, per-root counts, or accounting of the bytes the
// search reads and writes (never timed).
enum { MODE_PLAIN = 0, MODE_PER_ROOT = 1, MODE_ACCOUNT = 2 };

// Inclusion-exclusion over at most this many innermost levels.
constexpr int kIepMaxN = GP_IEP_MAX_INNER;

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
    // {task cursor, high word of the 128-bit total, then with xcd_block > 0
    // one task cursor per XCD}
    unsigned long long* queue;
    unsigned long long* result;    // {count (low word), flags, bytes}
    unsigned long long* per_root;  // optional, indexed by CSR entry of (v0, v1)
    // optional {sum over wavefronts of active clock ticks, wavefronts, longest
    // chunk of tasks in ticks}: the balanced run time of a sample and its tail
    unsigned long long* busy;
    // with busy: stop taking tasks once a wavefront has run this many clock
    // ticks (0: no limit); the count is then incomplete and flagged (bit 2)
    uint64_t budget_ticks;
    // optional (leaf mode 4, plans the host found eligible): per group,
    // n_hubs words {root tag, |N(x) & pre & cut|} for hub candidates x
    // or (IEP plans the host found eligible) one table for the launch of
    // n_hubs << memo_ways_log2 words {a + 1 with the high bit set, |N(a) & N(x)|}
    unsigned long long* memo;
    int32_t chunk;
    int32_t memo_ways_log2;
    // > 0: the task space is dealt to the XCDs in blocks of xcd_block tasks
    // (a multiple of chunk): block b goes to XCD b mod kXcds, each XCD takes
    // its blocks in order from its own cursor and then helps the others; 0:
    // one cursor for the device
    int64_t xcd_block;
};

typedef void (*KernelFn)(GpPlanDesc, CountArgs);

// Batched launch: one entry per plan. Each plan has its own launch shape
// (lanes per group, leaf mode, tasks per grab) and its own task cursor.
constexpr int kBatchMaxPlans = 64;

struct BatchPlan {
    const int2* roots;    // this plan's whole root array (cut already applied)
    int64_t root_offset;  // sampled roots: roots[root_offset + r * root_stride]
    int64_t root_stride;
    int64_t n_tasks;      // tasks of this plan in the launch
    int64_t task_offset;  // where in the plan's own task space the launch starts
    int64_t split_roots;  // as in CountArgs: the first split_roots roots run as
    int32_t split_ways;   // split_ways tasks each
    int32_t group;        // lanes per group: 64, 32 or 16
    int32_t leaf;         // 1, 3 or 4
    int32_t chunk;        // tasks per group per grab
    uint32_t tag_base;    // leaf-4 memo tags are tag_base + root + 1; 0: no memo
    int32_t pad;
};


// The descriptors and task ranges of one batched launch's plans, in the order
// waves take them, passed by value: kernel arguments live in constant memory,
// so every field is a scalar load, where a table read from global memory costs
// a vector load and registers at every use.
constexpr int kRunMaxPlans = 8;
struct RunDescs {
    GpPlanDesc d[kRunMaxPlans];
    BatchPlan bp[kRunMaxPlans];
};

struct BatchArgs {
    const int64_t* row_ptr;
    const int32_t* col;
    int32_t np;
    const uint32_t* hub_bits;
    int64_t hub_words;
    int32_t n_hubs;
    int32_t* scratch;        // per wavefront: slots_per_wave groups x nbuf slots x buf_cap
    int64_t buf_cap;
    int32_t nbuf;            // buffer slots per group (max over plans)
    int32_t slots_per_wave;  // 64 / (the smallest group of any plan)
    unsigned long long* memo;     // per wavefront: slots_per_wave x n_hubs words (or null)
    unsigned long long* queues;   // np task cursors
    unsigned long long* result;   // per plan {count low word, flags, busy clock ticks, high word}
};

typedef void (*BatchFn)(BatchArgs, RunDescs);

// Where a group's root tasks come from.
struct TaskSpace {
    const int2* roots;
    int64_t offset, stride;  // root r is roots[offset + r * stride]
    int64_t split_roots;     // task -> root as in CountArgs
    int32_t split_ways;
    uint32_t tag_base;       // memo tag of root r: tag_base + r + 1
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
    uint64_t* bytes;  // accounting mode: per-lane bytes
    const uint32_t* hub_bits;
    int64_t hub_words;
    int32_t n_hubs;
    int32_t sj, sJ;     // level-2 slice of the current task: candidates sj, sj + sJ, ...
    uint64_t deadline;  // clock tick after which every search loop stops (0: none)
    unsigned long long* memo;  // this group's last-level memo, or the launch's IEP memo (null: none)
    uint32_t tag;              // memo validity tag of the current root
    int32_t memo_log2;         // IEP memo: log2 of its words per hub
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

// acc += c, counting wrap-arounds of the low word in carry: (carry, acc) is
// the lane's exact 128-bit total.
__device__ __forceinline__ void add_count(uint64_t& acc, uint64_t c, uint64_t& carry) {
    const uint64_t s = acc + c;
    carry += (s < acc) ? 1u : 0u;
    acc = s;
}

// (carry, acc) += (hi, lo).
__device__ __forceinline__ void add_count128(uint64_t& acc, uint64_t& carry, uint64_t lo, uint64_t hi) {
    const uint64_t s = acc + lo;
    carry += hi + ((s < acc) ? 1u : 0u);
    acc = s;
}

// Wavefront sum of the lanes' 128-bit totals (hi, lo); every lane gets it.
__device__ __forceinline__ void wave_sum128(uint64_t& lo, uint64_t& hi) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint64_t tlo = __shfl_xor(lo, off, 64);
        const uint64_t thi = __shfl_xor(hi, off, 64);
        const uint64_t u = lo + tlo;
        hi += thi + (u < lo ? 1u : 0u);
        lo = u;
    }
}

// Add a 128-bit value to a device-wide total held as two words: the low word
// at *lo_word, the high word at *hi_word. Called by one lane.
__device__ __forceinline__ void publish128(unsigned long long* lo_word, unsigned long long* hi_word, uint64_t lo,
                                           uint64_t hi) {
    if (lo) {
        const unsigned long long old = atomicAdd(lo_word, (unsigned long long)lo);
        hi += (old + lo < old) ? 1u : 0u;
    }
    if (hi) atomicAdd(hi_word, (unsigned long long)hi);
}

// The end of every count: the 128-bit total (hi, *lo_word) divided by div
// (the IEP over-count, 1 otherwise). *lo_word receives the quotient's low 64
// bits; flags: bit 0 if the quotient does not fit in 64 bits, bit 1 if div
// does not divide the total (an internal error). Shift-and-subtract long
// division by one lane: it runs once per count.
__device__ __forceinline__ void finish128(unsigned long long* lo_word, unsigned long long* flags, uint64_t hi,
                                          uint64_t div) {
    const uint64_t lo = *lo_word;
    if (div <= 1) {
        if (hi) *flags |= 1ull;
        return;
    }
    uint64_t qhi = 0, qlo = 0, r = 0;
    for (int i = 127; i >= 0; --i) {
        const uint64_t bit = i >= 64 ? (hi >> (i - 64)) & 1u : (lo >> i) & 1u;
        const bool top = (r >> 63) != 0;  // r < div < 2^64, so 2r + bit may need 65 bits
        r = (r << 1) | bit;
        if (top || r >= div) {
            r -= div;
            if (i >= 64) qhi |= 1ull << (i - 64);
            else qlo |= 1ull << i;
        }
    }
    if (r) *flags |= 2ull;
    if (qhi) *flags |= 1ull;
    *lo_word = qlo;
}

// Bytes read by one binary search in a sorted list of n int32.
__device__ __forceinline__ uint64_t probe_bytes(int32_t n) {
    return 4ull * (uint64_t)(32 - __clz(n > 0 ? n : 1));
}
// Bytes of one membership test in s: a bitmap word, or a binary search.
__device__ __forceinline__ uint64_t test_bytes(const Set& s) {
    return s.bits ? 4ull : probe_bytes(s.n);
}
// Bytes of cutting s to [lo, hi): one binary search per bound applied.
__device__ __forceinline__ uint64_t cut_bytes(const Set& s, int32_t lo, int32_t hi) {
    return probe_bytes(s.n) * (uint64_t)((lo > 0) + (hi < 0x7fffffff));
}
// Bytes of a test-based intersection (group or galloping): every element of
// the smaller operand read and tested in the larger one.
__device__ __forceinline__ uint64_t probe_isect_bytes(Set a, Set b) {
    if (a.n > b.n) {
        const Set t = a;
        a = b;
        b = t;
    }
    return (uint64_t)a.n * (4ull + test_bytes(b));
}
// Bytes of intersect_count_serial: bitmap tests, galloping or a merge.
__device__ __forceinline__ uint64_t serial_isect_bytes(Set a, Set b) {
    if (a.n > b.n) {
        const Set t = a;
        a = b;
        b = t;
    }
    if (a.n == 0) return 0;
    if (b.bits || a.n * 16 < b.n) return probe_isect_bytes(a, b);
    return 4ull * (uint64_t)(a.n + b.n);
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
        uint64_t cb = 0;
        if constexpr (MODE == MODE_ACCOUNT) cb = cut_bytes(A, lo, hi) + cut_bytes(B, lo, hi);
        A = trim_u<G>(A, lo, hi);
        B = trim_u<G>(B, lo, hi);
        int32_t n = uni<G>(intersect_into<G>(c.g, A, B, c.bufs + (int64_t)b.dst * c.cap));
        if constexpr (MODE == MODE_ACCOUNT)
            if (c.g.gl == 0) *c.bytes += cb + probe_isect_bytes(A, B) + 4ull * (uint64_t)n;
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
        if constexpr (MODE == MODE_ACCOUNT) *c.bytes += cut_bytes(S, lo, hi);
        S = trim(S, lo, hi);
        uint32_t cnt = (uint32_t)S.n;
#pragma unroll
        for (int j = 0; j < K - 1; ++j) {
            if ((lv.inj >> j) & 1u) {
                int32_t y = v[j];
                if (y >= lo && y < hi) {
                    if constexpr (MODE == MODE_ACCOUNT) *c.bytes += test_bytes(S);
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
    // a hub operand is tested by bits, so only the other operand is cut; a
    // short list is range-tested element by element instead of cut
    if (B.bits && A.n <= kShortList && A.n * 4 <= B.n) {
        if constexpr (MODE == MODE_ACCOUNT) *c.bytes += 8ull * (uint64_t)A.n;
        return count_bits_range(A, lo, hi, B.bits, skip);
    }
    if (A.bits && B.n <= kShortList && B.n * 4 <= A.n) {
        if constexpr (MODE == MODE_ACCOUNT) *c.bytes += 8ull * (uint64_t)B.n;
        return count_bits_range(B, lo, hi, A.bits, skip);
    }
    if (B.bits) {
        const Set Ac = trim(A, lo, hi);
        if (Ac.n * 4 <= B.n) {
            if constexpr (MODE == MODE_ACCOUNT) *c.bytes += cut_bytes(A, lo, hi) + 8ull * (uint64_t)Ac.n;
            return count_bits(Ac, B.bits, skip);
        }
    } else if (A.bits) {
        const Set Bc = trim(B, lo, hi);
        if (Bc.n * 4 <= A.n) {
            if constexpr (MODE == MODE_ACCOUNT) *c.bytes += cut_bytes(B, lo, hi) + 8ull * (uint64_t)Bc.n;
            return count_bits(Bc, A.bits, skip);
        }
    }
    if constexpr (MODE == MODE_ACCOUNT) *c.bytes += cut_bytes(A, lo, hi) + cut_bytes(B, lo, hi);
    A = trim(A, lo, hi);
    B = trim(B, lo, hi);
    if constexpr (MODE == MODE_ACCOUNT) *c.bytes += serial_isect_bytes(A, B);
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
    uint64_t cb = 0;
    if constexpr (MODE == MODE_ACCOUNT) cb = cut_bytes(A, lo, hi) + cut_bytes(B, lo, hi);
    A = trim_u<G>(A, lo, hi);
    B = trim_u<G>(B, lo, hi);
    if constexpr (MODE == MODE_ACCOUNT)
        if (c.g.gl == 0) *c.bytes += cb + probe_isect_bytes(A, B);
    const uint32_t inj = lv.inj;
    return intersect_count_group<G>(c.g, A, B, [&](int32_t x) { return inj_hit<K>(inj, v, x); });
}

// Counting with inclusion-exclusion over the N innermost levels (Section
// IV-D). For bound values v[0..K-N-1] every inner level j has a candidate set
// S_j: its parents' common neighbors (all parents are outer levels: the inner
// pattern vertices are pairwise non-adjacent), cut by the restrictions to
// outer levels and without the outer images. The number of N-tuples with
// y_j in S_j and all y_j distinct is the inclusion-exclusion sum over the
// "y_a = y_b" conditions; Algorithm 2 evaluates each term as a product over
// the components of the conditions' graph of |intersection of the
// component's sets|. Terms whose graphs have the same components are
// collected here: a partition of the N levels into blocks contributes
// prod over blocks B of (-1)^(|B|-1) (|B|-1)! |∩_{j in B} S_j| (the sum of
// (-1)^edges over the connected graphs on |B| vertices). GRP: computed by the
// whole group (same value in every lane), else by one lane. The value fits
// in 128 bits (each |S_j| < 2^31, N <= 4).
//
// A set S_j is either explicit (one neighbor list, or a buffer built by the
// builds) or, when its last parent is the last outer level, left unbuilt as
// pre & N(x) (pre: a list or buffer; x: that outer vertex), like the last
// level of a plain count. Each |∩ S_j| walks the shortest operand of the
// sets involved, cut to the common range, and tests every element in the
// other operands (a bit in a hub's bitmap, else a binary search).
// The IEP memo: one table per launch, shared by every group, of W = 2^l
// words per hub (l = CountArgs::memo_ways_log2). Word x * W + (a mod W)
// holds |N(a) & N(x)| tagged a. The host takes the most ways, up to
// kIepMemoWaysMax, whose table fits kIepMemoBytes (or the room left).
constexpr int64_t kIepMemoWaysMax = 4096;
constexpr int64_t kIepMemoBytes = int64_t(2) << 30;

constexpr int low_bit(int m) {
    int i = 0;
    while (!((m >> i) & 1)) ++i;
    return i;
}

// |∩_{j in M} S_j| for one subset M of the inner levels (compile-time).
template <int K, int G, int MODE, int N, bool GRP, int M>
__device__ __forceinline__ uint64_t iep_subset_count(const GpPlanDesc& d, const Ctx<G>& c, const int32_t (&v)[K],
                                                     uint64_t& bytes) {
    constexpr int F = K - N;  // first inner level
    // the operands of the sets in M (two per unbuilt set, else one; an absent
    // second operand has p == nullptr) and the common range
    Set X[2 * N];
    int32_t L = 0, H = 0x7fffffff;
    uint32_t im = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        X[2 * j] = Set{nullptr, 0x7fffffff, nullptr};
        X[2 * j + 1] = Set{nullptr, 0x7fffffff, nullptr};
        if (!((M >> j) & 1)) continue;
        const GpLevel& lv = d.lv[F + j];
        int32_t lo, hi;
        bounds<K>(lv.hi_src, lv.lo_src, v, lo, hi);
        L = max(L, lo);
        H = min(H, hi);
        im |= lv.inj;
        if (lv.last_list >= 0) {
            if constexpr (GRP) {
                X[2 * j] = lv.pre_buf >= 0 ? c.buf_u(lv.pre_buf) : c.nbr_u(pick<K>(v, lv.pre_list));
                X[2 * j + 1] = c.nbr_u(pick<K>(v, lv.last_list));
            } else {
                X[2 * j] = lv.pre_buf >= 0 ? c.buf(lv.pre_buf) : c.nbr(pick<K>(v, lv.pre_list));
                X[2 * j + 1] = c.nbr(pick<K>(v, lv.last_list));
            }
        } else {
            if constexpr (GRP) X[2 * j] = lv.list >= 0 ? c.nbr_u(pick<K>(v, lv.list)) : c.buf_u(lv.buf);
            else X[2 * j] = lv.list >= 0 ? c.nbr(pick<K>(v, lv.list)) : c.buf(lv.buf);
        }
    }
    if constexpr (GRP && (M & (M - 1)) == 0) {
        // one unbuilt set N(a) & N(x) with no cut, x a hub: its size is a
        // function of (a, x) alone, the same for every plan, group and launch
        // on the graph. It is kept in the launch's shared memo table, in the
        // word of x chosen by a, tagged a (high bit set, apart from leaf mode
        // 4's root tags). Bindings that share a and x (roots with the same
        // hub endpoint reach the same x through many middle vertices, in
        // every group working on that endpoint) then walk the lists once.
        // Tag and size share one 64-bit word, written and read whole, so a
        // word another group overwrote, or one not yet visible, only ever
        // reads as a miss.
        constexpr int jj = low_bit(M);
        const GpLevel& lv = d.lv[F + jj];
        if (c.memo && lv.last_list >= 0 && lv.pre_buf < 0 && (lv.hi_src | lv.lo_src) == 0) {
            const int32_t xk = pick<K>(v, lv.last_list);
            if (xk < c.n_hubs) {
                const int32_t av = pick<K>(v, lv.pre_list);
                const uint32_t tag = 0x80000000u | (uint32_t)(av + 1);
                const Set A0 = X[2 * jj], A1 = X[2 * jj + 1];
                unsigned long long* const w =
                    c.memo + ((int64_t)xk << c.memo_log2) + (av & ((int32_t(1) << c.memo_log2) - 1));
                const unsigned long long e = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if constexpr (MODE == MODE_ACCOUNT) bytes += 8;
                uint64_t raw;
                if ((uint32_t)(e >> 32) == tag) {
                    raw = (uint32_t)e;
                } else {
                    const Set Wm = A0.n <= A1.n ? A0 : A1, Om = A0.n <= A1.n ? A1 : A0;
                    if constexpr (MODE == MODE_ACCOUNT) bytes += (uint64_t)Wm.n * (4 + test_bytes(Om)) + 8;
                    raw = 0;
                    for (int32_t base = 0; base < Wm.n; base += G) {
                        const int32_t i = base + c.g.gl;
                        const bool ok = i < Wm.n && member(Om, Wm.p[i]);
                        raw += (uint64_t)__popcll(c.g.ballot(ok));
                    }
                    if (c.g.gl == 0)
                        __hip_atomic_store(w, ((unsigned long long)tag << 32) | raw, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
                // outer images in the set (distinct: the binding is injective)
#pragma unroll
                for (int o = 0; o < F; ++o)
                    if ((im >> o) & 1u) {
                        const int32_t y = v[o];
                        if constexpr (MODE == MODE_ACCOUNT) bytes += test_bytes(A0) + test_bytes(A1);
                        if (member(A0, y) && member(A1, y)) --raw;
                    }
                return raw;
            }
        }
    }
    // the shortest operand, cut to [L, H), is walked
    int s = 0;
    int32_t sn = 0x7fffffff;
#pragma unroll
    for (int f = 0; f < 2 * N; ++f)
        if (((M >> (f / 2)) & 1) && X[f].p && X[f].n < sn) {
            sn = X[f].n;
            s = f;
        }
    Set W{nullptr, 0, nullptr};
#pragma unroll
    for (int f = 0; f < 2 * N; ++f)
        if (((M >> (f / 2)) & 1) && f == s) W = X[f];
    if constexpr (MODE == MODE_ACCOUNT) bytes += cut_bytes(W, L, H);
    if constexpr (GRP) W = trim_u<G>(W, L, H);
    else W = trim(W, L, H);
    constexpr bool one = (M & (M - 1)) == 0;
    if (one && X[2 * __builtin_ctz(M) + 1].p == nullptr) {
        // one built set: its size, without the outer images in it
        uint64_t cm = (uint64_t)W.n;
#pragma unroll
        for (int o = 0; o < F; ++o) {
            if ((im >> o) & 1u) {
                const int32_t y = v[o];
                if (y >= L && y < H) {
                    if constexpr (MODE == MODE_ACCOUNT) bytes += test_bytes(W);
                    if (member(W, y)) --cm;
                }
            }
        }
        return cm;
    }
    if constexpr (MODE == MODE_ACCOUNT) {
        uint64_t per = 4;
#pragma unroll
        for (int f = 0; f < 2 * N; ++f)
            if (((M >> (f / 2)) & 1) && X[f].p && f != s) per += test_bytes(X[f]);
        bytes += (uint64_t)W.n * per;
    }
    uint64_t cm = 0;
    const int32_t step = GRP ? G : 1;
    const int32_t first = GRP ? c.g.gl : 0;
    for (int32_t base = 0; base < W.n; base += step) {
        const int32_t i = base + first;
        bool ok = false;
        if (i < W.n) {
            const int32_t x = W.p[i];
            ok = !inj_hit<K>(im, v, x);
#pragma unroll
            for (int f = 0; f < 2 * N; ++f)
                if (((M >> (f / 2)) & 1) && f != s && X[f].p) ok = ok && member(X[f], x);
        }
        if constexpr (GRP) cm += (uint64_t)__popcll(c.g.ballot(ok));
        else cm += ok ? 1u : 0u;
    }
    return cm;
}

template <int K, int G, int MODE, int N, bool GRP, int... Ms>
__device__ __forceinline__ unsigned __int128 iep_combine(const GpPlanDesc& d, const Ctx<G>& c,
                                                         const int32_t (&v)[K], uint64_t& bytes,
                                                         std::integer_sequence<int, Ms...>) {
    // cnt[M] for every nonempty subset M (cnt[0] unused)
    const uint64_t cnt[(1 << N)] = {0, iep_subset_count<K, G, MODE, N, GRP, Ms + 1>(d, c, v, bytes)...};
    typedef unsigned __int128 u128;
    auto P = [&](int a) { return (u128)cnt[a]; };
    if constexpr (N == 2) {
        return P(1) * P(2) - P(3);
    } else if constexpr (N == 3) {
        return P(1) * P(2) * P(4) - P(3) * P(4) - P(5) * P(2) - P(6) * P(1) + 2 * P(7);
    } else {
        // blocks: singles 1 2 4 8; pairs 3 5 9 6 10 12; triples 7 11 13 14; all 15
        return P(1) * P(2) * P(4) * P(8) -
               (P(3) * P(4) * P(8) + P(5) * P(2) * P(8) + P(9) * P(2) * P(4) + P(6) * P(1) * P(8) +
                P(10) * P(1) * P(4) + P(12) * P(1) * P(2)) +
               (P(3) * P(12) + P(5) * P(10) + P(9) * P(6)) +
               2 * (P(7) * P(8) + P(11) * P(4) + P(13) * P(2) + P(14) * P(1)) - 6 * P(15);
    }
}

template <int K, int G, int MODE, int N, bool GRP>
__device__ __forceinline__ unsigned __int128 iep_value(const GpPlanDesc& d, const Ctx<G>& c,
                                                       const int32_t (&v)[K]) {
    static_assert(N >= 2 && N <= kIepMaxN && N <= K - 2, "IEP inner levels");
    uint64_t bytes = 0;
    const unsigned __int128 r =
        iep_combine<K, G, MODE, N, GRP>(d, c, v, bytes, std::make_integer_sequence<int, (1 << N) - 1>{});
    if constexpr (MODE == MODE_ACCOUNT) {
        if constexpr (GRP) {
            if (c.g.gl == 0) *c.bytes += bytes;
        } else {
            *c.bytes += bytes;
        }
    }
    return r;
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
                          int32_t st, uint32_t inj_l, uint64_t& acc, uint64_t& carry) {
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
                if constexpr (MODE == MODE_ACCOUNT) *c.bytes += cut_bytes(C, lo, hi);
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
                    add_count(acc, leaf_serial<K, G, MODE>(d, c, w), carry);
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
                               uint32_t inj_l, uint64_t& acc, uint64_t& carry) {
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
                            if (y >= lo && y < hi) {
                                if constexpr (MODE == MODE_ACCOUNT) *c.bytes += 4;
                                corr += ((bits[y >> 5] >> (y & 31)) & 1u) ? 1u : 0u;
                            }
                        }
                    const unsigned long long e = c.memo[x];
                    if constexpr (MODE == MODE_ACCOUNT) *c.bytes += 8;
                    if ((uint32_t)(e >> 32) == c.tag) {
                        add_count(acc, (uint32_t)e - corr, carry);
                    } else {
                        const Set Bn = c.nbr(x);
                        if constexpr (MODE == MODE_ACCOUNT) *c.bytes += cut_bytes(Bn, lo, hi);
                        B = trim(Bn, lo, hi);
                        if (B.n <= kCoopList) {
                            const uint32_t all = count_bits(B, bits, [](int32_t) { return false; });
                            c.memo[x] = ((unsigned long long)c.tag << 32) | all;
                            if constexpr (MODE == MODE_ACCOUNT) *c.bytes += 8ull * (uint64_t)B.n + 8;
                            add_count(acc, all - corr, carry);
                        } else {
                            longl = true;
                        }
                    }
                } else {
                    B = c.nbr(x);
                    if (B.n <= kShortList) {
                        if constexpr (MODE == MODE_ACCOUNT) *c.bytes += 8ull * (uint64_t)B.n;
                        add_count(acc, count_bits_range(B, lo, hi, bits, skip), carry);
                    } else {
                        if constexpr (MODE == MODE_ACCOUNT) *c.bytes += cut_bytes(B, lo, hi);
                        B = trim(B, lo, hi);
                        if (B.n <= kCoopList) {
                            if constexpr (MODE == MODE_ACCOUNT) *c.bytes += 8ull * (uint64_t)B.n;
                            add_count(acc, count_bits(B, bits, skip), carry);
                        } else {
                            longl = true;
                        }
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
            if constexpr (MODE == MODE_ACCOUNT)
                if (c.g.gl == 0) *c.bytes += 8ull * (uint64_t)on;
            add_count(acc, cnt, carry);
            if (c.memo && ox < c.n_hubs) {
                // the long list of a hub candidate: keep its whole count
                const uint32_t tot = (uint32_t)c.g.sum(all);
                if (c.g.gl == 0) {
                    c.memo[ox] = ((unsigned long long)c.tag << 32) | tot;
                    if constexpr (MODE == MODE_ACCOUNT) *c.bytes += 8;
                }
            }
        }
    }
    return true;
}

// The IEP leaf at the last outer level L (inner levels L+1 .. K-1): every
// candidate x of level L adds its inclusion-exclusion value. Lanes take
// different candidates when no build runs after level L is bound; otherwise
// the group binds one candidate at a time, runs the builds and computes the
// value together.
// A lane's walk for the IEP value of its own binding: the longest of its
// unbuilt inner sets' shorter operands (the single-set counts walk them; the
// intersections walk no more). Lanes whose walk exceeds kIepLaneWork leave
// their binding to the whole group (iep_group_pass), so one hub binding does
// not hold a wavefront's other lanes idle for thousands of steps.
constexpr int32_t kIepLaneWork = 128;

template <int K, int N, int G>
__device__ __forceinline__ int64_t iep_lane_work_g(const GpPlanDesc& d, const Ctx<G>& c, const int32_t (&w)[K]) {
    constexpr int F = K - N;
    int64_t work = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const GpLevel& lv = d.lv[F + j];
        if (lv.last_list < 0) continue;
        const int32_t a = pick<K>(w, lv.last_list);
        const int64_t na = c.row_ptr[a + 1] - c.row_ptr[a];
        int64_t np;
        if (lv.pre_buf >= 0) {
            np = c.lens[lv.pre_buf];
        } else {
            const int32_t b = pick<K>(w, lv.pre_list);
            np = c.row_ptr[b + 1] - c.row_ptr[b];
        }
        work = max(work, min(na, np));
    }
    return work;
}

// The bindings of the lanes flagged in `m` (a group ballot; x is each lane's
// level-L vertex), one at a time, each by the whole group.
template <int K, int L, int G, int MODE>
__device__ __forceinline__ void iep_group_pass(const GpPlanDesc& d, const Ctx<G>& c, const int32_t (&v)[K],
                                               uint64_t m, int32_t x, uint64_t& acc, uint64_t& carry) {
    constexpr int N = K - 1 - L;
    while (m) {
        const int src = __builtin_ctzll(m);
        m &= m - 1;
        int32_t w[K];
#pragma unroll
        for (int j = 0; j < K; ++j) w[j] = v[j];
        w[L] = uni<G>(c.g.bcast(x, src));
        const unsigned __int128 val = iep_value<K, G, MODE, N, true>(d, c, w);
        if (c.g.gl == 0) add_count128(acc, carry, (uint64_t)val, (uint64_t)(val >> 64));
    }
}

template <int K, int L, int G, int MODE>
__device__ void iep_level(const GpPlanDesc& d, const Ctx<G>& c, int32_t (&v)[K], Set S, int32_t st,
                          uint32_t inj_l, uint64_t& acc, uint64_t& carry) {
    constexpr int N = K - 1 - L;
    if (d.build_begin[L] == d.build_end[L]) {
        for (int32_t base = 0; base < S.n; base += G) {
            if (c.expired()) break;
            const int32_t i = base + c.g.gl;
            int32_t x = 0;
            bool longw = false;
            if (i < S.n) {
                x = S.p[(int64_t)i * st];
                if (!inj_hit<K>(inj_l, v, x)) {
                    int32_t w[K];
#pragma unroll
                    for (int j = 0; j < K; ++j) w[j] = v[j];
                    w[L] = x;
                    if (iep_lane_work_g<K, N, G>(d, c, w) > kIepLaneWork) {
                        longw = true;
                    } else {
                        const unsigned __int128 val = iep_value<K, G, MODE, N, false>(d, c, w);
                        add_count128(acc, carry, (uint64_t)val, (uint64_t)(val >> 64));
                    }
                }
            }
            iep_group_pass<K, L, G, MODE>(d, c, v, c.g.ballot(longw), x, acc, carry);
        }
    } else {
        for (int32_t t = 0; t < S.n; ++t) {
            if (c.expired()) break;
            const int32_t x = uni<G>(S.p[(int64_t)t * st]);
            if (inj_hit<K>(inj_l, v, x)) continue;
            v[L] = x;
            run_builds<K, G, MODE>(d, c, L, v);
            const unsigned __int128 val = iep_value<K, G, MODE, N, true>(d, c, v);
            if (c.g.gl == 0) add_count128(acc, carry, (uint64_t)val, (uint64_t)(val >> 64));
        }
    }
}

// IEP: 0 (plain), else the number of inner levels counted with
// inclusion-exclusion (a kernel is built per depth, so each carries only the
// registers of its own depth).
template <int K, int L, int G, int LEAF, int MODE, int IEP>
__device__ void search(const GpPlanDesc& d, const Ctx<G>& c, int32_t (&v)[K], uint64_t& acc,
                       uint64_t& carry) {
    if constexpr (IEP > 0 && L > K - 1 - IEP) {
        return;  // an IEP search ends at its last outer level
    } else {
        const GpLevel& lv = d.lv[L];
        int32_t lo, hi;
        bounds<K>(lv.hi_src, lv.lo_src, v, lo, hi);
        Set S = lv.list >= 0 ? c.nbr_u(pick<K>(v, lv.list)) : c.buf_u(lv.buf);
        if constexpr (MODE == MODE_ACCOUNT)
            if (c.g.gl == 0) *c.bytes += cut_bytes(S, lo, hi);
        S = trim_u<G>(S, lo, hi);
        // a split task binds only its slice of the level-2 candidates
        int32_t st = 1;
        if constexpr (L == 2) {
            if (c.sJ > 1) {
                S.n = S.n > c.sj ? (S.n - c.sj + c.sJ - 1) / c.sJ : 0;
                S.p += c.sj;
                st = c.sJ;
            }
        }
        if constexpr (MODE == MODE_ACCOUNT)
            if (c.g.gl == 0) *c.bytes += 4ull * (uint64_t)S.n;
        if constexpr (IEP > 0 && L == K - 1 - IEP) {
            // the last outer level: the inner ones are counted, not enumerated
            iep_level<K, L, G, MODE>(d, c, v, S, st, lv.inj, acc, carry);
            return;
        }
        if constexpr (L == K - 2) {
            if constexpr (LEAF == 4)
                if (coop_bits_leaf<K, G, MODE>(d, c, v, S, st, lv.inj, acc, carry)) return;
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
                            add_count(acc, leaf_serial<K, G, MODE>(d, c, w), carry);
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
                    if (c.g.gl == 0) add_count(acc, cnt, carry);
                }
            }
        } else {
            if constexpr (LEAF == 3 && L == K - 3 && IEP == 0) {
                if (d.build_begin[L] == d.build_end[L]) {
                    flat_leaf<K, G, MODE>(d, c, v, S, st, lv.inj, acc, carry);
                    return;
                }
            }
            for (int32_t t = 0; t < S.n; ++t) {
                if (c.expired()) break;
                const int32_t x = uni<G>(S.p[(int64_t)t * st]);
                if (inj_hit<K>(lv.inj, v, x)) continue;
                v[L] = x;
                run_builds<K, G, MODE>(d, c, L, v);
                search<K, L + 1, G, LEAF, MODE, IEP>(d, c, v, acc, carry);
            }
        }
    }
}

__device__ __forceinline__ int64_t entry_index(const int64_t* row_ptr, const int32_t* col,
                                               int32_t v0, int32_t v1) {
    int64_t b = row_ptr[v0];
    return b + lower_bound(col + b, (int32_t)(row_ptr[v0 + 1] - b), v1);
}

// One group's root tasks [t0, t1) of task space ts: every task binds its root
// edge (levels 0 and 1) and searches the rest. Patterns whose search ends at
// the root (k <= 3, or IEP over all k-2 levels after it) take different roots
// in different lanes. per_root (MODE_PER_ROOT): each root's count at the CSR
// entry of the root edge.
template <int K, int G, int LEAF, int MODE, int IEP>
__device__ __forceinline__ void run_tasks(const GpPlanDesc& d, Ctx<G>& c, const TaskSpace& ts, int64_t t0,
                                          int64_t t1, uint64_t& acc, uint64_t& carry,
                                          unsigned long long* per_root) {
    constexpr bool PER_ROOT = MODE == MODE_PER_ROOT;
    if constexpr (IEP > 0 && IEP == K - 2) {
        {
            // the root is the last outer level
            if (d.build_begin[1] == d.build_end[1]) {
                for (int64_t base = t0; base < t1; base += G) {
                    const int64_t r = base + c.g.gl;
                    int2 e = make_int2(0, 0);
                    bool longw = false;
                    if (r < t1) {
                        e = ts.roots[ts.offset + r * ts.stride];
                        if constexpr (MODE == MODE_ACCOUNT) *c.bytes += 8;
                        int32_t w[K];
#pragma unroll
                        for (int j = 0; j < K; ++j) w[j] = 0;
                        w[0] = e.x;
                        w[1] = e.y;
                        if (iep_lane_work_g<K, K - 2, G>(d, c, w) > kIepLaneWork) {
                            longw = true;
                        } else {
                            const unsigned __int128 val = iep_value<K, G, MODE, K - 2, false>(d, c, w);
                            add_count128(acc, carry, (uint64_t)val, (uint64_t)(val >> 64));
                            if constexpr (PER_ROOT)
                                per_root[entry_index(c.row_ptr, c.col, e.x, e.y)] = (unsigned long long)val;
                        }
                    }
                    // roots with long inner walks: the whole group, one at a time
                    uint64_t m = c.g.ballot(longw);
                    while (m) {
                        const int src = __builtin_ctzll(m);
                        m &= m - 1;
                        int32_t w[K];
#pragma unroll
                        for (int j = 0; j < K; ++j) w[j] = 0;
                        w[0] = uni<G>(c.g.bcast(e.x, src));
                        w[1] = uni<G>(c.g.bcast(e.y, src));
                        const unsigned __int128 val = iep_value<K, G, MODE, K - 2, true>(d, c, w);
                        if (c.g.gl == 0) {
                            add_count128(acc, carry, (uint64_t)val, (uint64_t)(val >> 64));
                            if constexpr (PER_ROOT)
                                per_root[entry_index(c.row_ptr, c.col, w[0], w[1])] = (unsigned long long)val;
                        }
                    }
                }
            } else {
                for (int64_t r = t0; r < t1; ++r) {
                    int2 e = ts.roots[ts.offset + r * ts.stride];
                    e.x = uni<G>(e.x);
                    e.y = uni<G>(e.y);
                    if constexpr (MODE == MODE_ACCOUNT)
                        if (c.g.gl == 0) *c.bytes += 8;
                    int32_t v[K];
#pragma unroll
                    for (int j = 0; j < K; ++j) v[j] = 0;
                    v[0] = e.x;
                    v[1] = e.y;
                    run_builds<K, G, MODE>(d, c, 1, v);
                    const unsigned __int128 val = iep_value<K, G, MODE, K - 2, true>(d, c, v);
                    if (c.g.gl == 0) {
                        add_count128(acc, carry, (uint64_t)val, (uint64_t)(val >> 64));
                        if constexpr (PER_ROOT)
                            per_root[entry_index(c.row_ptr, c.col, e.x, e.y)] = (unsigned long long)val;
                    }
                }
            }
            return;
        }
    }
    if constexpr (K <= 3 && LEAF != 2) {
        // lanes take different roots
        for (int64_t base = t0; base < t1; base += G) {
            int64_t r = base + c.g.gl;
            if (r < t1) {
                int2 e = ts.roots[ts.offset + r * ts.stride];
                uint64_t cnt = 1;
                if constexpr (MODE == MODE_ACCOUNT) *c.bytes += 8;
                if constexpr (K == 3) {
                    int32_t w[K] = {e.x, e.y, 0};
                    cnt = leaf_serial<K, G, MODE>(d, c, w);
                }
                add_count(acc, cnt, carry);
                if constexpr (PER_ROOT) per_root[entry_index(c.row_ptr, c.col, e.x, e.y)] = cnt;
            }
        }
    } else {
        for (int64_t t = t0; t < t1; ++t) {
            const int64_t r = task_root(t, ts.split_roots, ts.split_ways, c.sj, c.sJ);
            c.tag = ts.tag_base + (uint32_t)(r + 1);
            int2 e = ts.roots[ts.offset + r * ts.stride];
            e.x = uni<G>(e.x);
            e.y = uni<G>(e.y);
            const uint64_t before = acc;
            if constexpr (MODE == MODE_ACCOUNT)
                if (c.g.gl == 0) *c.bytes += 8;
            if constexpr (K <= 3) {
                uint64_t cnt = 1;
                if constexpr (K == 3) {
                    int32_t w[K] = {e.x, e.y, 0};
                    cnt = leaf_group<K, G, MODE>(d, c, w);
                }
                if (c.g.gl == 0) add_count(acc, cnt, carry);
            } else {
                int32_t v[K];
#pragma unroll
                for (int j = 0; j < K; ++j) v[j] = 0;
                v[0] = e.x;
                v[1] = e.y;
                run_builds<K, G, MODE>(d, c, 1, v);
                search<K, 2, G, LEAF, MODE, IEP>(d, c, v, acc, carry);
            }
            if constexpr (PER_ROOT) {
                uint64_t mine = c.g.sum(acc - before);
                if (c.g.gl == 0) per_root[entry_index(c.row_ptr, c.col, e.x, e.y)] = mine;
            }
        }
    }
}

// Wavefronts per SIMD the compiler is asked to keep resident (it trims
// registers, spilling a few if it must). The searches are bound by the
// latency of scattered loads, so more resident wavefronts pay even against
// some spills. Measured on R-MAT 17 for k = 5 (64-lane groups with lanes on
// separate candidates: 8, others 6) and on Chung-Lu 7000 for k = 6 (64-lane
// groups 6, others 5); k >= 7 keeps the compiler's choice. IEP over 3 or 4
// inner levels keeps 7 or 15 set sizes and their 128-bit products live: 5
// and 4 wavefronts.
// XCDs of the device; workgroups are dealt to them round robin in launch
// order, so block b of a grid runs on XCD b mod kXcds.
constexpr int kXcds = 8;
// Words of a launch's queue: cursor, high count word, one cursor per XCD.
constexpr int kQueueWords = 2 + kXcds;

// Tasks of XCD x when n tasks are dealt in blocks of B tasks, block b to
// XCD b mod kXcds.
__device__ __forceinline__ int64_t xcd_tasks(int64_t n, int64_t B, int x) {
    const int64_t round = (int64_t)kXcds * B;
    const int64_t full = n / round, rem = n - full * round;
    return full * B + min(max(rem - (int64_t)x * B, (int64_t)0), B);
}

// Global task of XCD x's j-th task.
__device__ __forceinline__ int64_t xcd_task(int64_t j, int64_t B, int x) {
    const int64_t b = j / B;
    return (b * kXcds + x) * B + (j - b * B);
}

// Next grab of a group: `chunk` tasks [*t0, *t1) from one cursor, or false
// once every cursor is exhausted. With XCD blocks the group starts at its
// own XCD's cursor (*q = 0) and moves on to the next XCD's when it runs dry;
// it never comes back to one that was dry.
template <int G>
__device__ __forceinline__ bool grab_tasks(const Group<G>& grp, unsigned long long* queue, int64_t n_tasks,
                                           int64_t chunk, int64_t xcd_block, int* q, int64_t* t0, int64_t* t1) {
    if (xcd_block <= 0) {
        unsigned long long v = 0;
        if (grp.gl == 0) v = atomicAdd(queue, (unsigned long long)chunk);
        const int64_t a = uni64<G>((int64_t)grp.bcast(v, 0));
        if (a >= n_tasks) return false;
        *t0 = a;
        *t1 = min(a + chunk, n_tasks);
        return true;
    }
    const int home = (int)(blockIdx.x % kXcds);
    while (*q < kXcds) {
        const int x = (home + *q) % kXcds;
        const int64_t nx = xcd_tasks(n_tasks, xcd_block, x);
        unsigned long long v = 0;
        if (grp.gl == 0) v = atomicAdd(&queue[2 + x], (unsigned long long)chunk);
        const int64_t j = uni64<G>((int64_t)grp.bcast(v, 0));
        if (j < nx) {
            *t0 = xcd_task(j, xcd_block, x);
            *t1 = *t0 + min(chunk, nx - j);
            return true;
        }
        ++*q;
    }
    return false;
}

constexpr int occupancy_target(int K, int G, int LEAF, int IEP = 0) {
    return IEP >= 3 ? (IEP == 3 ? 5 : 4)
           : K > 6  ? 1
           : K == 6 ? (G == 64 ? 6 : 5)
                    : (G == 64 && (LEAF == 1 || LEAF == 4) ? 8 : 6);
}

template <int K, int G, int LEAF, int MODE, int IEP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(occupancy_target(K, G, LEAF, IEP)))) void count_kernel(GpPlanDesc d, CountArgs a) {
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
    // leaf mode 4: a table per group; IEP: one table for the launch
    c.memo = a.memo ? (IEP > 0 ? a.memo : a.memo + group_id * (int64_t)a.n_hubs) : nullptr;
    c.tag = 0;
    c.memo_log2 = a.memo_ways_log2;
    const uint64_t t_begin = a.busy ? wall_clock64() : 0;
    c.deadline = a.busy && a.budget_ticks ? t_begin + a.budget_ticks : 0;
    uint64_t chunk_max = 0;
    bool stopped = false;
    TaskSpace ts;
    ts.roots = a.roots;
    ts.offset = a.root_offset;
    ts.stride = a.root_stride;
    ts.split_roots = a.split_roots;
    ts.split_ways = a.split_ways;
    ts.tag_base = 0;

    uint64_t acc = 0, carry = 0;
    const int64_t chunk = a.chunk;

    int q = 0;
    for (;;) {
        int64_t t0 = 0, t1 = 0;
        if (!grab_tasks<G>(c.g, a.queue, a.n_tasks, chunk, a.xcd_block, &q, &t0, &t1)) break;
        const uint64_t t_chunk = a.busy ? wall_clock64() : 0;
        run_tasks<K, G, LEAF, MODE, IEP>(d, c, ts, t0, t1, acc, carry, a.per_root);
        if (a.busy) {
            const uint64_t now = wall_clock64();
            chunk_max = max(chunk_max, now - t_chunk);
            if (c.deadline && now > c.deadline) {
                stopped = true;
                break;
            }
        }
    }

    // exact 128-bit wavefront sum, one pair of atomics per wavefront
    uint64_t s = acc, s_hi = carry;
    wave_sum128(s, s_hi);
    if constexpr (MODE == MODE_ACCOUNT) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) bytes += __shfl_xor(bytes, off, 64);
    }
    uint64_t cm = chunk_max;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) cm = max(cm, (uint64_t)__shfl_xor(cm, off, 64));
    const bool any_stop = __ballot(stopped) != 0;
    if (__lane_id() == 0) {
        publish128(&a.result[0], &a.queue[1], s, s_hi);
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
