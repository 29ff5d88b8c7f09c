// Embedding listing for gfx950: the search of the counting kernel with the
// last level enumerated instead of counted. Section II-A states the problem
// as finding every subgraph that is an image of the pattern; the count is the
// number of these. With the restriction closure in force each distinct
// subgraph is reached by exactly one map (Section IV-A), so every map the
// search completes is written out once.
//
// How it maps to the machine:
//   * the task queue, root arrays, candidate sets, intersections ("tmp"
//     buffers built by the same schedule of builds) and restriction cuts are
//     those of the counting kernel;
//   * one 64-lane group walks one search path; the levels above the
//     second-to-last bind one candidate at a time, then the lanes take
//     different second-to-last candidates and walk their last levels (k = 3:
//     the group tests the last level 64 candidates at once);
//   * two passes of the same search: the first stores how many embeddings
//     each root task has, an exclusive scan turns these into row offsets, and
//     the second writes each task's rows from its offset on, the lanes
//     stepping through their last levels in lockstep. The lanes that hold an
//     embedding at a step are compacted with a ballot into a stage of rows in
//     LDS, which goes out in contiguous blocks (coalesced stores); the group
//     keeps its running row in a scalar register: no atomics on the output,
//     and the rows come out in a fixed order (root task, then search order);
//   * a row holds the original vertex ids, indexed by pattern vertex.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "count_kernel.hpp"

namespace gplist {

using namespace gpdev;
using gpcount::kBlock;

constexpr int G = 64;

struct ListArgs {
    const int64_t* row_ptr;
    const int32_t* col;
    const int2* roots;
    int64_t n_roots;  // roots[root_offset + r * root_stride], r < n_roots
    int64_t root_offset;
    int64_t root_stride;
    const uint32_t* hub_bits;
    int64_t hub_words;
    int32_t n_hubs;
    int32_t* scratch;
    int64_t buf_cap;
    unsigned long long* queue;
    // count pass: embeddings of root task t; write pass: its first row
    unsigned long long* task_rows;
    int32_t* out;               // out_cap rows of k int32
    int64_t out_cap;
    const int32_t* orig;        // layout id -> original id
    int32_t col_of[GP_DESC_MAX_K];  // output column (pattern vertex) of schedule level i
    int32_t chunk;
};

// Rows of the write pass are staged in LDS and stored in contiguous runs:
// a group's rows of one root task are consecutive in the output, so kStage
// rows at a time go out as one block, lane i storing words i, i + G, ...
// (coalesced) instead of each lane storing its own row of K words at a
// K-word stride.
constexpr int kStage = 128;

struct Stage {
    int32_t* rows;  // LDS: kStage rows of K int32, in output column order
    uint64_t base;  // output row of staged row 0
    int32_t n;      // rows staged
};

template <int K>
__device__ __forceinline__ void flush(const Group<G>& g, const ListArgs& a, Stage& st) {
    gpcount::group_fence();
    const int64_t words = (int64_t)st.n * K;
    int32_t* o = a.out + (int64_t)st.base * K;
    for (int64_t i = g.gl; i < words; i += G)
        if (st.base + (uint64_t)(i / K) < (uint64_t)a.out_cap) o[i] = st.rows[i];
    gpcount::group_fence();
    st.base += (uint64_t)st.n;
    st.n = 0;
}

// Lanes whose `ok` is set hold an embedding: w[0..K-2] bound and x at the
// last level. The write pass places them as rows pos, pos + 1, ... in lane
// order (through the stage); both passes advance pos (group-uniform).
template <int K, bool WRITE>
__device__ __forceinline__ void emit(const Group<G>& g, const ListArgs& a, const int32_t (&w)[K], bool ok,
                                     int32_t x, uint64_t& pos, Stage& st) {
    const uint64_t m = g.ballot(ok);
    const int32_t cnt = (int32_t)__popcll(m);
    if constexpr (WRITE) {
        if (st.n + cnt > kStage) flush<K>(g, a, st);
        if (ok) {
            int32_t* r = st.rows + (int64_t)(st.n + (int32_t)g.below_mask_count(m)) * K;
#pragma unroll
            for (int j = 0; j < K - 1; ++j) r[a.col_of[j]] = a.orig[w[j]];
            r[a.col_of[K - 1]] = a.orig[x];
        }
        st.n += cnt;
    }
    pos += (uint64_t)cnt;
}

// Last level for bound v[0..K-2]: its candidate set is one list or buffer, or
// the intersection of a prefix set with the list of the level before it; cut
// to the restriction bounds, earlier images excluded.
template <int K, bool WRITE>
__device__ void list_last(const GpPlanDesc& d, const gpcount::Ctx<G>& c, const ListArgs& a,
                          const int32_t (&v)[K], uint64_t& pos, Stage& st) {
    const GpLevel& lv = d.lv[K - 1];
    int32_t lo, hi;
    gpcount::bounds<K>(lv.hi_src, lv.lo_src, v, lo, hi);
    const bool two = lv.last_list >= 0;
    Set S, T{nullptr, 0, nullptr};
    if (!two) {
        S = lv.list >= 0 ? c.nbr_u(gpcount::pick<K>(v, lv.list)) : c.buf_u(lv.buf);
    } else {
        S = lv.pre_buf >= 0 ? c.buf_u(lv.pre_buf) : c.nbr_u(gpcount::pick<K>(v, lv.pre_list));
        T = c.nbr_u(gpcount::pick<K>(v, lv.last_list));
    }
    S = gpcount::trim_u<G>(S, lo, hi);
    if (two) {
        T = gpcount::trim_u<G>(T, lo, hi);
        if (T.n < S.n) {
            const Set t = S;
            S = T;
            T = t;
        }
    }
    for (int32_t base = 0; base < S.n; base += G) {
        const int32_t i = base + c.g.gl;
        bool ok = false;
        int32_t x = 0;
        if (i < S.n) {
            x = S.p[i];
            ok = !gpcount::inj_hit<K>(lv.inj, v, x) && (!two || member(T, x));
        }
        emit<K, WRITE>(c.g, a, v, ok, x, pos, st);
    }
}

// The last level for one lane's own bound values w[0..K-2], by that lane
// alone: the number of embeddings (count pass).
template <int K>
__device__ uint32_t last_count(const GpPlanDesc& d, const gpcount::Ctx<G>& c, const int32_t (&w)[K]) {
    const GpLevel& lv = d.lv[K - 1];
    int32_t lo, hi;
    gpcount::bounds<K>(lv.hi_src, lv.lo_src, w, lo, hi);
    uint32_t n = 0;
    if (lv.last_list < 0) {
        const Set S = trim(lv.list >= 0 ? c.nbr(gpcount::pick<K>(w, lv.list)) : c.buf(lv.buf), lo, hi);
        for (int32_t i = 0; i < S.n; ++i) {
            const int32_t x = S.p[i];
            n += !gpcount::inj_hit<K>(lv.inj, w, x);
        }
    } else {
        Set A = trim(lv.pre_buf >= 0 ? c.buf(lv.pre_buf) : c.nbr(gpcount::pick<K>(w, lv.pre_list)), lo, hi);
        Set B = trim(c.nbr(gpcount::pick<K>(w, lv.last_list)), lo, hi);
        if (A.n > B.n) {
            const Set t = A;
            A = B;
            B = t;
        }
        for (int32_t i = 0; i < A.n; ++i) {
            const int32_t x = A.p[i];
            n += member(B, x) && !gpcount::inj_hit<K>(lv.inj, w, x);
        }
    }
    return n;
}

// Write pass of last_count: every lane walks its own last level one candidate
// per step, and a ballot per step places the step's embeddings at rows pos,
// pos + 1, ... in lane order (one walk, no count first). Lanes without a
// binding (have false) only join the ballots.
template <int K>
__device__ void last_lockstep(const GpPlanDesc& d, const gpcount::Ctx<G>& c, const ListArgs& a,
                              const int32_t (&w)[K], bool have, uint64_t& pos, Stage& st) {
    const GpLevel& lv = d.lv[K - 1];
    int32_t lo, hi;
    gpcount::bounds<K>(lv.hi_src, lv.lo_src, w, lo, hi);
    const bool two = lv.last_list >= 0;
    Set A{nullptr, 0, nullptr}, B{nullptr, 0, nullptr};
    if (have) {
        if (!two) {
            A = trim(lv.list >= 0 ? c.nbr(gpcount::pick<K>(w, lv.list)) : c.buf(lv.buf), lo, hi);
        } else {
            A = trim(lv.pre_buf >= 0 ? c.buf(lv.pre_buf) : c.nbr(gpcount::pick<K>(w, lv.pre_list)), lo, hi);
            B = trim(c.nbr(gpcount::pick<K>(w, lv.last_list)), lo, hi);
            if (A.n > B.n) {
                const Set t = A;
                A = B;
                B = t;
            }
        }
    }
    for (int32_t i = 0; c.g.ballot(i < A.n) != 0; ++i) {
        bool ok = false;
        int32_t x = 0;
        if (i < A.n) {
            x = A.p[i];
            ok = (!two || member(B, x)) && !gpcount::inj_hit<K>(lv.inj, w, x);
        }
        emit<K, true>(c.g, a, w, ok, x, pos, st);
    }
}

template <int K, int L, bool WRITE>
__device__ void list_search(const GpPlanDesc& d, const gpcount::Ctx<G>& c, const ListArgs& a, int32_t (&v)[K],
                            uint64_t& pos, Stage& st) {
    if constexpr (L == K - 1) {
        list_last<K, WRITE>(d, c, a, v, pos, st);
    } else if constexpr (L == K - 2) {
        // lanes take different candidates of the second-to-last level and
        // walk the last level alone
        const GpLevel& lv = d.lv[L];
        int32_t lo, hi;
        gpcount::bounds<K>(lv.hi_src, lv.lo_src, v, lo, hi);
        Set S = lv.list >= 0 ? c.nbr_u(gpcount::pick<K>(v, lv.list)) : c.buf_u(lv.buf);
        S = gpcount::trim_u<G>(S, lo, hi);
        for (int32_t base = 0; base < S.n; base += G) {
            const int32_t i = base + c.g.gl;
            int32_t w[K];
#pragma unroll
            for (int j = 0; j < K; ++j) w[j] = v[j];
            bool have = false;
            if (i < S.n) {
                w[L] = S.p[i];
                have = !gpcount::inj_hit<K>(lv.inj, v, w[L]);
            }
            if constexpr (WRITE) {
                last_lockstep<K>(d, c, a, w, have, pos, st);
            } else {
                const uint32_t mine = have ? last_count<K>(d, c, w) : 0u;
                pos += c.g.sum(mine);
            }
        }
    } else {
        const GpLevel& lv = d.lv[L];
        int32_t lo, hi;
        gpcount::bounds<K>(lv.hi_src, lv.lo_src, v, lo, hi);
        Set S = lv.list >= 0 ? c.nbr_u(gpcount::pick<K>(v, lv.list)) : c.buf_u(lv.buf);
        S = gpcount::trim_u<G>(S, lo, hi);
        for (int32_t t = 0; t < S.n; ++t) {
            const int32_t x = gpcount::uni<G>(S.p[t]);
            if (gpcount::inj_hit<K>(lv.inj, v, x)) continue;
            v[L] = x;
            gpcount::run_builds<K, G, gpcount::MODE_PLAIN>(d, c, L, v);
            list_search<K, L + 1, WRITE>(d, c, a, v, pos, st);
        }
    }
}

// WRITE = false: task_rows[t] = embeddings of root task t. WRITE = true:
// task rows written from task_rows[t] on (K = 2: root t is row t).
template <int K, bool WRITE>
__global__ __launch_bounds__(kBlock) void list_kernel(GpPlanDesc d, ListArgs a) {
    __shared__ int32_t s_len[kBlock / G][GP_DESC_MAX_BUILDS];
    __shared__ int32_t s_stage[WRITE ? kBlock / G : 1][WRITE ? kStage * K : 1];
    gpcount::Ctx<G> c;
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
    c.bytes = nullptr;
    c.sj = 0;
    c.sJ = 1;
    c.deadline = 0;
    c.memo = nullptr;
    c.tag = 0;
    c.memo_log2 = 0;
    const int64_t chunk = a.chunk;
    for (;;) {
        unsigned long long t0 = 0;
        if (c.g.gl == 0) t0 = atomicAdd(a.queue, (unsigned long long)chunk);
        t0 = (unsigned long long)gpcount::uni64<G>((int64_t)c.g.bcast(t0, 0));
        if ((int64_t)t0 >= a.n_roots) break;
        const int64_t t1 = min((int64_t)t0 + chunk, a.n_roots);
        if constexpr (K == 2) {
            // every root edge is an embedding: lanes take different roots
            static_assert(WRITE, "edges need no count pass");
            for (int64_t base = (int64_t)t0; base < t1; base += G) {
                const int64_t r = base + c.g.gl;
                if (r < t1 && r < a.out_cap) {
                    const int2 e = a.roots[a.root_offset + r * a.root_stride];
                    int32_t* o = a.out + r * 2;
                    o[a.col_of[0]] = a.orig[e.x];
                    o[a.col_of[1]] = a.orig[e.y];
                }
            }
        } else {
            for (int64_t t = (int64_t)t0; t < t1; ++t) {
                const int2 e = a.roots[a.root_offset + t * a.root_stride];
                int32_t v[K];
#pragma unroll
                for (int j = 0; j < K; ++j) v[j] = 0;
                v[0] = gpcount::uni<G>(e.x);
                v[1] = gpcount::uni<G>(e.y);
                uint64_t pos = WRITE ? (uint64_t)gpcount::uni64<G>((int64_t)a.task_rows[t]) : 0;
                Stage st{WRITE ? &s_stage[grp][0] : nullptr, pos, 0};
                gpcount::run_builds<K, G, gpcount::MODE_PLAIN>(d, c, 1, v);
                list_search<K, 2, WRITE>(d, c, a, v, pos, st);
                if constexpr (WRITE) flush<K>(c.g, a, st);
                if constexpr (!WRITE)
                    if (c.g.gl == 0) a.task_rows[t] = pos;
            }
        }
    }
}

__global__ void invert_ids(const int32_t* new_id, int64_t n, int32_t* orig) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) orig[new_id[i]] = (int32_t)i;
}

__global__ void zero_words(unsigned long long* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

// found = {total rows, 0}: the last offset plus the last task's count
__global__ void list_total(const unsigned long long* cnt, const unsigned long long* off, int64_t n,
                           unsigned long long* found) {
    if (threadIdx.x == 0) {
        found[0] = n > 0 ? off[n - 1] + cnt[n - 1] : 0;
        found[1] = 0;
    }
}

__global__ void set_total(unsigned long long* found, int64_t n) {
    if (threadIdx.x == 0) {
        found[0] = (unsigned long long)n;
        found[1] = 0;
    }
}

typedef void (*ListFn)(GpPlanDesc, ListArgs);

ListFn pick_list_kernel(int k, bool write) {
    switch (k) {
        case 2: return write ? list_kernel<2, true> : nullptr;
        case 3: return write ? list_kernel<3, true> : list_kernel<3, false>;
        case 4: return write ? list_kernel<4, true> : list_kernel<4, false>;
        case 5: return write ? list_kernel<5, true> : list_kernel<5, false>;
        case 6: return write ? list_kernel<6, true> : list_kernel<6, false>;
        case 7: return write ? list_kernel<7, true> : list_kernel<7, false>;
        case 8: return write ? list_kernel<8, true> : list_kernel<8, false>;
        default: return nullptr;
    }
}

}  // namespace gplist

namespace gpint {

gp_status launch_list(const DeviceGraph& g, const GpPlanDesc& d, const int32_t* order, const LaunchCfg& cfg,
                      hipStream_t stream, unsigned long long* found_dev, int32_t* out, int64_t out_cap) {
    using namespace gplist;
    if (d.iep) return GP_ERR_UNSUPPORTED;
    if (out_cap < 0 || (out_cap > 0 && !out) || !found_dev) return GP_ERR_ARG;
    if (cfg.waves_per_cu < 1 || cfg.waves_per_cu > 32 || cfg.chunk < 1) return GP_ERR_ARG;
    if (cfg.root_stride < 1 || cfg.root_offset < 0) return GP_ERR_ARG;
    ListFn count_fn = pick_list_kernel(d.k, false), write_fn = pick_list_kernel(d.k, true);
    if (!write_fn || (d.k > 2 && !count_fn)) return GP_ERR_UNSUPPORTED;

    // the plan's restriction between levels 0 and 1 picks the root array
    int64_t all_roots = g.nnz;
    const int2* roots = g.roots_all;
    if (d.root_cut == 1) {
        all_roots = g.n_lower;
        roots = g.roots_lower;
    } else if (d.root_cut == 2) {
        all_roots = g.n_upper;
        roots = g.roots_upper;
    }
    const int64_t n_roots = all_roots > cfg.root_offset
                                ? (all_roots - cfg.root_offset + cfg.root_stride - 1) / cfg.root_stride
                                : 0;

    const int64_t groups_per_block = kBlock / G;
    int64_t blocks = std::max<int64_t>(1, (int64_t)g.num_cus * cfg.waves_per_cu / (kBlock / 64));
    const int64_t cap = std::max<int64_t>(1, g.deg2);
    if (d.nbuf > 0) {
        const int64_t budget = int64_t(16) << 30;
        const int64_t per_block = groups_per_block * d.nbuf * cap * 4;
        blocks = std::min(blocks, std::max<int64_t>(1, budget / per_block));
    }
    const int64_t need = (n_roots + cfg.chunk - 1) / cfg.chunk;
    blocks = std::min(blocks, std::max<int64_t>(1, (need + groups_per_block - 1) / groups_per_block));

    // stream-ordered allocations, all released after the kernels
    std::vector<void*> owned;
    auto get = [&](void** p, size_t bytes) {
        if (hipMallocAsync(p, std::max<size_t>(bytes, 8), stream) != hipSuccess) return false;
        owned.push_back(*p);
        return true;
    };
    auto release = [&]() {
        for (void* p : owned) (void)hipFreeAsync(p, stream);
    };
    int32_t* scratch = nullptr;
    int32_t* orig = nullptr;
    unsigned long long *queue = nullptr, *cnt = nullptr, *off = nullptr;
    void* scan_tmp = nullptr;
    size_t scan_bytes = 0;
    const size_t scratch_bytes = d.nbuf > 0 ? (size_t)(blocks * groups_per_block * d.nbuf * cap * 4) : 0;
    const bool two_pass = d.k > 2 && n_roots > 0;
    if (two_pass && n_roots > (int64_t)INT32_MAX) return GP_ERR_UNSUPPORTED;  // the scan counts in int
    if (two_pass &&
        hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, (unsigned long long*)nullptr,
                                         (unsigned long long*)nullptr, (int)n_roots, stream) != hipSuccess)
        return GP_ERR_HIP;
    if (!get((void**)&queue, sizeof(unsigned long long)) || !get((void**)&orig, sizeof(int32_t) * g.n) ||
        (scratch_bytes && !get((void**)&scratch, scratch_bytes)) ||
        (two_pass && (!get((void**)&cnt, sizeof(unsigned long long) * n_roots) ||
                      !get((void**)&off, sizeof(unsigned long long) * n_roots) || !get(&scan_tmp, scan_bytes)))) {
        release();
        return GP_ERR_NOMEM;
    }
    if (g.n > 0)
        hipLaunchKernelGGL(invert_ids, dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, stream, g.new_id, g.n,
                           orig);

    ListArgs a;
    a.row_ptr = g.row_ptr;
    a.col = g.col;
    a.roots = roots;
    a.n_roots = n_roots;
    a.root_offset = cfg.root_offset;
    a.root_stride = cfg.root_stride;
    a.hub_bits = g.hub_bits;
    a.hub_words = g.hub_words;
    a.n_hubs = g.n_hubs;
    a.scratch = scratch;
    a.buf_cap = cap;
    a.queue = queue;
    a.task_rows = nullptr;
    a.out = out;
    a.out_cap = out_cap;
    a.orig = orig;
    for (int i = 0; i < GP_DESC_MAX_K; ++i) a.col_of[i] = i < d.k ? order[i] : 0;
    a.chunk = cfg.chunk;
    if (two_pass) {
        // rows per root task, their offsets, the total; then the rows
        a.task_rows = cnt;
        hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, stream, queue, 1);
        hipLaunchKernelGGL(count_fn, dim3((unsigned)blocks), dim3(kBlock), 0, stream, d, a);
        if (hipcub::DeviceScan::ExclusiveSum(scan_tmp, scan_bytes, cnt, off, (int)n_roots, stream) != hipSuccess) {
            release();
            return GP_ERR_HIP;
        }
        hipLaunchKernelGGL(list_total, dim3(1), dim3(64), 0, stream, cnt, off, n_roots, found_dev);
        a.task_rows = off;
        hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, stream, queue, 1);
        hipLaunchKernelGGL(write_fn, dim3((unsigned)blocks), dim3(kBlock), 0, stream, d, a);
    } else if (n_roots > 0) {
        // edges: root t is row t
        hipLaunchKernelGGL(set_total, dim3(1), dim3(64), 0, stream, found_dev, n_roots);
        hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, stream, queue, 1);
        hipLaunchKernelGGL(write_fn, dim3((unsigned)blocks), dim3(kBlock), 0, stream, d, a);
    } else {
        hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, stream, found_dev, 2);
    }
    const hipError_t le = hipGetLastError();
    release();
    return le == hipSuccess ? GP_OK : GP_ERR_HIP;
}

}  // namespace gpint
