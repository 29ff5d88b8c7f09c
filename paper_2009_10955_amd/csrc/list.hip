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
//   * one 64-lane group walks one search path; the levels above the last bind
//     one candidate at a time, and the last level is tested 64 candidates at
//     once, one per lane;
//   * the lanes that hold an embedding are compacted with a ballot, and one
//     atomic per 64 candidates reserves consecutive output rows;
//   * a row holds the original vertex ids, indexed by pattern vertex.
#include <hip/hip_runtime.h>

#include <algorithm>

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
    unsigned long long* found;  // embeddings found so far = next output row
    int32_t* out;               // out_cap rows of k int32
    int64_t out_cap;
    const int32_t* orig;        // layout id -> original id
    int32_t col_of[GP_DESC_MAX_K];  // output column (pattern vertex) of schedule level i
    int32_t chunk;
};

// Write out the lanes whose `ok` is set: the first K-1 levels are bound to
// v[0..K-2] (the same in every lane, or per lane for K = 2) and the last to x.
template <int K>
__device__ __forceinline__ void emit(const Group<G>& g, const ListArgs& a, const int32_t (&v)[K], bool ok,
                                     int32_t x) {
    const uint64_t m = g.ballot(ok);
    if (m == 0) return;
    unsigned long long base = 0;
    if (g.gl == 0) base = atomicAdd(a.found, (unsigned long long)__popcll(m));
    base = g.bcast(base, 0);
    if (ok) {
        const uint64_t row = base + g.below_mask_count(m);
        if (row < (uint64_t)a.out_cap) {
            int32_t* o = a.out + (int64_t)row * K;
#pragma unroll
            for (int j = 0; j < K - 1; ++j) o[a.col_of[j]] = a.orig[v[j]];
            o[a.col_of[K - 1]] = a.orig[x];
        }
    }
}

// Last level for bound v[0..K-2]: its candidate set is one list or buffer, or
// the intersection of a prefix set with the list of the level before it; cut
// to the restriction bounds, earlier images excluded.
template <int K>
__device__ void list_last(const GpPlanDesc& d, const gpcount::Ctx<G>& c, const ListArgs& a,
                          const int32_t (&v)[K]) {
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
        emit<K>(c.g, a, v, ok, x);
    }
}

template <int K, int L>
__device__ void list_search(const GpPlanDesc& d, const gpcount::Ctx<G>& c, const ListArgs& a, int32_t (&v)[K]) {
    if constexpr (L == K - 1) {
        list_last<K>(d, c, a, v);
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
            list_search<K, L + 1>(d, c, a, v);
        }
    }
}

template <int K>
__global__ __launch_bounds__(kBlock) void list_kernel(GpPlanDesc d, ListArgs a) {
    __shared__ int32_t s_len[kBlock / G][GP_DESC_MAX_BUILDS];
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
    const int64_t chunk = a.chunk;
    for (;;) {
        unsigned long long t0 = 0;
        if (c.g.gl == 0) t0 = atomicAdd(a.queue, (unsigned long long)chunk);
        t0 = (unsigned long long)gpcount::uni64<G>((int64_t)c.g.bcast(t0, 0));
        if ((int64_t)t0 >= a.n_roots) break;
        const int64_t t1 = min((int64_t)t0 + chunk, a.n_roots);
        if constexpr (K == 2) {
            // every root edge is an embedding: lanes take different roots
            for (int64_t base = (int64_t)t0; base < t1; base += G) {
                const int64_t r = base + c.g.gl;
                const bool ok = r < t1;
                int2 e = make_int2(0, 0);
                if (ok) e = a.roots[a.root_offset + r * a.root_stride];
                const int32_t v[2] = {e.x, 0};
                emit<2>(c.g, a, v, ok, e.y);
            }
        } else {
            for (int64_t t = (int64_t)t0; t < t1; ++t) {
                const int2 e = a.roots[a.root_offset + t * a.root_stride];
                int32_t v[K];
#pragma unroll
                for (int j = 0; j < K; ++j) v[j] = 0;
                v[0] = gpcount::uni<G>(e.x);
                v[1] = gpcount::uni<G>(e.y);
                gpcount::run_builds<K, G, gpcount::MODE_PLAIN>(d, c, 1, v);
                list_search<K, 2>(d, c, a, v);
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

typedef void (*ListFn)(GpPlanDesc, ListArgs);

ListFn pick_list_kernel(int k) {
    switch (k) {
        case 2: return list_kernel<2>;
        case 3: return list_kernel<3>;
        case 4: return list_kernel<4>;
        case 5: return list_kernel<5>;
        case 6: return list_kernel<6>;
        case 7: return list_kernel<7>;
        case 8: return list_kernel<8>;
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
    ListFn fn = pick_list_kernel(d.k);
    if (!fn) return GP_ERR_UNSUPPORTED;

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

    int32_t* scratch = nullptr;
    int32_t* orig = nullptr;
    unsigned long long* queue = nullptr;
    const size_t scratch_bytes = d.nbuf > 0 ? (size_t)(blocks * groups_per_block * d.nbuf * cap * 4) : 0;
    GP_HIP_TRY(hipMallocAsync((void**)&queue, sizeof(unsigned long long), stream));
    if (hipMallocAsync((void**)&orig, sizeof(int32_t) * std::max<int64_t>(1, g.n), stream) != hipSuccess) {
        (void)hipFreeAsync(queue, stream);
        return GP_ERR_NOMEM;
    }
    if (scratch_bytes && hipMallocAsync((void**)&scratch, scratch_bytes, stream) != hipSuccess) {
        (void)hipFreeAsync(orig, stream);
        (void)hipFreeAsync(queue, stream);
        return GP_ERR_NOMEM;
    }
    hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, stream, queue, 1);
    hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, stream, found_dev, 2);
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
    a.found = found_dev;
    a.out = out;
    a.out_cap = out_cap;
    a.orig = orig;
    for (int i = 0; i < GP_DESC_MAX_K; ++i) a.col_of[i] = i < d.k ? order[i] : 0;
    a.chunk = cfg.chunk;
    if (n_roots > 0) hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(kBlock), 0, stream, d, a);
    const hipError_t le = hipGetLastError();
    if (scratch) (void)hipFreeAsync(scratch, stream);
    (void)hipFreeAsync(orig, stream);
    (void)hipFreeAsync(queue, stream);
    return le == hipSuccess ? GP_OK : GP_ERR_HIP;
}

}  // namespace gpint
