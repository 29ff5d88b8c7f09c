// Graph layout in HBM (device side of gp_load_graph).
//
// Input: an undirected simple graph as CSR with sorted, contiguous neighbor
// lists (Section IV-E). Steps, all on the device:
//   1. validate: rows non-decreasing, columns in range, each list strictly
//      ascending (no duplicates), no self-loops, every (u,v) has (v,u);
//   2. relabel by descending degree, ties by ascending id (radix sort of
//      (degree, id) keys), rebuild the CSR by a radix sort of relabelled
//      (src, dst) keys, so every list is again ascending;
//   3. root-edge arrays: all entries, entries with v1 < v0, entries with
//      v1 > v0, each in CSR order (hubs first);
//   4. content hash of the input (order-independent sum of mixed entries).
// The triangle count for the cost model is taken afterwards by the counting
// kernel itself (see the API layer).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "internal.hpp"
#include "sets.hpp"

using namespace gpdev;

namespace {

enum : unsigned {
    F_RANGE = 1,
    F_UNSORTED = 2,
    F_SELFLOOP = 4,
    F_DUP = 8,
    F_ASYM = 16,
};

__device__ __forceinline__ int64_t row_of(const int64_t* row_ptr, int64_t n, int64_t e) {
    // last v with row_ptr[v] <= e
    int64_t lo = 0, hi = n;  // answer in [0, n)
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (row_ptr[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void check_rows(const int64_t* row_ptr, int64_t n, int64_t nnz, unsigned* flags) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        int64_t b = row_ptr[v], e = row_ptr[v + 1];
        if (b > e || b < 0 || e > nnz || e - b > 0x7fffffff) atomicOr(flags, (unsigned)F_UNSORTED);
    }
}

__global__ void check_entries(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz,
                              unsigned* flags) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t v = row_of(row_ptr, n, e);
        int32_t w = col[e];
        unsigned f = 0;
        if (w < 0 || w >= n) {
            f |= F_RANGE;
        } else {
            if (w == v) f |= F_SELFLOOP;
            if (e + 1 < row_ptr[v + 1]) {
                int32_t nx = col[e + 1];
                if (nx == w) f |= F_DUP;
                else if (nx < w) f |= F_UNSORTED;
            }
            int64_t b = row_ptr[w];
            int64_t len = row_ptr[w + 1] - b;
            if (len < 0 || b < 0 || b + len > nnz) {
                f |= F_UNSORTED;
            } else if (!contains(col + b, (int32_t)len, (int32_t)v)) {
                f |= F_ASYM;
            }
        }
        if (f) atomicOr(flags, f);
    }
}

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    // splitmix64 finaliser
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

__global__ void hash_input(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz,
                           unsigned long long* out) {
    uint64_t h = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nnz + n + 1;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i < nnz) h += mix64(((uint64_t)i << 32) ^ (uint32_t)col[i]);
        else h += mix64(0xabcdef0000000000ull ^ ((uint64_t)(i - nnz) << 40) ^ (uint64_t)row_ptr[i - nnz]);
    }
    for (int off = 32; off >= 1; off >>= 1) h += __shfl_xor(h, off, 64);
    if (__lane_id() == 0) atomicAdd(out, (unsigned long long)h);
}

__global__ void degree_keys(const int64_t* row_ptr, int64_t n, uint64_t* keys) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        uint64_t deg = (uint64_t)(row_ptr[v + 1] - row_ptr[v]);
        keys[v] = ((uint64_t)(0xffffffffu - (uint32_t)deg) << 32) | (uint64_t)v;
    }
}

__global__ void assign_ids(const uint64_t* sorted, const int64_t* row_ptr, int64_t n,
                           int32_t* new_id, int64_t* new_deg) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        int64_t old = (int64_t)(sorted[p] & 0xffffffffu);
        new_id[old] = (int32_t)p;
        new_deg[p] = row_ptr[old + 1] - row_ptr[old];
    }
}

__global__ void edge_keys(const int64_t* row_ptr, const int32_t* col, const int32_t* new_id,
                          int64_t n, int64_t nnz, int shift, uint64_t* keys) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t v = row_of(row_ptr, n, e);
        keys[e] = ((uint64_t)(uint32_t)new_id[v] << shift) | (uint64_t)(uint32_t)new_id[col[e]];
    }
}

__global__ void unpack_edges(const uint64_t* keys, int64_t nnz, int shift, int32_t* col,
                             int2* roots_all) {
    const uint64_t mask = (uint64_t(1) << shift) - 1;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint64_t k = keys[e];
        int32_t w = (int32_t)(k & mask);
        int32_t v = (int32_t)(k >> shift);
        col[e] = w;
        roots_all[e] = make_int2(v, w);
    }
}

// Number of neighbors below v (the lower part of each sorted list).
__global__ void count_lower(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t* lower,
                            int64_t* upper) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        int64_t b = row_ptr[v];
        int32_t len = (int32_t)(row_ptr[v + 1] - b);
        int32_t lo = lower_bound(col + b, len, (int32_t)v);
        lower[v] = lo;
        upper[v] = len - lo;
    }
}

__global__ void scatter_roots(const int64_t* row_ptr, const int2* roots_all, int64_t n, int64_t nnz,
                              const int64_t* lower_cnt, const int64_t* lower_off,
                              const int64_t* upper_off, int2* roots_lower, int2* roots_upper) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        int2 r = roots_all[e];
        int64_t v = r.x;
        int64_t k = e - row_ptr[v];
        if (k < lower_cnt[v]) roots_lower[lower_off[v] + k] = r;
        else roots_upper[upper_off[v] + (k - lower_cnt[v])] = r;
    }
}

// Root arrays ordered by their smaller endpoint, which in the degree-sorted
// layout is the higher-degree one: the heaviest roots come first (they start
// first, and the kernel can split a prefix of them). roots_upper stays in CSR
// order (v0 < v1, v0 ascending); roots_lower holds the same edges reversed in
// the same order; roots_all interleaves the two.
__global__ void order_roots(const int2* roots_upper, int64_t n_upper, int2* roots_lower, int2* roots_all) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_upper;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int2 u = roots_upper[k];
        const int2 r = make_int2(u.y, u.x);
        roots_lower[k] = r;
        roots_all[2 * k] = u;
        roots_all[2 * k + 1] = r;
    }
}

__global__ void fill_hub_bits(const int64_t* row_ptr, const int32_t* col, int64_t n_hubs,
                              int64_t n_entries, int64_t words, uint32_t* bits) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_entries;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = row_of(row_ptr, n_hubs, e);
        const int32_t w = col[e];
        atomicOr(&bits[v * words + (w >> 5)], 1u << (w & 31));
    }
}

unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return (unsigned)b;
}

struct TempPool {
    hipStream_t s;
    void* ptrs[32];
    int n = 0;
    explicit TempPool(hipStream_t st) : s(st) {}
    hipError_t get(void** p, size_t bytes) {
        hipError_t e = hipMallocAsync(p, bytes ? bytes : 8, s);
        if (e == hipSuccess && n < 32) ptrs[n++] = *p;
        return e;
    }
    ~TempPool() {
        for (int i = 0; i < n; ++i) (void)hipFreeAsync(ptrs[i], s);
    }
};

}  // namespace

namespace gpint {

// Fills g (device buffers owned by g). row_ptr/col are device pointers.
gp_status build_layout(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz,
                       hipStream_t s, DeviceGraph* g) {
    TempPool tmp(s);
    unsigned* flags = nullptr;
    unsigned long long* hash = nullptr;
    GP_HIP_TRY(tmp.get((void**)&flags, sizeof(unsigned)));
    GP_HIP_TRY(tmp.get((void**)&hash, sizeof(unsigned long long)));
    GP_HIP_TRY(hipMemsetAsync(flags, 0, sizeof(unsigned), s));
    GP_HIP_TRY(hipMemsetAsync(hash, 0, sizeof(unsigned long long), s));
    if (n > 0) hipLaunchKernelGGL(check_rows, dim3(grid_for(n)), dim3(256), 0, s, row_ptr, n, nnz, flags);
    unsigned hflags = 0;
    GP_HIP_TRY(hipMemcpyAsync(&hflags, flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    GP_HIP_TRY(hipStreamSynchronize(s));
    if (hflags) return GP_ERR_CSR_UNSORTED;
    if (nnz > 0) {
        hipLaunchKernelGGL(check_entries, dim3(grid_for(nnz)), dim3(256), 0, s, row_ptr, col, n, nnz,
                           flags);
        GP_HIP_TRY(hipGetLastError());
        GP_HIP_TRY(hipMemcpyAsync(&hflags, flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
        GP_HIP_TRY(hipStreamSynchronize(s));
        if (hflags & F_RANGE) return GP_ERR_CSR_RANGE;
        if (hflags & F_UNSORTED) return GP_ERR_CSR_UNSORTED;
        if (hflags & F_SELFLOOP) return GP_ERR_CSR_SELFLOOP;
        if (hflags & F_DUP) return GP_ERR_CSR_DUPLICATE;
        if (hflags & F_ASYM) return GP_ERR_CSR_ASYMMETRIC;
    }
    hipLaunchKernelGGL(hash_input, dim3(grid_for(nnz + n + 1)), dim3(256), 0, s, row_ptr, col, n, nnz,
                       hash);

    // device buffers owned by the graph
    const int64_t nn = n > 0 ? n : 1;
    const int64_t ne = nnz > 0 ? nnz : 1;
    GP_HIP_TRY(hipMalloc((void**)&g->row_ptr, sizeof(int64_t) * (n + 1)));
    GP_HIP_TRY(hipMalloc((void**)&g->col, sizeof(int32_t) * ne));
    GP_HIP_TRY(hipMalloc((void**)&g->roots_all, sizeof(int2) * ne));
    GP_HIP_TRY(hipMalloc((void**)&g->new_id, sizeof(int32_t) * nn));

    // 2. relabel by descending degree, ties by ascending id
    uint64_t *vkeys = nullptr, *vkeys_sorted = nullptr;
    int64_t* new_deg = nullptr;
    GP_HIP_TRY(tmp.get((void**)&vkeys, sizeof(uint64_t) * nn));
    GP_HIP_TRY(tmp.get((void**)&vkeys_sorted, sizeof(uint64_t) * nn));
    GP_HIP_TRY(tmp.get((void**)&new_deg, sizeof(int64_t) * (n + 1)));
    if (n > 0) hipLaunchKernelGGL(degree_keys, dim3(grid_for(n)), dim3(256), 0, s, row_ptr, n, vkeys);
    size_t tb = 0;
    GP_HIP_TRY(hipcub::DeviceRadixSort::SortKeys(nullptr, tb, vkeys, vkeys_sorted, (int)n, 0, 64, s));
    void* tstore = nullptr;
    GP_HIP_TRY(tmp.get(&tstore, tb));
    GP_HIP_TRY(hipcub::DeviceRadixSort::SortKeys(tstore, tb, vkeys, vkeys_sorted, (int)n, 0, 64, s));
    if (n > 0)
        hipLaunchKernelGGL(assign_ids, dim3(grid_for(n)), dim3(256), 0, s, vkeys_sorted, row_ptr, n,
                           g->new_id, new_deg);
    GP_HIP_TRY(hipMemsetAsync(new_deg + n, 0, sizeof(int64_t), s));
    // row_ptr of the layout = exclusive scan of new degrees (n+1 entries)
    tb = 0;
    GP_HIP_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, new_deg, g->row_ptr, (int)(n + 1), s));
    void* tscan = nullptr;
    GP_HIP_TRY(tmp.get(&tscan, tb));
    GP_HIP_TRY(hipcub::DeviceScan::ExclusiveSum(tscan, tb, new_deg, g->row_ptr, (int)(n + 1), s));

    int bits = 1;
    while ((int64_t(1) << bits) < nn) ++bits;
    const int shift = bits;
    uint64_t *ekeys = nullptr, *ekeys_sorted = nullptr;
    GP_HIP_TRY(tmp.get((void**)&ekeys, sizeof(uint64_t) * ne));
    GP_HIP_TRY(tmp.get((void**)&ekeys_sorted, sizeof(uint64_t) * ne));
    if (nnz > 0)
        hipLaunchKernelGGL(edge_keys, dim3(grid_for(nnz)), dim3(256), 0, s, row_ptr, col, g->new_id, n,
                           nnz, shift, ekeys);
    tb = 0;
    GP_HIP_TRY(hipcub::DeviceRadixSort::SortKeys(nullptr, tb, ekeys, ekeys_sorted, (int)nnz, 0,
                                                 2 * bits, s));
    void* tsort = nullptr;
    GP_HIP_TRY(tmp.get(&tsort, tb));
    GP_HIP_TRY(hipcub::DeviceRadixSort::SortKeys(tsort, tb, ekeys, ekeys_sorted, (int)nnz, 0,
                                                 2 * bits, s));
    if (nnz > 0)
        hipLaunchKernelGGL(unpack_edges, dim3(grid_for(nnz)), dim3(256), 0, s, ekeys_sorted, nnz, shift,
                           g->col, g->roots_all);

    // 3. oriented root arrays
    int64_t *lower_cnt = nullptr, *upper_cnt = nullptr, *lower_off = nullptr, *upper_off = nullptr;
    GP_HIP_TRY(tmp.get((void**)&lower_cnt, sizeof(int64_t) * (n + 1)));
    GP_HIP_TRY(tmp.get((void**)&upper_cnt, sizeof(int64_t) * (n + 1)));
    GP_HIP_TRY(tmp.get((void**)&lower_off, sizeof(int64_t) * (n + 1)));
    GP_HIP_TRY(tmp.get((void**)&upper_off, sizeof(int64_t) * (n + 1)));
    GP_HIP_TRY(hipMemsetAsync(lower_cnt + n, 0, sizeof(int64_t), s));
    GP_HIP_TRY(hipMemsetAsync(upper_cnt + n, 0, sizeof(int64_t), s));
    if (n > 0)
        hipLaunchKernelGGL(count_lower, dim3(grid_for(n)), dim3(256), 0, s, g->row_ptr, g->col, n,
                           lower_cnt, upper_cnt);
    tb = 0;
    GP_HIP_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, lower_cnt, lower_off, (int)(n + 1), s));
    void* tscan2 = nullptr;
    GP_HIP_TRY(tmp.get(&tscan2, tb));
    GP_HIP_TRY(hipcub::DeviceScan::ExclusiveSum(tscan2, tb, lower_cnt, lower_off, (int)(n + 1), s));
    GP_HIP_TRY(hipcub::DeviceScan::ExclusiveSum(tscan2, tb, upper_cnt, upper_off, (int)(n + 1), s));
    int64_t hv[2] = {0, 0};
    GP_HIP_TRY(hipMemcpyAsync(&hv[0], lower_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    GP_HIP_TRY(hipMemcpyAsync(&hv[1], upper_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    int64_t degs[2] = {0, 0};
    if (n > 0) GP_HIP_TRY(hipMemcpyAsync(&degs[0], new_deg, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (n > 1) GP_HIP_TRY(hipMemcpyAsync(&degs[1], new_deg + 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    unsigned long long hhash = 0;
    GP_HIP_TRY(hipMemcpyAsync(&hhash, hash, sizeof(hhash), hipMemcpyDeviceToHost, s));
    GP_HIP_TRY(hipStreamSynchronize(s));
    g->n_lower = hv[0];
    g->n_upper = hv[1];
    GP_HIP_TRY(hipMalloc((void**)&g->roots_lower, sizeof(int2) * (hv[0] > 0 ? hv[0] : 1)));
    GP_HIP_TRY(hipMalloc((void**)&g->roots_upper, sizeof(int2) * (hv[1] > 0 ? hv[1] : 1)));
    if (nnz > 0)
        hipLaunchKernelGGL(scatter_roots, dim3(grid_for(nnz)), dim3(256), 0, s, g->row_ptr, g->roots_all,
                           n, nnz, lower_cnt, lower_off, upper_off, g->roots_lower, g->roots_upper);
    GP_HIP_TRY(hipGetLastError());
    if (hv[0] != hv[1] || hv[0] + hv[1] != nnz) return GP_ERR_INTERNAL;  // validated symmetric, loop-free
    if (hv[1] > 0)
        hipLaunchKernelGGL(order_roots, dim3(grid_for(hv[1])), dim3(256), 0, s, g->roots_upper, hv[1],
                           g->roots_lower, g->roots_all);
    GP_HIP_TRY(hipGetLastError());
    // upper_pref[i]: roots of each ordered array per orientation whose smaller
    // endpoint is below 2^i
    for (int i = 0; i < 32; ++i) {
        const int64_t v = std::min<int64_t>(int64_t(1) << i, n);
        GP_HIP_TRY(hipMemcpyAsync(&g->upper_pref[i], upper_off + v, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    }
    GP_HIP_TRY(hipStreamSynchronize(s));
    g->n = n;
    g->nnz = nnz;
    g->max_deg = degs[0];
    g->deg2 = degs[1];
    g->stats.n = n;
    g->stats.m = nnz / 2;
    g->stats.max_degree = degs[0];
    g->stats.hash = hhash;
    return GP_OK;
}

// Dense neighbor bitmaps for the highest-degree vertices. In the
// degree-descending layout they are ids [0, n_hubs), whose lists are the first
// row_ptr[n_hubs] CSR entries. A vertex qualifies with degree >= min_degree;
// the count is capped so that all bitmaps fit in budget_bytes.
gp_status build_hub_bitmaps(DeviceGraph* g, int64_t min_degree, int64_t budget_bytes, hipStream_t s) {
    g->n_hubs = 0;
    g->hub_words = (g->n + 31) / 32;
    if (g->n == 0 || g->nnz == 0 || g->hub_words == 0) return GP_OK;
    const int64_t per = g->hub_words * 4;
    int64_t cap = std::min<int64_t>(g->n, budget_bytes / per);
    if (cap <= 0) return GP_OK;
    std::vector<int64_t> rp(cap + 1);
    GP_HIP_TRY(hipMemcpyAsync(rp.data(), g->row_ptr, sizeof(int64_t) * (cap + 1), hipMemcpyDeviceToHost, s));
    GP_HIP_TRY(hipStreamSynchronize(s));
    int64_t h = 0;
    while (h < cap && rp[h + 1] - rp[h] >= min_degree) ++h;
    if (h == 0) return GP_OK;
    GP_HIP_TRY(hipMalloc((void**)&g->hub_bits, (size_t)(h * per)));
    GP_HIP_TRY(hipMemsetAsync(g->hub_bits, 0, (size_t)(h * per), s));
    const int64_t entries = rp[h];
    hipLaunchKernelGGL(fill_hub_bits, dim3(grid_for(entries)), dim3(256), 0, s, g->row_ptr, g->col, h,
                       entries, g->hub_words, g->hub_bits);
    GP_HIP_TRY(hipGetLastError());
    GP_HIP_TRY(hipStreamSynchronize(s));
    g->n_hubs = (int32_t)h;
    g->stats.hub_vertices = h;
    g->stats.hub_bitmap_bytes = h * per;
    return GP_OK;
}

}  // namespace gpint
