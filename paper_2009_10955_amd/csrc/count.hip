// Host side of the counting kernel: launch geometry, scratch, dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "count_kernel.hpp"

namespace gpcount {
KernelFn pick_kernel_k2(int group, int leaf, int mode);
KernelFn pick_kernel_k3(int group, int leaf, int mode);
KernelFn pick_kernel_k4(int group, int leaf, int mode);
KernelFn pick_kernel_k5(int group, int leaf, int mode);
KernelFn pick_kernel_k6(int group, int leaf, int mode);
KernelFn pick_kernel_k7(int group, int leaf, int mode);
KernelFn pick_kernel_k8(int group, int leaf, int mode);

namespace {
__global__ void init_counters(unsigned long long* p, int n) {
    int i = threadIdx.x;
    if (i < n) p[i] = 0;
}

KernelFn pick_kernel(int k, int group, int leaf, int mode) {
    switch (k) {
        case 2: return pick_kernel_k2(group, leaf, mode);
        case 3: return pick_kernel_k3(group, leaf, mode);
        case 4: return pick_kernel_k4(group, leaf, mode);
        case 5: return pick_kernel_k5(group, leaf, mode);
        case 6: return pick_kernel_k6(group, leaf, mode);
        case 7: return pick_kernel_k7(group, leaf, mode);
        case 8: return pick_kernel_k8(group, leaf, mode);
        default: return nullptr;
    }
}
}  // namespace
}  // namespace gpcount

using namespace gpcount;

namespace gpint {

LaunchCfg default_launch(const GpPlanDesc& d) {
    LaunchCfg cfg;
    cfg.group = 16;
    cfg.waves_per_cu = 16;
    cfg.chunk = d.k <= 3 ? 256 : 4;
    cfg.leaf = 1;
    return cfg;
}

LaunchCfg apply_launch(LaunchCfg cfg, const gp_launch* l) {
    if (l) {
        if (l->group) cfg.group = l->group;
        if (l->waves_per_cu) cfg.waves_per_cu = l->waves_per_cu;
        if (l->chunk) cfg.chunk = l->chunk;
        if (l->leaf_mode) cfg.leaf = l->leaf_mode;
        if (l->root_stride) cfg.root_stride = l->root_stride;
        cfg.root_offset = l->root_offset;
    }
    return cfg;
}

static const int2* pick_roots(const DeviceGraph& g, int root_cut, int64_t* n) {
    if (root_cut == 1) {
        *n = g.n_lower;
        return g.roots_lower;
    }
    if (root_cut == 2) {
        *n = g.n_upper;
        return g.roots_upper;
    }
    *n = g.nnz;
    return g.roots_all;
}

gp_status launch_count(const DeviceGraph& g, const GpPlanDesc& d, const LaunchCfg& cfg,
                       hipStream_t stream, unsigned long long* result_dev,
                       unsigned long long* per_root, bool account) {
    if (cfg.group != 64 && cfg.group != 32 && cfg.group != 16 && cfg.group != 8) return GP_ERR_ARG;
    if (cfg.leaf < 1 || cfg.leaf > 3) return GP_ERR_ARG;
    if (cfg.waves_per_cu < 1 || cfg.waves_per_cu > 32 || cfg.chunk < 1) return GP_ERR_ARG;
    const int mode = account ? MODE_ACCOUNT : (per_root ? MODE_PER_ROOT : MODE_PLAIN);
    KernelFn fn = pick_kernel(d.k, cfg.group, cfg.leaf, mode);
    if (!fn) return GP_ERR_UNSUPPORTED;

    int64_t all_roots = 0;
    const int2* roots = pick_roots(g, d.root_cut, &all_roots);
    if (cfg.root_stride < 1 || cfg.root_offset < 0) return GP_ERR_ARG;
    // sampled task space: roots[offset + t * stride]
    const int64_t n_roots =
        all_roots > cfg.root_offset ? (all_roots - cfg.root_offset + cfg.root_stride - 1) / cfg.root_stride : 0;

    const int waves_per_block = kBlock / 64;
    int64_t blocks = std::max<int64_t>(1, (int64_t)g.num_cus * cfg.waves_per_cu / waves_per_block);
    const int64_t groups_per_block = kBlock / cfg.group;
    int64_t cap = std::max<int64_t>(1, g.deg2);
    // keep scratch within a fixed budget: fewer resident groups if needed
    const int64_t budget = int64_t(16) << 30;
    if (d.nbuf > 0) {
        int64_t per_block = groups_per_block * d.nbuf * cap * 4;
        int64_t max_blocks = std::max<int64_t>(1, budget / per_block);
        blocks = std::min(blocks, max_blocks);
    }
    // a grid larger than the number of root tasks only adds idle groups
    int64_t need = (n_roots + cfg.chunk - 1) / cfg.chunk;
    int64_t need_blocks = std::max<int64_t>(1, (need + groups_per_block - 1) / groups_per_block);
    blocks = std::min(blocks, need_blocks);

    int32_t* scratch = nullptr;
    unsigned long long* queue = nullptr;
    size_t scratch_bytes = d.nbuf > 0 ? (size_t)(blocks * groups_per_block * d.nbuf * cap * 4) : 0;
    GP_HIP_TRY(hipMallocAsync((void**)&queue, sizeof(unsigned long long) * 2, stream));
    if (scratch_bytes) {
        if (hipMallocAsync((void**)&scratch, scratch_bytes, stream) != hipSuccess) {
            (void)hipFreeAsync(queue, stream);
            return GP_ERR_NOMEM;
        }
    }
    hipLaunchKernelGGL(init_counters, dim3(1), dim3(64), 0, stream, queue, 1);
    hipLaunchKernelGGL(init_counters, dim3(1), dim3(64), 0, stream, result_dev, account ? 3 : 2);

    CountArgs a;
    a.row_ptr = g.row_ptr;
    a.col = g.col;
    a.roots = roots;
    a.n_roots = n_roots;
    a.root_offset = cfg.root_offset;
    a.hub_bits = g.hub_bits;
    a.hub_words = g.hub_words;
    a.n_hubs = g.n_hubs;
    a.root_stride = cfg.root_stride;
    a.scratch = scratch;
    a.buf_cap = cap;
    a.queue = queue;
    a.result = result_dev;
    a.per_root = per_root;
    a.chunk = cfg.chunk;
    if (n_roots > 0) hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(kBlock), 0, stream, d, a);
    hipError_t le = hipGetLastError();
    if (scratch) (void)hipFreeAsync(scratch, stream);
    (void)hipFreeAsync(queue, stream);
    if (le != hipSuccess) return GP_ERR_HIP;
    return GP_OK;
}

gp_status launch_count_batch(const DeviceGraph& g, const GpPlanDesc* descs, int np,
                             const LaunchCfg& cfg, hipStream_t stream,
                             unsigned long long* result_dev) {
    // One plan at a time for now; the single-launch batch kernel replaces this.
    for (int i = 0; i < np; ++i) {
        gp_status s = launch_count(g, descs[i], cfg, stream, result_dev + 2 * i, nullptr, false);
        if (s != GP_OK) return s;
    }
    return GP_OK;
}

}  // namespace gpint
