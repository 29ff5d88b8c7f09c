// Host side of the counting kernel: launch geometry, scratch, dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "count_kernel.hpp"

namespace gpcount {
KernelFn pick_kernel_k2(int group, int leaf, int mode, bool iep);
KernelFn pick_kernel_k3(int group, int leaf, int mode, bool iep);
KernelFn pick_kernel_k4(int group, int leaf, int mode, bool iep);
KernelFn pick_kernel_k5(int group, int leaf, int mode, bool iep);
KernelFn pick_kernel_k6(int group, int leaf, int mode, bool iep);
KernelFn pick_kernel_k7(int group, int leaf, int mode, bool iep);
KernelFn pick_kernel_k8(int group, int leaf, int mode, bool iep);
#define GP_DECL_BATCH(g, k, l) BatchFn batch_kernel_g##g##_k##k##_l##l();
GP_DECL_BATCH(64, 5, 1) GP_DECL_BATCH(64, 6, 1) GP_DECL_BATCH(64, 8, 1)
GP_DECL_BATCH(32, 5, 1) GP_DECL_BATCH(32, 6, 1) GP_DECL_BATCH(32, 8, 1)
GP_DECL_BATCH(64, 5, 3) GP_DECL_BATCH(64, 6, 3) GP_DECL_BATCH(64, 8, 3)
GP_DECL_BATCH(32, 5, 3) GP_DECL_BATCH(32, 6, 3) GP_DECL_BATCH(32, 8, 3)
GP_DECL_BATCH(16, 5, 1) GP_DECL_BATCH(16, 6, 1) GP_DECL_BATCH(16, 8, 1)
GP_DECL_BATCH(16, 5, 3) GP_DECL_BATCH(16, 6, 3) GP_DECL_BATCH(16, 8, 3)
GP_DECL_BATCH(64, 5, 4) GP_DECL_BATCH(64, 6, 4) GP_DECL_BATCH(64, 8, 4)
GP_DECL_BATCH(32, 5, 4) GP_DECL_BATCH(32, 6, 4) GP_DECL_BATCH(32, 8, 4)
GP_DECL_BATCH(16, 5, 4) GP_DECL_BATCH(16, 6, 4) GP_DECL_BATCH(16, 8, 4)
#undef GP_DECL_BATCH

BatchFn pick_batch_kernel(int group, int kmax, int leaf) {
    const int km = kmax <= 5 ? 5 : (kmax <= 6 ? 6 : 8);
    if (leaf == 4) {
        if (group == 64) return km == 5 ? batch_kernel_g64_k5_l4() : (km == 6 ? batch_kernel_g64_k6_l4() : batch_kernel_g64_k8_l4());
        if (group == 16) return km == 5 ? batch_kernel_g16_k5_l4() : (km == 6 ? batch_kernel_g16_k6_l4() : batch_kernel_g16_k8_l4());
        return km == 5 ? batch_kernel_g32_k5_l4() : (km == 6 ? batch_kernel_g32_k6_l4() : batch_kernel_g32_k8_l4());
    }
    if (leaf == 3) {
        if (group == 64) return km == 5 ? batch_kernel_g64_k5_l3() : (km == 6 ? batch_kernel_g64_k6_l3() : batch_kernel_g64_k8_l3());
        if (group == 16) return km == 5 ? batch_kernel_g16_k5_l3() : (km == 6 ? batch_kernel_g16_k6_l3() : batch_kernel_g16_k8_l3());
        return km == 5 ? batch_kernel_g32_k5_l3() : (km == 6 ? batch_kernel_g32_k6_l3() : batch_kernel_g32_k8_l3());
    }
    if (group == 64) return km == 5 ? batch_kernel_g64_k5_l1() : (km == 6 ? batch_kernel_g64_k6_l1() : batch_kernel_g64_k8_l1());
    if (group == 16) return km == 5 ? batch_kernel_g16_k5_l1() : (km == 6 ? batch_kernel_g16_k6_l1() : batch_kernel_g16_k8_l1());
    return km == 5 ? batch_kernel_g32_k5_l1() : (km == 6 ? batch_kernel_g32_k6_l1() : batch_kernel_g32_k8_l1());
}

namespace {
__global__ void init_counters(unsigned long long* p, int n) {
    int i = threadIdx.x;
    if (i < n) p[i] = 0;
}

KernelFn pick_kernel(int k, int group, int leaf, int mode, bool iep) {
    switch (k) {
        case 2: return pick_kernel_k2(group, leaf, mode, iep);
        case 3: return pick_kernel_k3(group, leaf, mode, iep);
        case 4: return pick_kernel_k4(group, leaf, mode, iep);
        case 5: return pick_kernel_k5(group, leaf, mode, iep);
        case 6: return pick_kernel_k6(group, leaf, mode, iep);
        case 7: return pick_kernel_k7(group, leaf, mode, iep);
        case 8: return pick_kernel_k8(group, leaf, mode, iep);
        default: return nullptr;
    }
}

__global__ void zero_u64(unsigned long long* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Whether leaf mode 4 may keep its last-level counts per root: the last
// level is pre & N(v[k-2]) with pre the list of a root level, its cut comes
// from the root levels only, and every earlier image it must avoid is a
// parent of level k-2.
bool memo_eligible(const GpPlanDesc& d) {
    if (d.k < 4 || d.iep) return false;
    const GpLevel& ll = d.lv[d.k - 1];
    if (ll.last_list != d.k - 2 || ll.pre_buf >= 0 || ll.pre_list < 0 || ll.pre_list > 1) return false;
    if ((ll.hi_src | ll.lo_src) & ~3u) return false;
    return (ll.inj & ~(uint32_t)d.lv[d.k - 2].parents) == 0;
}

// Divide an IEP total by its over-count; flag 2 if it does not divide.
__global__ void iep_divide(unsigned long long* result, unsigned long long div) {
    if (threadIdx.x == 0 && div > 0) {
        const unsigned long long t = result[0];
        if (t % div) result[1] |= 2ull;
        result[0] = t / div;
    }
}
}  // namespace
}  // namespace gpcount

using namespace gpcount;

namespace gpint {

LaunchCfg default_launch(const GpPlanDesc& d) {
    LaunchCfg cfg;
    cfg.group = 64;
    cfg.waves_per_cu = 32;
    cfg.chunk = d.k <= 3 ? 256 : 4;
    cfg.leaf = 1;
    cfg.split_ways = 16;
    cfg.split_vertices = 256;
    return cfg;
}

int resident_waves_per_cu(const GpPlanDesc& d, const LaunchCfg& cfg) {
    const bool iep = d.iep != 0;
    const int group = iep ? (cfg.group >= 64 ? 64 : 32) : cfg.group;
    KernelFn fn = pick_kernel(d.k, group, cfg.leaf, MODE_PLAIN, iep);
    int nb = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)fn, kBlock, 0) != hipSuccess ||
        nb <= 0)
        return cfg.waves_per_cu;
    return std::min(cfg.waves_per_cu, nb * (kBlock / 64));
}

LaunchCfg apply_launch(LaunchCfg cfg, const gp_launch* l) {
    if (l) {
        if (l->group) cfg.group = l->group;
        if (l->waves_per_cu) cfg.waves_per_cu = l->waves_per_cu;
        if (l->chunk) cfg.chunk = l->chunk;
        if (l->leaf_mode) cfg.leaf = l->leaf_mode;
        if (l->root_stride) cfg.root_stride = l->root_stride;
        cfg.root_offset = l->root_offset;
        if (l->split_ways) cfg.split_ways = l->split_ways;
        if (l->split_vertices) cfg.split_vertices = l->split_vertices;
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

// Roots split into several tasks: the first `roots` of the (sampled) root
// array, whose smaller endpoint is below 2^floor(log2(split_vertices)).
// Per-root and byte-accounting counts stay one task per root, and so do
// patterns with no level-2 loop (k <= 3, IEP at k = 4).
struct SplitPlan {
    int64_t roots = 0;
    int ways = 1;
};

static SplitPlan split_plan(const DeviceGraph& g, const GpPlanDesc& d, const LaunchCfg& cfg, int mode,
                            int64_t n_roots, int64_t stride, int64_t offset) {
    SplitPlan sp;
    const bool iep = d.iep != 0;
    if (mode != MODE_PLAIN || d.k < 4 || (iep && d.k == 4) || cfg.split_ways <= 1 || cfg.split_vertices <= 0)
        return sp;
    int i = 0;
    while (i < 31 && (int64_t(1) << (i + 1)) <= cfg.split_vertices) ++i;
    const int64_t pref = g.upper_pref[i] * (d.root_cut == 0 ? 2 : 1);
    const int64_t sampled = pref > offset ? (pref - offset + stride - 1) / stride : 0;
    sp.roots = std::min(n_roots, sampled);
    sp.ways = cfg.split_ways;
    return sp;
}

static const int2* pick_roots(const DeviceGraph& g, int root_cut, int64_t* n);

int64_t task_count(const DeviceGraph& g, const GpPlanDesc& d, const LaunchCfg& cfg) {
    int64_t n = 0;
    (void)pick_roots(g, d.root_cut, &n);
    const SplitPlan sp = split_plan(g, d, cfg, MODE_PLAIN, n, 1, 0);
    return n + sp.roots * (sp.ways - 1);
}

gp_status launch_count(const DeviceGraph& g, const GpPlanDesc& d, const LaunchCfg& cfg,
                       hipStream_t stream, unsigned long long* result_dev,
                       unsigned long long* per_root, bool account, unsigned long long* busy) {
    if (cfg.group != 64 && cfg.group != 32 && cfg.group != 16 && cfg.group != 8) return GP_ERR_ARG;
    if (cfg.leaf < 1 || cfg.leaf > 4) return GP_ERR_ARG;
    if (cfg.waves_per_cu < 1 || cfg.waves_per_cu > 32 || cfg.chunk < 1) return GP_ERR_ARG;
    const int mode = account ? MODE_ACCOUNT : (per_root ? MODE_PER_ROOT : MODE_PLAIN);
    const bool iep = d.iep != 0;
    const int group = iep ? (cfg.group >= 64 ? 64 : 32) : cfg.group;  // IEP kernels: 64 or 32 lanes
    KernelFn fn = pick_kernel(d.k, group, cfg.leaf, mode, iep);
    if (!fn) return GP_ERR_UNSUPPORTED;

    int64_t all_roots = 0;
    const int2* roots = pick_roots(g, d.root_cut, &all_roots);
    if (cfg.root_stride < 1 || cfg.root_offset < 0) return GP_ERR_ARG;
    if (cfg.split_ways < 1 || cfg.split_ways > 4096 || cfg.split_vertices < 0 || cfg.budget_ms < 0)
        return GP_ERR_ARG;
    // sampled roots: roots[offset + r * stride]
    auto sampled = [&](int64_t n) {
        return n > cfg.root_offset ? (n - cfg.root_offset + cfg.root_stride - 1) / cfg.root_stride : 0;
    };
    const int64_t n_roots = sampled(all_roots);
    const SplitPlan sp = split_plan(g, d, cfg, mode, n_roots, cfg.root_stride, cfg.root_offset);
    const int64_t split_roots = sp.roots;
    const int split_ways = sp.ways;
    const int64_t n_tasks = n_roots + split_roots * (split_ways - 1);

    const int waves_per_block = kBlock / 64;
    int64_t blocks = std::max<int64_t>(1, (int64_t)g.num_cus * cfg.waves_per_cu / waves_per_block);
    const int64_t groups_per_block = kBlock / group;
    int64_t cap = std::max<int64_t>(1, g.deg2);
    // keep scratch within a fixed budget: fewer resident groups if needed
    const int64_t budget = int64_t(16) << 30;
    if (d.nbuf > 0) {
        int64_t per_block = groups_per_block * d.nbuf * cap * 4;
        int64_t max_blocks = std::max<int64_t>(1, budget / per_block);
        blocks = std::min(blocks, max_blocks);
    }
    // a grid larger than the number of root tasks only adds idle groups
    int64_t need = (n_tasks + cfg.chunk - 1) / cfg.chunk;
    int64_t need_blocks = std::max<int64_t>(1, (need + groups_per_block - 1) / groups_per_block);
    blocks = std::min(blocks, need_blocks);

    int32_t* scratch = nullptr;
    unsigned long long* queue = nullptr;
    unsigned long long* memo = nullptr;
    size_t scratch_bytes = d.nbuf > 0 ? (size_t)(blocks * groups_per_block * d.nbuf * cap * 4) : 0;
    // leaf mode 4's per-task memo: one word per hub per group, within 4 GiB
    const int64_t memo_words = blocks * groups_per_block * (int64_t)g.n_hubs;
    const bool use_memo = cfg.leaf == 4 && mode != MODE_ACCOUNT && !iep && g.n_hubs > 0 && memo_eligible(d) &&
                          n_tasks < (int64_t(1) << 31) && memo_words * 8 <= (int64_t(4) << 30);
    GP_HIP_TRY(hipMallocAsync((void**)&queue, sizeof(unsigned long long) * 2, stream));
    if (scratch_bytes) {
        if (hipMallocAsync((void**)&scratch, scratch_bytes, stream) != hipSuccess) {
            (void)hipFreeAsync(queue, stream);
            return GP_ERR_NOMEM;
        }
    }
    if (use_memo) {
        if (hipMallocAsync((void**)&memo, (size_t)memo_words * 8, stream) != hipSuccess) {
            if (scratch) (void)hipFreeAsync(scratch, stream);
            (void)hipFreeAsync(queue, stream);
            return GP_ERR_NOMEM;
        }
        hipLaunchKernelGGL(zero_u64, dim3((unsigned)std::min<int64_t>(4096, (memo_words + 255) / 256)), dim3(256), 0,
                           stream, memo, memo_words);
    }
    hipLaunchKernelGGL(init_counters, dim3(1), dim3(64), 0, stream, queue, 1);
    hipLaunchKernelGGL(init_counters, dim3(1), dim3(64), 0, stream, result_dev, account ? 3 : 2);
    if (busy) hipLaunchKernelGGL(init_counters, dim3(1), dim3(64), 0, stream, busy, 3);

    CountArgs a;
    a.row_ptr = g.row_ptr;
    a.col = g.col;
    a.roots = roots;
    a.n_roots = n_roots;
    a.n_tasks = n_tasks;
    a.split_roots = split_roots;
    a.split_ways = split_ways;
    a.budget_ticks = busy && cfg.budget_ms > 0 ? (uint64_t)(cfg.budget_ms * g.wall_khz) : 0;
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
    a.busy = busy;
    a.memo = memo;
    a.chunk = cfg.chunk;
    if (n_tasks > 0) hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(kBlock), 0, stream, d, a);
    if (iep)
        hipLaunchKernelGGL(iep_divide, dim3(1), dim3(64), 0, stream, result_dev, (unsigned long long)d.iep_div);
    hipError_t le = hipGetLastError();
    if (scratch) (void)hipFreeAsync(scratch, stream);
    if (memo) (void)hipFreeAsync(memo, stream);
    (void)hipFreeAsync(queue, stream);
    if (le != hipSuccess) return GP_ERR_HIP;
    return GP_OK;
}

int64_t root_task_count(const DeviceGraph& g, const GpPlanDesc& d) {
    int64_t n = 0;
    (void)pick_roots(g, d.root_cut, &n);
    return n;
}

void batch_release(BatchState* st) {
    (void)hipFree(st->descs);
    (void)hipFree(st->plans);
    (void)hipFree(st->scratch);
    (void)hipFree(st->queue);
    (void)hipFree(st->result);
    *st = BatchState{};
}

// Per-plan task ranges and the launch geometry for np plans.
static gp_status batch_layout(const DeviceGraph& g, const GpPlanDesc* descs, const int64_t* offsets,
                              const int64_t* counts, int np, const LaunchCfg& cfg, BatchState* b,
                              std::vector<BatchPlan>* plans) {
    plans->resize(np);
    int64_t total = 0;
    int32_t nbuf = 0;
    b->kmax = 2;
    for (int i = 0; i < np; ++i) {
        int64_t n_all = 0;
        const int2* roots = pick_roots(g, descs[i].root_cut, &n_all);
        // offsets and counts are in the plan's task space (split roots count once per task)
        const SplitPlan sp = descs[i].iep ? SplitPlan{} : split_plan(g, descs[i], cfg, MODE_PLAIN, n_all, 1, 0);
        const int64_t n_tasks = n_all + sp.roots * (sp.ways - 1);
        int64_t off = offsets ? offsets[i] : 0;
        int64_t cnt = counts ? counts[i] : n_tasks;
        if (off < 0 || cnt < 0) return GP_ERR_ARG;
        off = std::min(off, n_tasks);
        cnt = std::min(cnt, n_tasks - off);
        (*plans)[i].roots = roots;
        (*plans)[i].n_tasks = cnt;
        (*plans)[i].task_begin = total;
        (*plans)[i].task_offset = off;
        (*plans)[i].split_roots = sp.roots;
        (*plans)[i].split_ways = sp.ways;
        (*plans)[i].leaf = b->leaf;
        total += cnt;
        nbuf = std::max(nbuf, descs[i].nbuf);
        b->kmax = std::max(b->kmax, (int)descs[i].k);
    }
    b->np = np;
    b->total_tasks = total;
    b->nbuf = nbuf;
    return GP_OK;
}

static int64_t batch_blocks(const DeviceGraph& g, const BatchState& b, int waves_per_cu, int32_t nbuf,
                            int64_t total) {
    const int64_t groups_per_block = kBlock / b.group;
    int64_t blocks = std::max<int64_t>(1, (int64_t)g.num_cus * waves_per_cu / (kBlock / 64));
    if (nbuf > 0) {
        const int64_t budget = int64_t(16) << 30;
        blocks = std::min(blocks, std::max<int64_t>(1, budget / (groups_per_block * nbuf * b.cap * 4)));
    }
    const int64_t need = (total + b.chunk - 1) / b.chunk;
    return std::min(blocks, std::max<int64_t>(1, (need + groups_per_block - 1) / groups_per_block));
}

gp_status batch_prepare(const DeviceGraph& g, const GpPlanDesc* descs, const int* leafs,
                        const int64_t* offsets, const int64_t* counts, int np,
                        const LaunchCfg& cfg, hipStream_t stream, BatchState* st) {
    (void)leafs;
    if (np < 1 || np > kBatchMaxPlans) return GP_ERR_ARG;
    BatchState b;
    b.group = cfg.group >= 64 ? 64 : (cfg.group >= 32 || cfg.group <= 0 ? 32 : 16);
    b.leaf = cfg.leaf == 3 || cfg.leaf == 4 ? cfg.leaf : 1;
    b.chunk = std::max(1, cfg.chunk);
    b.cap = std::max<int64_t>(1, g.deg2);
    std::vector<BatchPlan> plans;
    gp_status rc = batch_layout(g, descs, offsets, counts, np, cfg, &b, &plans);
    if (rc != GP_OK) return rc;
    const int64_t groups_per_block = kBlock / b.group;
    b.blocks = batch_blocks(g, b, cfg.waves_per_cu, b.nbuf, b.total_tasks);
    if (hipMalloc(&b.descs, sizeof(GpPlanDesc) * np) != hipSuccess ||
        hipMalloc(&b.plans, sizeof(BatchPlan) * np) != hipSuccess ||
        hipMalloc((void**)&b.queue, sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc((void**)&b.result, 3 * sizeof(unsigned long long) * np) != hipSuccess ||
        (b.nbuf > 0 &&
         hipMalloc((void**)&b.scratch, (size_t)(b.blocks * groups_per_block * b.nbuf * b.cap * 4)) != hipSuccess))
        rc = GP_ERR_NOMEM;
    if (rc == GP_OK &&
        (hipMemcpyAsync(b.descs, descs, sizeof(GpPlanDesc) * np, hipMemcpyHostToDevice, stream) != hipSuccess ||
         hipMemcpyAsync(b.plans, plans.data(), sizeof(BatchPlan) * np, hipMemcpyHostToDevice, stream) !=
             hipSuccess ||
         hipStreamSynchronize(stream) != hipSuccess))
        rc = GP_ERR_HIP;
    if (rc != GP_OK) {
        batch_release(&b);
        return rc;
    }
    *st = b;
    return GP_OK;
}

gp_status batch_enqueue(const DeviceGraph& g, const BatchState& st, hipStream_t stream) {
    BatchFn fn = pick_batch_kernel(st.group, st.kmax, st.leaf);
    hipLaunchKernelGGL(init_counters, dim3(1), dim3(64), 0, stream, st.queue, 1);
    for (int i = 0; i < 3 * st.np; i += 64)
        hipLaunchKernelGGL(init_counters, dim3(1), dim3(64), 0, stream, st.result + i,
                           std::min(64, 3 * st.np - i));
    BatchArgs a;
    a.row_ptr = g.row_ptr;
    a.col = g.col;
    a.descs = (const GpPlanDesc*)st.descs;
    a.plans = (const BatchPlan*)st.plans;
    a.np = st.np;
    a.total_tasks = st.total_tasks;
    a.hub_bits = g.hub_bits;
    a.hub_words = g.hub_words;
    a.n_hubs = g.n_hubs;
    a.scratch = st.scratch;
    a.buf_cap = st.cap;
    a.nbuf = st.nbuf;
    a.queue = st.queue;
    a.result = st.result;
    a.chunk = st.chunk;
    if (st.total_tasks > 0)
        hipLaunchKernelGGL(fn, dim3((unsigned)st.blocks), dim3(kBlock), 0, stream, a);
    return hipGetLastError() == hipSuccess ? GP_OK : GP_ERR_HIP;
}

gp_status arena_create(const DeviceGraph& g, int nbuf_cap, const LaunchCfg& cfg, BatchArena* ar) {
    BatchArena a;
    a.cfg = cfg;
    BatchState& b = a.st;
    b.group = cfg.group >= 64 ? 64 : (cfg.group >= 32 || cfg.group <= 0 ? 32 : 16);
    b.leaf = cfg.leaf == 3 || cfg.leaf == 4 ? cfg.leaf : 1;
    b.chunk = std::max(1, cfg.chunk);
    b.cap = std::max<int64_t>(1, g.deg2);
    a.nbuf_cap = std::max(0, std::min(nbuf_cap, GP_DESC_MAX_BUILDS));
    a.blocks_cap = batch_blocks(g, b, cfg.waves_per_cu, a.nbuf_cap, INT64_MAX / 4);
    const int64_t groups_per_block = kBlock / b.group;
    bool ok = hipMalloc(&b.descs, sizeof(GpPlanDesc) * kBatchMaxPlans) == hipSuccess &&
              hipMalloc(&b.plans, sizeof(BatchPlan) * kBatchMaxPlans) == hipSuccess &&
              hipMalloc((void**)&b.queue, sizeof(unsigned long long)) == hipSuccess &&
              hipMalloc((void**)&b.result, 3 * sizeof(unsigned long long) * kBatchMaxPlans) == hipSuccess &&
              (a.nbuf_cap == 0 ||
               hipMalloc((void**)&b.scratch,
                         (size_t)(a.blocks_cap * groups_per_block * a.nbuf_cap * b.cap * 4)) == hipSuccess) &&
              hipHostMalloc((void**)&a.h_descs, sizeof(GpPlanDesc) * kBatchMaxPlans, hipHostMallocDefault) ==
                  hipSuccess &&
              hipHostMalloc(&a.h_plans, sizeof(BatchPlan) * kBatchMaxPlans, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void**)&a.h_result, 3 * sizeof(unsigned long long) * kBatchMaxPlans,
                            hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        arena_release(&a);
        return GP_ERR_NOMEM;
    }
    *ar = a;
    return GP_OK;
}

gp_status arena_launch(const DeviceGraph& g, BatchArena* ar, const GpPlanDesc* descs, const int64_t* offsets,
                       const int64_t* counts, int np, hipStream_t stream) {
    if (np < 1 || np > kBatchMaxPlans) return GP_ERR_ARG;
    BatchState& b = ar->st;
    std::vector<BatchPlan> plans;
    gp_status rc = batch_layout(g, descs, offsets, counts, np, ar->cfg, &b, &plans);
    if (rc != GP_OK) return rc;
    if (b.nbuf > ar->nbuf_cap) return GP_ERR_NOMEM;
    // the scratch was carved for nbuf_cap slots per group; any smaller nbuf fits
    b.blocks = std::min(ar->blocks_cap, batch_blocks(g, b, ar->cfg.waves_per_cu, b.nbuf, b.total_tasks));
    if (b.nbuf > 0) {
        const int64_t groups_per_block = kBlock / b.group;
        const int64_t fit = ar->blocks_cap * groups_per_block * ar->nbuf_cap / (groups_per_block * b.nbuf);
        b.blocks = std::min(b.blocks, std::max<int64_t>(1, fit));
    }
    std::memcpy(ar->h_descs, descs, sizeof(GpPlanDesc) * np);
    std::memcpy(ar->h_plans, plans.data(), sizeof(BatchPlan) * np);
    GP_HIP_TRY(hipMemcpyAsync(b.descs, ar->h_descs, sizeof(GpPlanDesc) * np, hipMemcpyHostToDevice, stream));
    GP_HIP_TRY(hipMemcpyAsync(b.plans, ar->h_plans, sizeof(BatchPlan) * np, hipMemcpyHostToDevice, stream));
    rc = batch_enqueue(g, b, stream);
    if (rc != GP_OK) return rc;
    GP_HIP_TRY(hipMemcpyAsync(ar->h_result, b.result, 3 * sizeof(unsigned long long) * np, hipMemcpyDeviceToHost,
                              stream));
    return GP_OK;
}

void arena_release(BatchArena* ar) {
    batch_release(&ar->st);
    if (ar->h_descs) (void)hipHostFree(ar->h_descs);
    if (ar->h_plans) (void)hipHostFree(ar->h_plans);
    if (ar->h_result) (void)hipHostFree(ar->h_result);
    *ar = BatchArena{};
}

}  // namespace gpint
