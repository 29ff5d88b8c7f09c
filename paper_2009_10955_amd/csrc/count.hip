// Host side of the counting kernel: launch geometry, scratch, dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "count_kernel.hpp"

namespace gpcount {
KernelFn pick_kernel_k2(int group, int leaf, int mode, int iep);
KernelFn pick_kernel_k3(int group, int leaf, int mode, int iep);
KernelFn pick_kernel_k4(int group, int leaf, int mode, int iep);
KernelFn pick_kernel_k5(int group, int leaf, int mode, int iep);
KernelFn pick_kernel_k6(int group, int leaf, int mode, int iep);
KernelFn pick_kernel_k7(int group, int leaf, int mode, int iep);
KernelFn pick_kernel_k8(int group, int leaf, int mode, int iep);
BatchFn batch_kernel_k2_2(int group, int leaf, int iep);
BatchFn batch_kernel_k3_3(int group, int leaf, int iep);
BatchFn batch_kernel_k4_4(int group, int leaf, int iep);
BatchFn batch_kernel_k5_5(int group, int leaf, int iep);
BatchFn batch_kernel_k6_6(int group, int leaf, int iep);
BatchFn batch_kernel_k7_8(int group, int leaf, int iep);

// The batched kernel of a run whose plans have k in [kmin, kmax]: one pattern
// size up to 6, or sizes 7 and 8.
BatchFn pick_batch_kernel(int kmin, int kmax, int group, int leaf, int iep) {
    if (kmin == kmax) {
        switch (kmin) {
            case 2: return batch_kernel_k2_2(group, leaf, iep);
            case 3: return batch_kernel_k3_3(group, leaf, iep);
            case 4: return batch_kernel_k4_4(group, leaf, iep);
            case 5: return batch_kernel_k5_5(group, leaf, iep);
            case 6: return batch_kernel_k6_6(group, leaf, iep);
            default: break;
        }
    }
    if (kmin >= 7 && kmax <= 8) return batch_kernel_k7_8(group, leaf, iep);
    return nullptr;
}

namespace {
__global__ void init_counters(unsigned long long* p, int n) {
    int i = threadIdx.x;
    if (i < n) p[i] = 0;
}

// A solo batch run's high count word into its plan's result words.
__global__ void move_high_word(const unsigned long long* from, unsigned long long* to) {
    if (threadIdx.x == 0) *to = *from;
}

KernelFn pick_kernel(int k, int group, int leaf, int mode, int iep) {
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
// IEP plans: some inner set is left unbuilt as N(a) & N(x) with a an outer
// vertex's list and no cut, so its size depends on (a, x) alone and the
// kernel keeps it in a table shared by the launch's groups
// (count_kernel.hpp, iep_subset_count).
bool iep_memo_eligible(const GpPlanDesc& d) {
    if (!d.iep) return false;
    for (int j = d.k - d.iep; j < d.k; ++j) {
        const GpLevel& lv = d.lv[j];
        if (lv.last_list >= 0 && lv.pre_buf < 0 && lv.pre_list >= 0 && (lv.hi_src | lv.lo_src) == 0) return true;
    }
    return false;
}

// log2 of the IEP memo's words per hub: the most ways, up to
// kIepMemoWaysMax, whose table of n_hubs x ways words fits words_cap
// words; -1 if not even one way fits.
int iep_memo_log2(int64_t n_hubs, int64_t words_cap) {
    if (n_hubs <= 0 || words_cap < n_hubs) return -1;
    int l = 0;
    while ((int64_t(2) << l) <= kIepMemoWaysMax && (n_hubs << (l + 1)) <= words_cap) ++l;
    return l;
}

bool memo_eligible(const GpPlanDesc& d) {
    if (d.k < 4 || d.iep) return false;
    const GpLevel& ll = d.lv[d.k - 1];
    if (ll.last_list != d.k - 2 || ll.pre_buf >= 0 || ll.pre_list < 0 || ll.pre_list > 1) return false;
    if ((ll.hi_src | ll.lo_src) & ~3u) return false;
    return (ll.inj & ~(uint32_t)d.lv[d.k - 2].parents) == 0;
}

// The count's last step: the 128-bit total (queue[1], result[0]) divided by
// the IEP over-count (1 for plain counts), with the overflow flag set only if
// the quotient does not fit in 64 bits; check: flag a remainder (a whole
// count must divide exactly).
__global__ void finish_count(unsigned long long* result, const unsigned long long* queue, unsigned long long div,
                             int check) {
    if (threadIdx.x == 0) {
        const unsigned long long flags = result[1];
        finish128(&result[0], &result[1], queue[1], div);
        if (!check) result[1] = (result[1] & ~2ull) | (flags & 2ull);
    }
}

// The counting kernels' accumulation on given values: each lane adds its
// share with add_count (carries counted), the wavefronts sum exactly in 128
// bits and publish into w[2] (low word) and w[1] (high word), as a count's
// wavefronts publish into result[0] and queue[1].
__global__ void sum_check_kernel(const unsigned long long* vals, int64_t n, unsigned long long* w) {
    uint64_t acc = 0, carry = 0;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step)
        add_count(acc, vals[i], carry);
    wave_sum128(acc, carry);
    if (__lane_id() == 0) publish128(&w[2], &w[1], acc, carry);
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

int resident_waves_per_cu(const DeviceGraph& g, const GpPlanDesc& d, const LaunchCfg& cfg) {
    const bool iep = d.iep != 0;
    const int group = iep ? (cfg.group >= 64 ? 64 : 32) : cfg.group;
    KernelFn fn = pick_kernel(d.k, group, cfg.leaf, MODE_PLAIN, d.iep);
    (void)g;
    int nb = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)fn, kBlock, 0) != hipSuccess || nb <= 0)
        return cfg.waves_per_cu;
    return std::min(cfg.waves_per_cu, nb * (kBlock / 64));
}

int64_t xcd_block_tasks(const DeviceGraph& g, const LaunchCfg& cfg, int group) {
    (void)g;
    (void)group;
    if (cfg.xcd <= 0) return 0;  // the default: one cursor (measured faster)
    const int64_t chunk = std::max(1, cfg.chunk);
    return (cfg.xcd + chunk - 1) / chunk * chunk;
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
        if (l->xcd_tasks) cfg.xcd = l->xcd_tasks;
        if (l->batch_runs) cfg.batch_runs = l->batch_runs;
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
// Per-root counts stay one task per root, and so do patterns with no level-2
// loop (k <= 3, or IEP over every level after the root).
struct SplitPlan {
    int64_t roots = 0;
    int ways = 1;
};

static SplitPlan split_plan(const DeviceGraph& g, const GpPlanDesc& d, const LaunchCfg& cfg, int mode,
                            int64_t n_roots, int64_t stride, int64_t offset) {
    SplitPlan sp;
    if (mode == MODE_PER_ROOT || d.k < 4 || (d.iep && d.iep == d.k - 2) || cfg.split_ways <= 1 ||
        cfg.split_vertices <= 0)
        return sp;
    int i = 0;
    while (i < 31 && (int64_t(1) << (i + 1)) <= cfg.split_vertices) ++i;
    const int64_t pref = g.upper_pref[i] * (d.root_cut == 0 ? 2 : 1);
    const int64_t sampled = pref > offset ? (pref - offset + stride - 1) / stride : 0;
    sp.roots = std::min(n_roots, sampled);
    sp.ways = cfg.split_ways;
    return sp;
}

int64_t task_count(const DeviceGraph& g, const GpPlanDesc& d, const LaunchCfg& cfg) {
    int64_t n = 0;
    (void)pick_roots(g, d.root_cut, &n);
    const SplitPlan sp = split_plan(g, d, cfg, MODE_PLAIN, n, 1, 0);
    return n + sp.roots * (sp.ways - 1);
}

namespace {
constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
}  // namespace

gp_status launch_count(const DeviceGraph& g, const GpPlanDesc& d, const LaunchCfg& cfg,
                       hipStream_t stream, unsigned long long* result_dev,
                       unsigned long long* per_root, bool account, unsigned long long* busy,
                       const Workspace* ws) {
    if (cfg.group != 64 && cfg.group != 32 && cfg.group != 16 && cfg.group != 8) return GP_ERR_ARG;
    if (cfg.leaf < 1 || cfg.leaf > 4) return GP_ERR_ARG;
    if (cfg.waves_per_cu < 1 || cfg.waves_per_cu > 32 || cfg.chunk < 1) return GP_ERR_ARG;
    const int mode = account ? MODE_ACCOUNT : (per_root ? MODE_PER_ROOT : MODE_PLAIN);
    const bool iep = d.iep != 0;
    const int group = iep ? (cfg.group >= 64 ? 64 : 32) : cfg.group;  // IEP kernels: 64 or 32 lanes
    KernelFn fn = pick_kernel(d.k, group, cfg.leaf, mode, d.iep);
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
    const int64_t cap = std::max<int64_t>(1, g.deg2);
    const int64_t per_block = d.nbuf > 0 ? groups_per_block * d.nbuf * cap * 4 : 0;
    // keep scratch within a fixed budget (or the caller's workspace): fewer
    // resident groups if needed
    const int64_t budget = ws ? (int64_t)ws->bytes - (int64_t)kAlign : int64_t(16) << 30;
    if (ws && budget < 0) return GP_ERR_ARG;
    if (per_block > 0) {
        if (ws && per_block > budget) return GP_ERR_NOMEM;  // not even one block's buffers fit
        blocks = std::min(blocks, std::max<int64_t>(1, budget / per_block));
    }
    // a grid larger than the number of root tasks only adds idle groups
    int64_t need = (n_tasks + cfg.chunk - 1) / cfg.chunk;
    int64_t need_blocks = std::max<int64_t>(1, (need + groups_per_block - 1) / groups_per_block);
    blocks = std::min(blocks, need_blocks);

    const size_t scratch_bytes = (size_t)(blocks * per_block);
    // leaf mode 4's per-task memo: one word per hub per group, within 4 GiB
    // (within what the workspace has left); the IEP memo: one table for the
    // launch, 2^l words per hub, within 2 GiB (or the room left)
    const int64_t memo_cap = ws ? budget - (int64_t)align_up(scratch_bytes) : (int64_t(4) << 30);
    const int iep_log2 =
        iep && iep_memo_eligible(d) ? iep_memo_log2(g.n_hubs, std::min(memo_cap, kIepMemoBytes) / 8) : -1;
    const int64_t memo_words = iep ? (iep_log2 >= 0 ? (int64_t)g.n_hubs << iep_log2 : 0)
                                   : blocks * groups_per_block * (int64_t)g.n_hubs;
    const bool leaf4_memo = cfg.leaf == 4 && mode != MODE_PER_ROOT && !iep && memo_eligible(d) &&
                            n_tasks < (int64_t(1) << 31);
    const bool use_memo = (leaf4_memo || iep_log2 >= 0) && g.n_hubs > 0 && memo_words * 8 <= memo_cap;

    int32_t* scratch = nullptr;
    unsigned long long* queue = nullptr;
    unsigned long long* memo = nullptr;
    if (ws) {
        char* base = (char*)ws->base;
        queue = (unsigned long long*)base;
        if (scratch_bytes) scratch = (int32_t*)(base + kAlign);
        if (use_memo) memo = (unsigned long long*)(base + kAlign + align_up(scratch_bytes));
    } else {
        GP_HIP_TRY(hipMallocAsync((void**)&queue, sizeof(unsigned long long) * kQueueWords, stream));
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
        }
    }
    if (use_memo)
        hipLaunchKernelGGL(zero_u64, dim3((unsigned)std::min<int64_t>(4096, (memo_words + 255) / 256)), dim3(256), 0,
                           stream, memo, memo_words);
    hipLaunchKernelGGL(init_counters, dim3(1), dim3(64), 0, stream, queue, kQueueWords);
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
    a.memo_ways_log2 = std::max(iep_log2, 0);
    a.xcd_block = xcd_block_tasks(g, cfg, group);
    if (n_tasks > 0)
        hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(kBlock), 0, stream, d, a);
    // a sample's total need not be a multiple of the over-count: its quotient
    // is an estimate, not checked
    const bool whole = cfg.root_stride == 1 && cfg.root_offset == 0 && !(busy && cfg.budget_ms > 0);
    hipLaunchKernelGGL(finish_count, dim3(1), dim3(64), 0, stream, result_dev, queue,
                       (unsigned long long)(iep ? d.iep_div : 1), whole ? 1 : 0);
    hipError_t le = hipGetLastError();
    if (!ws) {
        if (scratch) (void)hipFreeAsync(scratch, stream);
        if (memo) (void)hipFreeAsync(memo, stream);
        (void)hipFreeAsync(queue, stream);
    }
    if (le != hipSuccess) return GP_ERR_HIP;
    return GP_OK;
}

gp_status check_sum(const uint64_t* values, int64_t n, uint64_t div, hipStream_t stream, uint64_t* out,
                    uint32_t* flags) {
    if (n < 0 || (n > 0 && !values) || div < 1) return GP_ERR_ARG;
    unsigned long long* w = nullptr;  // {cursor (unused), high word, low word, flags}, then the values
    GP_HIP_TRY(hipMallocAsync((void**)&w, sizeof(unsigned long long) * (4 + (size_t)n), stream));
    unsigned long long h[4] = {0, 0, 0, 0};
    hipError_t e = hipSuccess;
    hipLaunchKernelGGL(init_counters, dim3(1), dim3(64), 0, stream, w, 4);
    if (n > 0)
        e = hipMemcpyAsync(w + 4, values, sizeof(unsigned long long) * (size_t)n, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(sum_check_kernel, dim3(4), dim3(kBlock), 0, stream, w + 4, n, w);
        hipLaunchKernelGGL(finish_count, dim3(1), dim3(64), 0, stream, w + 2, w, (unsigned long long)div, 1);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(h, w, sizeof h, hipMemcpyDeviceToHost, stream);
    (void)hipFreeAsync(w, stream);
    if (hipStreamSynchronize(stream) != hipSuccess || e != hipSuccess) return GP_ERR_HIP;
    *out = h[2];
    *flags = (uint32_t)h[3];
    return GP_OK;
}

// Workspace of launch_count_noalloc: every GPU the library runs on holds one
// copy of this array until the process ends. In host code its name is only a
// stand-in; the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device.
static __device__ __align__(256) unsigned char scratch[kNoallocWorkspaceBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};
}  // namespace

// The device address of this GPU's copy of `scratch` (the device must be
// current), looked up on the first call per device.
static gp_status scratch_address(int device, void** ptr) {
    if (device < 0 || device >= 64) return GP_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GP_ERR_HIP;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return GP_OK;
}

gp_status launch_count_noalloc(const DeviceGraph& g, const GpPlanDesc& d, const LaunchCfg& cfg,
                               hipStream_t stream, unsigned long long* result_dev) {
    void* base = nullptr;
    const gp_status st = scratch_address(g.device, &base);
    if (st != GP_OK) return st;
    Workspace ws;
    ws.base = base;
    ws.bytes = kNoallocWorkspaceBytes;
    return launch_count(g, d, cfg, stream, result_dev, nullptr, false, nullptr, &ws);
}

int64_t root_task_count(const DeviceGraph& g, const GpPlanDesc& d) {
    int64_t n = 0;
    (void)pick_roots(g, d.root_cut, &n);
    return n;
}

void batch_release(BatchState* st) {
    (void)hipFree(st->scratch);
    (void)hipFree(st->memo);
    (void)hipFree(st->queues);
    (void)hipFree(st->result);
    (void)hipFree(st->run_queues);
    *st = BatchState{};
}

// A plan's shape inside a batch: IEP plans run in 64- or 32-lane groups,
// others in 64, 32, 16 or 8 (floored at min_group); leaf modes 1, 3 or 4 (2
// runs as 1).
static void batch_shape(const GpPlanDesc& d, const LaunchCfg& c, int min_group, BatchPlan* bp) {
    const int want = std::max(c.group, min_group);
    if (d.iep) bp->group = want >= 64 ? 64 : 32;
    else bp->group = want >= 64 ? 64 : (want >= 32 ? 32 : (want >= 16 ? 16 : 8));
    bp->leaf = d.iep ? 1 : (c.leaf == 3 || c.leaf == 4 ? c.leaf : 1);
    bp->chunk = std::max(1, c.chunk);
}

int batch_shape_key(const GpPlanDesc& d, const LaunchCfg& c, int min_group) {
    BatchPlan bp;
    batch_shape(d, c, min_group, &bp);
    return (std::min(d.k, 7) << 16) | (bp.group << 8) | (bp.leaf << 4) | d.iep;
}

// The host copy of a batch's plan table (launches pass it by value).
static void store_plans(BatchState* b, const std::vector<BatchPlan>& plans) {
    b->h_plans.assign((const char*)plans.data(), (const char*)(plans.data() + plans.size()));
}

// Per-plan task ranges, shapes and the launch geometry for np plans.
static gp_status batch_layout(const DeviceGraph& g, const GpPlanDesc* descs, const LaunchCfg* cfgs,
                              const int64_t* offsets, const int64_t* counts, int np, int min_group_floor,
                              BatchState* b, std::vector<BatchPlan>* plans) {
    plans->resize(np);
    b->runs.clear();
    std::vector<int64_t> nroots(np, 0);
    std::vector<bool> whole(np, false);
    int32_t nbuf = 0;
    b->kmax = 2;
    int64_t tag_next = 1;  // memo tags of the eligible plans: disjoint ranges
    bool any_memo = false;
    for (int i = 0; i < np; ++i) {
        int64_t n_all = 0;
        const int2* roots = pick_roots(g, descs[i].root_cut, &n_all);
        // a strided root sample per plan, as in launch_count
        const int64_t stride = std::max<int64_t>(1, cfgs[i].root_stride);
        const int64_t roff = std::max<int64_t>(0, cfgs[i].root_offset);
        const int64_t n_sampled = n_all > roff ? (n_all - roff + stride - 1) / stride : 0;
        // offsets and counts are in the plan's task space (split roots count once per task)
        const SplitPlan sp = split_plan(g, descs[i], cfgs[i], MODE_PLAIN, n_sampled, stride, roff);
        const int64_t n_tasks = n_sampled + sp.roots * (sp.ways - 1);
        int64_t off = offsets ? offsets[i] : 0;
        int64_t cnt = counts ? counts[i] : n_tasks;
        if (off < 0 || cnt < 0) return GP_ERR_ARG;
        off = std::min(off, n_tasks);
        cnt = std::min(cnt, n_tasks - off);
        whole[i] = off == 0 && cnt == n_tasks;
        nroots[i] = n_sampled;
        BatchPlan& bp = (*plans)[i];
        std::memset(&bp, 0, sizeof bp);
        bp.roots = roots;
        bp.root_offset = roff;
        bp.root_stride = stride;
        bp.n_tasks = cnt;
        bp.task_offset = off;
        bp.split_roots = sp.roots;
        bp.split_ways = sp.ways;
        batch_shape(descs[i], cfgs[i], min_group_floor, &bp);
        // consecutive plans of one shape share a launch (up to kRunMaxPlans:
        // their descriptors are its kernel arguments)
        const int iep_depth = descs[i].iep;
        const int ksize = std::min((int)descs[i].k, 7);  // sizes 7 and 8 share a kernel
        if (b->runs.empty() || b->runs.back().group != bp.group || b->runs.back().leaf != bp.leaf ||
            b->runs.back().iep != iep_depth || std::min(b->runs.back().kmin, 7) != ksize ||
            b->runs.back().p1 - b->runs.back().p0 >= kRunMaxPlans || cfgs[i].batch_runs == 2) {
            BatchRun r;
            r.p0 = i;
            r.group = bp.group;
            r.leaf = bp.leaf;
            r.iep = iep_depth;
            r.kmin = r.kmax = descs[i].k;
            b->runs.push_back(r);
        }
        b->runs.back().p1 = i + 1;
        b->runs.back().kmin = std::min(b->runs.back().kmin, (int)descs[i].k);
        b->runs.back().kmax = std::max(b->runs.back().kmax, (int)descs[i].k);
        b->runs.back().waves_per_cu = std::max(b->runs.back().waves_per_cu, cfgs[i].waves_per_cu);
        bp.tag_base = 0;
        if (bp.leaf == 4 && !descs[i].iep && g.n_hubs > 0 && memo_eligible(descs[i]) &&
            tag_next + n_all < (int64_t(1) << 31) - 1) {  // below the IEP memo's tags
            bp.tag_base = (uint32_t)tag_next - 1;  // tags tag_base + root + 1 >= tag_next
            tag_next += n_all;
            any_memo = true;
        }
        // an IEP plan run alone keeps its inner set sizes in the same region
        if (descs[i].iep && g.n_hubs > 0 && iep_memo_eligible(descs[i])) any_memo = true;
        nbuf = std::max(nbuf, descs[i].nbuf);
        b->kmax = std::max(b->kmax, (int)descs[i].k);
    }
    b->np = np;
    b->nbuf = nbuf;
    b->use_memo = any_memo;
    for (BatchRun& r : b->runs) {
        const BatchPlan& bp = (*plans)[r.p0];
        r.solo = r.p1 - r.p0 == 1 && whole[r.p0] && bp.tag_base == 0 && r.kmin == r.kmax;
        r.roots = bp.roots;
        r.n_roots = nroots[r.p0];
        r.root_offset = bp.root_offset;
        r.root_stride = bp.root_stride;
        r.n_tasks = bp.n_tasks;
        r.split_roots = bp.split_roots;
        r.split_ways = bp.split_ways;
        r.chunk = bp.chunk;
    }
    b->h_descs.assign(descs, descs + np);
    store_plans(b, *plans);
    return GP_OK;
}

// Wavefront-resident blocks: the device's share, within the scratch and memo
// budgets. Scratch per wavefront: slots_per_wave groups x nbuf x cap int32.
static int64_t batch_blocks(const DeviceGraph& g, int waves_per_cu, int slots_per_wave, int32_t nbuf, int64_t cap,
                            bool memo) {
    const int waves_per_block = kBlock / 64;
    int64_t blocks = std::max<int64_t>(1, (int64_t)g.num_cus * waves_per_cu / waves_per_block);
    if (nbuf > 0) {
        const int64_t budget = int64_t(16) << 30;
        blocks = std::min(blocks, std::max<int64_t>(1, budget / ((int64_t)waves_per_block * slots_per_wave * nbuf *
                                                                  cap * 4)));
    }
    if (memo && g.n_hubs > 0) {
        const int64_t budget = int64_t(4) << 30;
        blocks = std::min(blocks, std::max<int64_t>(1, budget / ((int64_t)waves_per_block * slots_per_wave *
                                                                  g.n_hubs * 8)));
    }
    return blocks;
}

// Group slots (scratch and memo tables) a run's launch addresses.
static int64_t run_group_slots(const BatchRun& r) { return r.blocks * (kBlock / 64) * (64 / r.group); }

gp_status batch_prepare(const DeviceGraph& g, const GpPlanDesc* descs, const LaunchCfg* cfgs,
                        const int64_t* offsets, const int64_t* counts, int np, int waves_per_cu,
                        hipStream_t stream, BatchState* st) {
    if (np < 1 || np > kBatchMaxPlans) return GP_ERR_ARG;
    BatchState b;
    b.cap = std::max<int64_t>(1, g.deg2);
    std::vector<BatchPlan> plans;
    gp_status rc = batch_layout(g, descs, cfgs, offsets, counts, np, 8, &b, &plans);
    if (rc != GP_OK) return rc;
    // every run at its own width and residency; the regions fit the largest
    int64_t slots = 0;
    for (BatchRun& r : b.runs) {
        r.blocks = batch_blocks(g, std::min(waves_per_cu, r.waves_per_cu), 64 / r.group, b.nbuf, b.cap, b.use_memo);
        slots = std::max(slots, run_group_slots(r));
    }
    b.memo_words = b.use_memo ? slots * (int64_t)g.n_hubs : 0;
    // room for the IEP memo's most ways when an eligible IEP plan runs alone
    for (const BatchRun& r : b.runs)
        for (int p = r.p0; p < r.p1 && b.use_memo; ++p)
            if (r.solo && descs[p].iep && iep_memo_eligible(descs[p])) {
                const int l = iep_memo_log2(g.n_hubs, kIepMemoBytes / 8);
                if (l >= 0) b.memo_words = std::max(b.memo_words, (int64_t)g.n_hubs << l);
            }
    if (hipMalloc((void**)&b.queues, sizeof(unsigned long long) * np) != hipSuccess ||
        hipMalloc((void**)&b.run_queues, sizeof(unsigned long long) * kBatchMaxPlans * kQueueWords) != hipSuccess ||
        hipMalloc((void**)&b.result, 4 * sizeof(unsigned long long) * np) != hipSuccess ||
        (b.nbuf > 0 && hipMalloc((void**)&b.scratch, (size_t)(slots * b.nbuf * b.cap * 4)) != hipSuccess) ||
        (b.memo_words > 0 && hipMalloc((void**)&b.memo, (size_t)b.memo_words * 8) != hipSuccess))
        rc = GP_ERR_NOMEM;
    if (rc == GP_OK && hipStreamSynchronize(stream) != hipSuccess) rc = GP_ERR_HIP;
    if (rc != GP_OK) {
        batch_release(&b);
        return rc;
    }
    *st = b;
    return GP_OK;
}

gp_status batch_update(const DeviceGraph& g, BatchState* st, const GpPlanDesc* descs, const LaunchCfg* cfgs,
                       hipStream_t stream) {
    BatchState b = *st;
    std::vector<BatchPlan> plans;
    gp_status rc = batch_layout(g, descs, cfgs, nullptr, nullptr, st->np, 8, &b, &plans);
    if (rc != GP_OK) return rc;
    bool same = b.nbuf == st->nbuf && b.use_memo == st->use_memo && b.runs.size() == st->runs.size();
    for (size_t i = 0; same && i < b.runs.size(); ++i)
        same = b.runs[i].p0 == st->runs[i].p0 && b.runs[i].p1 == st->runs[i].p1 &&
               b.runs[i].group == st->runs[i].group && b.runs[i].leaf == st->runs[i].leaf &&
               b.runs[i].iep == st->runs[i].iep;
    if (!same) return GP_ERR_ARG;  // the shapes the buffers were carved for must not change
    (void)stream;
    // launches take their task ranges as kernel arguments: the caller
    // enqueues (or captures) the batch again
    for (size_t i = 0; i < b.runs.size(); ++i) b.runs[i].blocks = st->runs[i].blocks;  // the carved grids
    st->runs = b.runs;
    st->h_plans = b.h_plans;
    return GP_OK;
}

gp_status batch_enqueue(const DeviceGraph& g, const BatchState& st, hipStream_t stream) {
    if (st.runs.empty()) return GP_ERR_ARG;
    for (const BatchRun& r : st.runs)
        if (!pick_batch_kernel(r.kmin, r.kmax, r.group, r.leaf, r.iep) || r.blocks < 1) return GP_ERR_UNSUPPORTED;
    for (int i = 0; i < st.np; i += 64)
        hipLaunchKernelGGL(init_counters, dim3(1), dim3(64), 0, stream, st.queues + i, std::min(64, st.np - i));
    for (int i = 0; i < 4 * st.np; i += 64)
        hipLaunchKernelGGL(init_counters, dim3(1), dim3(64), 0, stream, st.result + i,
                           std::min(64, 4 * st.np - i));
    if (st.memo_words > 0)
        hipLaunchKernelGGL(zero_u64, dim3((unsigned)std::min<int64_t>(4096, (st.memo_words + 255) / 256)), dim3(256),
                           0, stream, st.memo, st.memo_words);
    // one persistent launch per run of same-shape plans, in batch order. The
    // runs share the scratch and memo regions: launches on one stream never
    // overlap, and memo tags are disjoint per plan.
    for (size_t ri = 0; ri < st.runs.size(); ++ri) {
        const BatchRun& r = st.runs[ri];
        if (r.solo) {
            // the plain counting kernel over the plan's whole task space; its
            // queue words are the run's own, and the high count word is moved
            // into the plan's result words after it
            const int p = r.p0;
            const GpPlanDesc& d = st.h_descs[p];
            KernelFn fn = pick_kernel(d.k, r.group, r.leaf, MODE_PLAIN, d.iep);
            if (!fn) return GP_ERR_UNSUPPORTED;
            unsigned long long* q = st.run_queues + ri * kQueueWords;
            hipLaunchKernelGGL(init_counters, dim3(1), dim3(64), 0, stream, q, kQueueWords);
            CountArgs a;
            a.row_ptr = g.row_ptr;
            a.col = g.col;
            a.roots = r.roots;
            a.n_roots = r.n_roots;
            a.n_tasks = r.n_tasks;
            a.split_roots = r.split_roots;
            a.split_ways = r.split_ways;
            a.budget_ticks = 0;
            a.root_offset = r.root_offset;
            a.hub_bits = g.hub_bits;
            a.hub_words = g.hub_words;
            a.n_hubs = g.n_hubs;
            a.root_stride = r.root_stride;
            a.scratch = st.scratch;
            a.buf_cap = st.cap;
            a.queue = q;
            a.result = st.result + 4 * p;
            a.per_root = nullptr;
            a.busy = nullptr;
            // the IEP memo holds sizes fixed by the graph, valid in every
            // launch: the region needs no clearing between runs
            const int iep_log2 = d.iep && iep_memo_eligible(d) && st.memo_words > 0
                                     ? iep_memo_log2(g.n_hubs, std::min(st.memo_words, kIepMemoBytes / 8))
                                     : -1;
            a.memo = iep_log2 >= 0 ? st.memo : nullptr;
            a.memo_ways_log2 = std::max(iep_log2, 0);
            a.chunk = r.chunk;
            a.xcd_block = 0;
            if (r.n_tasks > 0)
                hipLaunchKernelGGL(fn, dim3((unsigned)r.blocks), dim3(kBlock), 0, stream, d, a);
            hipLaunchKernelGGL(move_high_word, dim3(1), dim3(64), 0, stream, q + 1, st.result + 4 * p + 3);
            continue;
        }
        BatchArgs a;
        a.row_ptr = g.row_ptr;
        a.col = g.col;
        a.np = r.p1 - r.p0;
        a.hub_bits = g.hub_bits;
        a.hub_words = g.hub_words;
        a.n_hubs = g.n_hubs;
        a.scratch = st.scratch;
        a.buf_cap = st.cap;
        a.nbuf = st.nbuf;
        a.slots_per_wave = 64 / r.group;
        a.memo = st.memo_words > 0 ? st.memo : nullptr;
        a.queues = st.queues + r.p0;
        a.result = st.result + 4 * r.p0;
        RunDescs rd;
        std::memset(&rd, 0, sizeof rd);
        for (int p = r.p0; p < r.p1; ++p) {
            rd.d[p - r.p0] = st.h_descs[p];
            rd.bp[p - r.p0] = reinterpret_cast<const BatchPlan*>(st.h_plans.data())[p];
        }
        hipLaunchKernelGGL(pick_batch_kernel(r.kmin, r.kmax, r.group, r.leaf, r.iep), dim3((unsigned)r.blocks), dim3(kBlock),
                           0, stream, a, rd);
    }
    return hipGetLastError() == hipSuccess ? GP_OK : GP_ERR_HIP;
}

gp_status arena_create(const DeviceGraph& g, int nbuf_cap, int waves_per_cu, int min_group, BatchArena* ar) {
    BatchArena a;
    a.waves_per_cu = waves_per_cu;
    BatchState& b = a.st;
    b.cap = std::max<int64_t>(1, g.deg2);
    a.min_group = min_group >= 64 ? 64 : (min_group >= 32 ? 32 : (min_group >= 16 ? 16 : 8));
    a.nbuf_cap = std::max(0, std::min(nbuf_cap, GP_DESC_MAX_BUILDS));
    // room for the smallest group width and for the memo of leaf-4 plans
    a.blocks_cap = batch_blocks(g, waves_per_cu, 64 / a.min_group, a.nbuf_cap, b.cap, true);
    a.slots_cap = a.blocks_cap * (kBlock / 64) * (64 / a.min_group);
    a.memo_words_cap = g.n_hubs > 0 ? a.slots_cap * (int64_t)g.n_hubs : 0;
    bool ok = hipMalloc((void**)&b.queues, sizeof(unsigned long long) * kBatchMaxPlans) == hipSuccess &&
              hipMalloc((void**)&b.run_queues, sizeof(unsigned long long) * kBatchMaxPlans * kQueueWords) ==
                  hipSuccess &&
              hipMalloc((void**)&b.result, 4 * sizeof(unsigned long long) * kBatchMaxPlans) == hipSuccess &&
              (a.nbuf_cap == 0 ||
               hipMalloc((void**)&b.scratch, (size_t)(a.slots_cap * a.nbuf_cap * b.cap * 4)) == hipSuccess) &&
              (a.memo_words_cap == 0 || hipMalloc((void**)&b.memo, (size_t)a.memo_words_cap * 8) == hipSuccess) &&
              hipHostMalloc((void**)&a.h_result, 4 * sizeof(unsigned long long) * kBatchMaxPlans,
                            hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        arena_release(&a);
        return GP_ERR_NOMEM;
    }
    *ar = a;
    return GP_OK;
}

gp_status arena_launch(const DeviceGraph& g, BatchArena* ar, const GpPlanDesc* descs, const LaunchCfg* cfgs,
                       const int64_t* offsets, const int64_t* counts, int np, hipStream_t stream) {
    if (np < 1 || np > kBatchMaxPlans) return GP_ERR_ARG;
    BatchState& b = ar->st;
    std::vector<BatchPlan> plans;
    gp_status rc = batch_layout(g, descs, cfgs, offsets, counts, np, ar->min_group, &b, &plans);
    if (rc != GP_OK) return rc;
    if (b.nbuf > ar->nbuf_cap) return GP_ERR_NOMEM;
    // each run within the regions carved at creation: group slots x nbuf
    // buffers of scratch, group slots x n_hubs memo words
    int64_t room = b.nbuf > 0 ? ar->slots_cap * ar->nbuf_cap / b.nbuf : ar->slots_cap;
    if (b.use_memo) room = std::min(room, ar->slots_cap);
    int64_t slots = 0;
    for (BatchRun& r : b.runs) {
        const int64_t per_block = (kBlock / 64) * (64 / r.group);
        r.blocks = batch_blocks(g, std::min(ar->waves_per_cu, r.waves_per_cu), 64 / r.group, b.nbuf, b.cap,
                                b.use_memo);
        r.blocks = std::max<int64_t>(1, std::min(r.blocks, room / per_block));
        slots = std::max(slots, run_group_slots(r));
    }
    b.memo_words = b.use_memo ? slots * (int64_t)g.n_hubs : 0;
    if (b.memo_words > ar->memo_words_cap) {
        // no room for every wave's table: run the leaf-4 plans without the memo
        for (auto& bp : plans) bp.tag_base = 0;
        b.memo_words = 0;
    }
    store_plans(&b, plans);
    rc = batch_enqueue(g, b, stream);
    if (rc != GP_OK) return rc;
    GP_HIP_TRY(hipMemcpyAsync(ar->h_result, b.result, 4 * sizeof(unsigned long long) * np, hipMemcpyDeviceToHost,
                              stream));
    return GP_OK;
}

gp_status batch_result(const GpPlanDesc& d, const unsigned long long* r, uint64_t* out, bool whole) {
    unsigned __int128 t = ((unsigned __int128)r[3] << 64) | (unsigned __int128)r[0];
    const uint64_t div = d.iep ? (uint64_t)d.iep_div : 1;
    if (div > 1) {
        // a whole count is a multiple of the over-count; a sample's need not be
        if (whole && t % div) return GP_ERR_INTERNAL;
        t /= div;
    }
    if (t >> 64) return GP_ERR_OVERFLOW;
    *out = (uint64_t)t;
    return GP_OK;
}

void arena_release(BatchArena* ar) {
    batch_release(&ar->st);
    if (ar->h_result) (void)hipHostFree(ar->h_result);
    *ar = BatchArena{};
}

}  // namespace gpint
