// Batched persistent kernels: several plans (patterns or configurations of
// uneven cost, any k, counted plainly or with inclusion-exclusion) over one
// graph, captured together in one hipGraph.
//
// Every plan keeps the launch shape tuned for it alone: lanes per group (64,
// 32, 16 or 8), leaf mode (1, 3 or 4) and inclusion-exclusion depth, plus its
// tasks per grab. The plans of one shape and one pattern size (k <= 6; sizes
// 7 and 8 share) run in ONE persistent launch of a kernel compiled for that
// shape and size only, with a task cursor per plan:
// wavefronts take the plans in order, grab a piece of the current plan's
// tasks (64/G groups, bp.chunk tasks each), and move to the next plan once
// its cursor is exhausted, so plans of uneven cost fill each other's tails
// (Section IV-E's task partitioning, across patterns). One kernel per shape,
// not one kernel for all shapes: a body that branches over several shapes
// keeps the register allocation of their union, and the spills that follow
// cost more than a launch (the same holds for pattern sizes). Per-plan
// 128-bit counts (and the wall-clock time spent on each plan, for the serving
// scheduler) are summed per wavefront in LDS and published once at the end.
// Built once per pattern size k <= 6 (-DGP_BATCH_KMIN=k -DGP_BATCH_KMAX=k)
// and once for sizes 7 and 8.
#include "count_kernel.hpp"

#if !defined(GP_BATCH_KMAX) || !defined(GP_BATCH_KMIN)
#error "GP_BATCH_KMIN and GP_BATCH_KMAX must be defined"
#endif

namespace gpcount {

namespace {

constexpr int KMIN = GP_BATCH_KMIN;
constexpr int KMAX = GP_BATCH_KMAX;

// Tasks [t0, t1) of plan bp (in the plan's own task space), shared by the
// wavefront's 64/G groups: group j takes the j-th run of bp.chunk tasks.
template <int G, int LEAF, int IEP>
__device__ void run_piece(const BatchArgs& a, const GpPlanDesc& d, const BatchPlan& bp, int64_t t0, int64_t t1,
                          int32_t* lens_base, int64_t wave_global, uint64_t& acc, uint64_t& carry) {
    Ctx<G> c;
    const int j = (threadIdx.x & 63) / G;
    c.row_ptr = a.row_ptr;
    c.col = a.col;
    c.cap = a.buf_cap;
    c.hub_bits = a.hub_bits;
    c.hub_words = a.hub_words;
    c.n_hubs = a.n_hubs;
    const int64_t slot = wave_global * a.slots_per_wave + j;
    c.bufs = a.scratch ? a.scratch + slot * (int64_t)a.nbuf * a.buf_cap : nullptr;
    c.lens = lens_base + j * GP_DESC_MAX_BUILDS;
    c.bytes = nullptr;
    c.sj = 0;
    c.sJ = 1;
    c.deadline = 0;
    c.memo = (a.memo && bp.tag_base) ? a.memo + slot * (int64_t)a.n_hubs : nullptr;
    c.tag = 0;
    c.memo_log2 = 0;
    TaskSpace ts;
    ts.roots = bp.roots;
    ts.offset = bp.root_offset;
    ts.stride = bp.root_stride;
    ts.split_roots = bp.split_roots;
    ts.split_ways = bp.split_ways;
    ts.tag_base = bp.tag_base;
    const int64_t a0 = t0 + (int64_t)j * bp.chunk;
    const int64_t a1 = min(a0 + (int64_t)bp.chunk, t1);
    if (a0 >= a1) return;
    switch (d.k) {
#define GP_BATCH_CASE(KK)                                                                                     \
    case KK:                                                                                                  \
        if constexpr (KK >= KMIN && KK <= KMAX) {                                                             \
            if constexpr (IEP > 0) {                                                                          \
                if constexpr (KK >= IEP + 2) run_tasks<KK, G, 1, MODE_PLAIN, IEP>(d, c, ts, a0, a1, acc, carry, nullptr); \
            } else {                                                                                          \
                constexpr int LF = (LEAF == 3 && KK >= 5) ? 3 : ((LEAF == 4 && KK >= 4) ? 4 : 1);             \
                run_tasks<KK, G, LF, MODE_PLAIN, 0>(d, c, ts, a0, a1, acc, carry, nullptr);                   \
            }                                                                                                 \
        }                                                                                                     \
        break;
        GP_BATCH_CASE(2)
        GP_BATCH_CASE(3)
        GP_BATCH_CASE(4)
        GP_BATCH_CASE(5)
        GP_BATCH_CASE(6)
        GP_BATCH_CASE(7)
        GP_BATCH_CASE(8)
#undef GP_BATCH_CASE
        default:
            break;
    }
}

template <int G, int LEAF, int IEP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(occupancy_target(KMAX, G, LEAF, IEP)))) void batch_kernel(BatchArgs a, RunDescs rd) {
    __shared__ int32_t s_len[kBlock / G][GP_DESC_MAX_BUILDS];
    __shared__ unsigned long long s_lo[kBlock / 64][kBatchMaxPlans];
    __shared__ unsigned long long s_hi[kBlock / 64][kBatchMaxPlans];
    __shared__ unsigned long long s_busy[kBlock / 64][kBatchMaxPlans];
    const int wave = threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    for (int p = lane; p < kBatchMaxPlans; p += 64) {
        s_lo[wave][p] = 0;
        s_hi[wave][p] = 0;
        s_busy[wave][p] = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const int64_t wave_global = (int64_t)blockIdx.x * (kBlock / 64) + wave;
    int32_t* lens_base = &s_len[wave * (64 / G)][0];
    constexpr int64_t kGroups = 64 / G;

    int p = 0;
    while (p < a.np) {
        const BatchPlan& bp = rd.bp[p];
        const int64_t W = kGroups * bp.chunk;
        unsigned long long q = 0;
        if (lane == 0) q = atomicAdd(&a.queues[p], (unsigned long long)W);
        const int64_t t0 = uni64<64>((int64_t)__shfl(q, 0, 64));
        const int64_t n_tasks = bp.n_tasks;
        if (t0 >= n_tasks) {
            ++p;
            continue;
        }
        const int64_t t1 = min(t0 + W, n_tasks);
        const GpPlanDesc& d = rd.d[p];
        const uint64_t clk0 = wall_clock64();
        uint64_t acc = 0, carry = 0;
        run_piece<G, LEAF, IEP>(a, d, bp, bp.task_offset + t0, bp.task_offset + t1, lens_base, wave_global, acc,
                                carry);
        // exact 128-bit wavefront sum into this wavefront's LDS counter of plan p
        wave_sum128(acc, carry);
        if (lane == 0) {
            const unsigned long long old = s_lo[wave][p];
            const unsigned long long lo = old + acc;
            s_lo[wave][p] = lo;
            s_hi[wave][p] += carry + (lo < old ? 1u : 0u);
            s_busy[wave][p] += (unsigned long long)(wall_clock64() - clk0);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    for (int i = lane; i < a.np; i += 64) {
        publish128(&a.result[4 * i], &a.result[4 * i + 3], s_lo[wave][i], s_hi[wave][i]);
        if (s_busy[wave][i]) atomicAdd(&a.result[4 * i + 2], s_busy[wave][i]);
    }
}

}  // namespace

#define GP_CAT2(a, b) a##b
#define GP_CAT(a, b) GP_CAT2(a, b)

// The kernel of one batch shape: group width 64/32/16/8 with leaf mode 1, 3 or
// 4 (IEP depth 0), or group width 64/32 with IEP depth 2..4 (leaf mode 1);
// null for any other shape.
BatchFn GP_CAT(GP_CAT(GP_CAT(batch_kernel_k, GP_BATCH_KMIN), _), GP_BATCH_KMAX)(int group, int leaf, int iep) {
    if (iep) {
        if (leaf != 1 || (group != 64 && group != 32)) return nullptr;
#define GP_IEP_CASE(D)                                                                \
    if (iep == D) return group == 64 ? batch_kernel<64, 1, D> : batch_kernel<32, 1, D>;
        GP_IEP_CASE(2)
        GP_IEP_CASE(3)
        GP_IEP_CASE(4)
#undef GP_IEP_CASE
        return nullptr;
    }
#define GP_PLAIN_CASE(GG)                                                       \
    if (group == GG) {                                                          \
        if (leaf == 1) return batch_kernel<GG, 1, 0>;                           \
        if (leaf == 3) return batch_kernel<GG, 3, 0>;                           \
        if (leaf == 4) return batch_kernel<GG, 4, 0>;                           \
        return nullptr;                                                         \
    }
    GP_PLAIN_CASE(64)
    GP_PLAIN_CASE(32)
    GP_PLAIN_CASE(16)
    GP_PLAIN_CASE(8)
#undef GP_PLAIN_CASE
    return nullptr;
}

}  // namespace gpcount
