// Batched persistent kernel: several plans (patterns or configurations of
// uneven cost, any k) over one graph in ONE launch.
//
// The task space is the concatenation of every plan's root tasks, handed out
// in chunks by one device-wide atomic counter; a chunk that straddles two
// plans is split at the boundary, so no task is lost and plans of uneven cost
// fill each other's tails. Each group of G lanes interprets the descriptor of
// the plan its task belongs to; per-plan counts (and the wall-clock time
// groups spent on each plan, for the serving scheduler) are reduced per group
// into LDS and flushed once per wavefront at the end. Built once per group size,
// largest pattern size and leaf mode (-DGP_BATCH_G=64/32/16, -DGP_BATCH_KMAX=
// 5/6/8, -DGP_BATCH_LEAF=1/3/4), so a batch carries only the register
// footprint of its own shapes.
#include "count_kernel.hpp"

#if !defined(GP_BATCH_G) || !defined(GP_BATCH_KMAX) || !defined(GP_BATCH_LEAF)
#error "GP_BATCH_G, GP_BATCH_KMAX and GP_BATCH_LEAF must be defined"
#endif

namespace gpcount {

namespace {

constexpr int G = GP_BATCH_G;
constexpr int KMAX = GP_BATCH_KMAX;
constexpr int LEAF = GP_BATCH_LEAF;  // 1, 3 (flattened where possible) or 4 (long lists by the group)

template <int K>
__device__ __forceinline__ void batch_roots(const GpPlanDesc& d, Ctx<G>& c, const BatchPlan& bp, int64_t t0,
                                            int64_t t1, uint64_t& acc, bool& ovf) {
    if constexpr (K > KMAX) {
        return;
    } else if constexpr (K <= 3) {
        // lanes take different roots (never split)
        for (int64_t base = t0; base < t1; base += G) {
            const int64_t r = base + c.g.gl;
            if (r < t1) {
                const int2 e = bp.roots[bp.task_offset + r];
                uint64_t cnt = 1;
                if constexpr (K == 3) {
                    int32_t w[K] = {e.x, e.y, 0};
                    cnt = leaf_serial<K, G, MODE_PLAIN>(d, c, w);
                }
                add_count(acc, cnt, ovf);
            }
        }
    } else {
        for (int64_t t = t0; t < t1; ++t) {
            const int64_t r = task_root(bp.task_offset + t, bp.split_roots, bp.split_ways, c.sj, c.sJ);
            int2 e = bp.roots[r];
            e.x = uni<G>(e.x);
            e.y = uni<G>(e.y);
            int32_t v[K];
#pragma unroll
            for (int j = 0; j < K; ++j) v[j] = 0;
            v[0] = e.x;
            v[1] = e.y;
            run_builds<K, G, MODE_PLAIN>(d, c, 1, v);
            search<K, 2, G, LEAF, MODE_PLAIN, false>(d, c, v, acc, ovf);
        }
    }
}

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(occupancy_target(KMAX, G, LEAF)))) void batch_kernel(BatchArgs a) {
    __shared__ int32_t s_len[kBlock / G][GP_DESC_MAX_BUILDS];
    __shared__ unsigned long long s_cnt[kBlock / 64][kBatchMaxPlans];
    __shared__ unsigned s_ovf[kBlock / 64][kBatchMaxPlans];
    __shared__ unsigned long long s_busy[kBlock / 64][kBatchMaxPlans];
    const int wave = threadIdx.x / 64;
    for (int p = threadIdx.x & 63; p < kBatchMaxPlans; p += 64) {
        s_cnt[wave][p] = 0;
        s_ovf[wave][p] = 0;
        s_busy[wave][p] = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

    Ctx<G> c;
    c.row_ptr = a.row_ptr;
    c.col = a.col;
    c.cap = a.buf_cap;
    c.hub_bits = a.hub_bits;
    c.hub_words = a.hub_words;
    c.n_hubs = a.n_hubs;
    const int grp = threadIdx.x / G;
    const int64_t group_id = (int64_t)blockIdx.x * (kBlock / G) + grp;
    c.bufs = a.scratch ? a.scratch + group_id * (int64_t)a.nbuf * a.buf_cap : nullptr;
    c.lens = s_len[grp];
    c.bytes = nullptr;
    c.sj = 0;
    c.sJ = 1;
    c.deadline = 0;
    c.memo = nullptr;
    c.tag = 0;
    const int64_t chunk = a.chunk;

    for (;;) {
        unsigned long long q = 0;
        if (c.g.gl == 0) q = atomicAdd(a.queue, (unsigned long long)chunk);
        q = (unsigned long long)uni64<G>((int64_t)c.g.bcast(q, 0));
        const int64_t t0 = (int64_t)q;
        if (t0 >= a.total_tasks) break;
        const int64_t t_end = min(t0 + chunk, a.total_tasks);
        int p = 0;
        while (p + 1 < a.np && a.plans[p + 1].task_begin <= t0) ++p;
        for (int64_t tt = t0; tt < t_end;) {
            while (p + 1 < a.np && a.plans[p + 1].task_begin <= tt) ++p;
            const BatchPlan& bp = a.plans[p];
            const int64_t piece_end = min(t_end, bp.task_begin + bp.n_tasks);
            const GpPlanDesc& d = a.descs[p];
            const uint64_t clk0 = wall_clock64();
            uint64_t acc = 0;
            bool ovf = false;
            const int64_t l0 = tt - bp.task_begin, l1 = piece_end - bp.task_begin;
            switch (d.k) {
                case 2: batch_roots<2>(d, c, bp, l0, l1, acc, ovf); break;
                case 3: batch_roots<3>(d, c, bp, l0, l1, acc, ovf); break;
                case 4: batch_roots<4>(d, c, bp, l0, l1, acc, ovf); break;
                case 5: batch_roots<5>(d, c, bp, l0, l1, acc, ovf); break;
                case 6: batch_roots<6>(d, c, bp, l0, l1, acc, ovf); break;
                case 7: batch_roots<7>(d, c, bp, l0, l1, acc, ovf); break;
                case 8: batch_roots<8>(d, c, bp, l0, l1, acc, ovf); break;
                default: break;
            }
            // group sum with carry detection, into the wave's LDS counter
            uint64_t s = acc;
#pragma unroll
            for (int off = G / 2; off >= 1; off >>= 1) {
                const uint64_t t = __shfl_xor(s, off, G);
                const uint64_t u = s + t;
                ovf |= (u < s);
                s = u;
            }
            const bool any_ovf = c.g.ballot(ovf) != 0;
            if (c.g.gl == 0) {
                const unsigned long long old = atomicAdd(&s_cnt[wave][p], (unsigned long long)s);
                if (any_ovf || old + s < old) s_ovf[wave][p] = 1;
                atomicAdd(&s_busy[wave][p], (unsigned long long)(wall_clock64() - clk0));
            }
            tt = piece_end;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    for (int p = threadIdx.x & 63; p < a.np; p += 64) {
        const unsigned long long v = s_cnt[wave][p];
        if (v) {
            const unsigned long long old = atomicAdd(&a.result[3 * p], v);
            if (old + v < old) atomicOr(&a.result[3 * p + 1], 1ull);
        }
        if (s_ovf[wave][p]) atomicOr(&a.result[3 * p + 1], 1ull);
        if (s_busy[wave][p]) atomicAdd(&a.result[3 * p + 2], s_busy[wave][p]);
    }
}

}  // namespace

#define GP_CAT2(a, b) a##b
#define GP_CAT(a, b) GP_CAT2(a, b)

BatchFn GP_CAT(GP_CAT(GP_CAT(GP_CAT(GP_CAT(batch_kernel_g, GP_BATCH_G), _k), GP_BATCH_KMAX), _l),
               GP_BATCH_LEAF)() {
    return batch_kernel;
}

}  // namespace gpcount
