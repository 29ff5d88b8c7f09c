// Library-internal declarations shared by the HIP translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gp.h"
#include "plan_desc.h"

namespace gpint {

// Graph as resident in HBM: relabelled by descending degree, each list
// ascending, plus the root-edge arrays the counting kernel walks.
struct DeviceGraph {
    int device = 0;
    int num_cus = 0;
    int64_t n = 0, nnz = 0;
    int64_t* row_ptr = nullptr;   // n+1
    int32_t* col = nullptr;       // nnz
    int2* roots_all = nullptr;    // every directed entry (v0, v1), CSR order
    int2* roots_lower = nullptr;  // entries with v1 < v0, CSR order
    int2* roots_upper = nullptr;  // entries with v1 > v0, CSR order
    int64_t n_lower = 0, n_upper = 0;
    int32_t* new_id = nullptr;    // original id -> layout id
    uint32_t* hub_bits = nullptr; // dense neighbor bitmaps of vertices [0, n_hubs)
    int64_t hub_words = 0;        // uint32 words per bitmap = ceil(n / 32)
    int32_t n_hubs = 0;
    int64_t max_deg = 0;          // largest degree
    int64_t deg2 = 0;             // second largest degree (bound on any |N(a) & N(b)|, a != b)
    gp_stats stats{};
};

struct LaunchCfg {
    int group = 64;
    int waves_per_cu = 8;
    int chunk = 8;
    int leaf = 1;
    int64_t root_stride = 1;  // count only roots[offset + t * stride]
    int64_t root_offset = 0;
};

// Launch one count of plan d over g on `stream`. result_dev: {count,
// overflow flag} (plus algorithmic bytes when `account`), zeroed by this call
// on the stream. per_root may be null. Scratch is allocated stream-ordered
// and released after the kernel.
gp_status launch_count(const DeviceGraph& g, const GpPlanDesc& d, const LaunchCfg& cfg,
                       hipStream_t stream, unsigned long long* result_dev,
                       unsigned long long* per_root, bool account = false);

// Launch one persistent kernel over the union of the plans' root tasks.
// result_dev: 2*np u64 ({count, overflow} per plan).
gp_status launch_count_batch(const DeviceGraph& g, const GpPlanDesc* descs, int np,
                             const LaunchCfg& cfg, hipStream_t stream,
                             unsigned long long* result_dev);

// Launch defaults for a plan descriptor, and overriding them with the
// non-zero fields of a caller's gp_launch.
LaunchCfg default_launch(const GpPlanDesc& d);
LaunchCfg apply_launch(LaunchCfg cfg, const gp_launch* l);

}  // namespace gpint

#define GP_HIP_TRY(expr)                       \
    do {                                       \
        hipError_t _e = (expr);                \
        if (_e != hipSuccess) return GP_ERR_HIP; \
    } while (0)
