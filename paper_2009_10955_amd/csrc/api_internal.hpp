// Handle types behind the C ABI, shared by the API and tuner units.
#pragma once
#include <vector>

#include "gp.h"
#include "internal.hpp"
#include "planner.hpp"

struct gp_graph {
    gpint::DeviceGraph dg;
};

struct gp_plan {
    gp::Pattern pattern;
    uint64_t aut = 0;
    std::vector<gp::Rel> sets;
    std::vector<gp::Perm> schedules;
    gp::Perm order{};
    gp::Rel set = 0;
    GpPlanDesc desc{};
    gp_plan_info info{};
    bool tuned = false;          // launch below was measured on a graph
    double tuned_ms = 0;         // its measured (or estimated) full-run time
    gpint::LaunchCfg launch{};
};

struct gp_batch {
    const gp_graph* g = nullptr;
    int np = 0;
    gpint::BatchState st;
    std::vector<GpPlanDesc> descs;           // in batch order
    std::vector<gpint::LaunchCfg> cfgs;      // in batch order
    std::vector<int> slot;                   // caller's plan i runs as batch plan slot[i]
    unsigned long long* host_res = nullptr;  // pinned, 4*np
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace gpint {
// Launch configuration for a count of plan p: the plan's tuned launch (if
// any) or the defaults, with every non-zero field of l overriding it.
LaunchCfg launch_for_plan(const gp_plan* p, const gp_launch* l, const DeviceGraph& g);

// Full-run time (ms) of plan d with cfg, estimated from a strided sample of
// about 4096 root tasks: the wavefronts' summed busy time scaled to all tasks
// over the resident wavefronts, or the longest task chunk if that is longer.
// budget_ms > 0 stops the sample early (the result is then 1e300). res: 5
// device words. Negative on a HIP failure. Blocks on s.
double estimate_full_ms(const DeviceGraph& g, const GpPlanDesc& d, LaunchCfg cfg, double budget_ms,
                        hipStream_t s, unsigned long long* res, uint64_t* sample_count = nullptr,
                        int64_t* sample_stride = nullptr);

// The same in two halves, for callers that overlap the sample with other
// work: estimate_begin enqueues the sample on s (results in res[0..4]);
// estimate_end turns a host copy h of those five words into the estimate.
gp_status estimate_begin(const DeviceGraph& g, const GpPlanDesc& d, LaunchCfg cfg, double budget_ms,
                         hipStream_t s, unsigned long long* res, int64_t* stride_out);
double estimate_end(const DeviceGraph& g, const GpPlanDesc& d, const LaunchCfg& cfg,
                    const unsigned long long* h, int64_t stride);
}  // namespace gpint
