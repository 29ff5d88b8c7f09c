// Library-internal declarations shared by the HIP translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "gp.h"
#include "plan_desc.h"

namespace gpint {

// Graph as resident in HBM: relabelled by descending degree, each list
// ascending, plus the root-edge arrays the counting kernel walks.
struct DeviceGraph {
    int device = 0;
    int num_cus = 0;
    double wall_khz = 100000;  // rate of the device's constant wall clock
    int64_t n = 0, nnz = 0;
    int64_t* row_ptr = nullptr;   // n+1
    int32_t* col = nullptr;       // nnz
    // Root edges, ordered by their smaller endpoint (heaviest first):
    int2* roots_upper = nullptr;  // entries with v1 > v0, CSR order
    int2* roots_lower = nullptr;  // entries with v1 < v0: roots_upper reversed, same order
    int2* roots_all = nullptr;    // every directed entry: the two interleaved
    int64_t n_lower = 0, n_upper = 0;
    int64_t upper_pref[32] = {};  // roots_upper entries with v0 < 2^i
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
    // roots whose smaller endpoint is below split_vertices (rounded down to a
    // power of two) run as split_ways tasks each; 1: no splitting
    int split_ways = 1;
    int64_t split_vertices = 0;
    double budget_ms = 0;  // time limit per wavefront (measurement only; 0: none)
    // tasks per XCD block (the task space dealt to the XCDs in blocks); 0 or
    // -1: one cursor for the device
    int64_t xcd = 0;
    int batch_runs = 0;  // batches: 2 = every plan its own launch
};

// Tasks per XCD block of a launch: cfg.xcd rounded up to a multiple of the
// grab, or 0 for one cursor (the default).
int64_t xcd_block_tasks(const DeviceGraph& g, const LaunchCfg& cfg, int group);

// Device memory a launch may use instead of allocating its own: the task
// cursor and high count word, the per-group candidate buffers and, when room
// is left, leaf mode 4's memo. The grid shrinks so the buffers fit.
struct Workspace {
    void* base = nullptr;  // 256-byte aligned
    size_t bytes = 0;
};

// Wavefronts per compute unit that a launch of d with cfg keeps resident.
int resident_waves_per_cu(const DeviceGraph& g, const GpPlanDesc& d, const LaunchCfg& cfg);

// Launch one count of plan d over g on `stream`. result_dev: {count,
// flags} (plus bytes when `account`), zeroed by this call on the stream.
// per_root may be null. Scratch is allocated stream-ordered and released
// after the kernel, or carved from ws when given (then nothing is allocated).
gp_status launch_count(const DeviceGraph& g, const GpPlanDesc& d, const LaunchCfg& cfg,
                       hipStream_t stream, unsigned long long* result_dev,
                       unsigned long long* per_root, bool account = false,
                       unsigned long long* busy = nullptr, const Workspace* ws = nullptr);

// launch_count without allocating: the task cursor, candidate buffers and
// memo come from one static device array of kNoallocWorkspaceBytes per GPU
// (the grid shrinks so they fit; GP_ERR_NOMEM when not even one block's
// buffers fit). Calls that overlap on one GPU share that array and race.
constexpr size_t kNoallocWorkspaceBytes = size_t(32) << 20;
gp_status launch_count_noalloc(const DeviceGraph& g, const GpPlanDesc& d, const LaunchCfg& cfg,
                               hipStream_t stream, unsigned long long* result_dev);

// Enqueue a listing of plan d over g on `stream`: found_dev (2 device words)
// receives {embeddings found, 0}; the first out_cap of them are written to out
// as rows of k int32 original vertex ids, column order[i] holding schedule
// level i. Scratch is allocated stream-ordered and released after the kernel.
gp_status launch_list(const DeviceGraph& g, const GpPlanDesc& d, const int32_t* order, const LaunchCfg& cfg,
                      hipStream_t stream, unsigned long long* found_dev, int32_t* out, int64_t out_cap);

// Consecutive batch plans [p0, p1) of one launch shape: one persistent launch
// of the kernel compiled for that shape.
struct BatchRun {
    int p0 = 0, p1 = 0;
    int group = 64, leaf = 1, iep = 0;
    int kmin = 2, kmax = 2;  // pattern sizes of its plans (one size up to 6; 7 and 8 together)
    int waves_per_cu = 1;  // the largest of its plans'
    int64_t blocks = 0;    // grid of its launch
    // one plan over its whole task space, without the memo: launched as the
    // plain counting kernel (its descriptor a kernel argument), which the
    // per-plan machinery of the batched kernel only slows down; its task
    // space as that kernel takes it
    bool solo = false;
    const int2* roots = nullptr;
    int64_t n_roots = 0, root_offset = 0, root_stride = 1, n_tasks = 0, split_roots = 0;
    int32_t split_ways = 1, chunk = 1;
};

// Device state of one batch: descriptors, per-plan task ranges and shapes,
// scratch, memo, task cursors and results, all allocated up front so that the
// launches themselves allocate nothing (they can be captured in a hipGraph and
// replayed).
struct BatchState {
    int np = 0;
    int kmax = 2;
    bool use_memo = false;
    int32_t nbuf = 0;
    int64_t cap = 0;
    int64_t memo_words = 0;
    int32_t* scratch = nullptr;
    unsigned long long* memo = nullptr;
    unsigned long long* queues = nullptr;  // np task cursors
    unsigned long long* result = nullptr;  // 4*np: count low word, flags, busy clock ticks, count high word
    unsigned long long* run_queues = nullptr;  // kBatchMaxPlans * kQueueWords: solo runs' queue words
    std::vector<BatchRun> runs;            // host: the launches, in batch order
    std::vector<GpPlanDesc> h_descs;       // host copies: launches take them as kernel arguments
    std::vector<char> h_plans;             // the per-plan task ranges and shapes, likewise
};

// A reusable batch for repeated launches with changing plans and task
// ranges (the serving loop): device buffers for 64 plans, a scratch region
// for nbuf_cap slots per group at the narrowest group width, and a memo, are
// allocated once; each launch copies descriptors and ranges from pinned
// staging memory and reads results back into pinned memory (h_result, valid
// once the stream has passed the launch).
struct BatchArena {
    BatchState st;
    int waves_per_cu = 32;
    int min_group = 64;
    int nbuf_cap = 0;
    int64_t blocks_cap = 0;
    int64_t slots_cap = 0;  // group slots of the scratch region (nbuf_cap buffers each)
    int64_t memo_words_cap = 0;
    unsigned long long* h_result = nullptr;
};
gp_status arena_create(const DeviceGraph& g, int nbuf_cap, int waves_per_cu, int min_group, BatchArena* a);
gp_status arena_launch(const DeviceGraph& g, BatchArena* a, const GpPlanDesc* descs, const LaunchCfg* cfgs,
                       const int64_t* offsets, const int64_t* counts, int np, hipStream_t stream);
void arena_release(BatchArena* a);

// Plan i runs with launch shape cfgs[i] (group, leaf, chunk, root splitting)
// and covers its tasks [offset_i, offset_i + count_i); offsets/counts null =
// every task. Consecutive plans of one shape share a launch, so callers
// order plans by shape (batch_shape_key) to launch each shape once.
gp_status batch_prepare(const DeviceGraph& g, const GpPlanDesc* descs, const LaunchCfg* cfgs,
                        const int64_t* offsets, const int64_t* counts, int np, int waves_per_cu,
                        hipStream_t stream, BatchState* st);
// Re-lay the task ranges of a prepared batch for new per-plan launch
// configurations (root samples); the shapes must be those it was prepared
// with. Copies the plan table to the device and waits. A captured batch must
// be captured again afterwards: solo runs take their task space as kernel
// arguments.
gp_status batch_update(const DeviceGraph& g, BatchState* st, const GpPlanDesc* descs, const LaunchCfg* cfgs,
                       hipStream_t stream);
// The launch shape a plan takes in a batch (pattern size class, group width,
// leaf mode, IEP depth; group widths floored at min_group) as one comparable
// key.
int batch_shape_key(const GpPlanDesc& d, const LaunchCfg& c, int min_group);
// Enqueue counter reset + one launch per run on `stream` (no allocation).
gp_status batch_enqueue(const DeviceGraph& g, const BatchState& st, hipStream_t stream);
void batch_release(BatchState* st);
// A plan's 128-bit batch total {low, flags, busy, high} divided by its IEP
// over-count (rounded down): GP_OK and *out, or GP_ERR_OVERFLOW. whole: the
// total covers every root task, so a remainder is GP_ERR_INTERNAL.
gp_status batch_result(const GpPlanDesc& d, const unsigned long long* r4, uint64_t* out, bool whole);
// The counting kernels' accumulation and final step applied to n given
// values (host memory): *out = (sum / div) mod 2^64, *flags bit 0 if the
// quotient does not fit in 64 bits, bit 1 if div does not divide the sum.
gp_status check_sum(const uint64_t* values, int64_t n, uint64_t div, hipStream_t stream, uint64_t* out,
                    uint32_t* flags);
// Number of root tasks of a descriptor (its cut picks the root array).
int64_t root_task_count(const DeviceGraph& g, const GpPlanDesc& d);
// Tasks of plan d over g with cfg's root splitting (no sampling).
int64_t task_count(const DeviceGraph& g, const GpPlanDesc& d, const LaunchCfg& cfg);

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
