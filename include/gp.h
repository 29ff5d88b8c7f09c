/*
 * gp.h -- C ABI of the MI355X (gfx950) pattern-embedding counting library.
 *
 * The library counts the embeddings of a small connected unlabeled pattern in
 * a large undirected data graph, following GraphPi (arXiv 2009.10955):
 *   - Section II-A defines the problem: the number of distinct subgraphs of
 *     the data graph that are edge-preserving bijective images of the pattern
 *     (non-induced: extra data edges among the image vertices are allowed);
 *   - Section IV-A (Algorithm 1) generates restriction sets (id(a) > id(b)
 *     pairs) that make every embedding be found exactly once;
 *   - Section IV-B filters schedules (matching orders) in two phases;
 *   - Section IV-C ranks (schedule, restriction set) configurations with a
 *     nested cost model;
 *   - Sections II-B and IV-B describe the nested-loop search whose candidate
 *     sets are intersections of sorted neighbor lists cut by the restrictions.
 * The users' view matches Section III: a pattern and a graph in the form of
 * adjacency lists in, a count out.
 *
 * Conventions for every call:
 *   - Return value: GP_OK (0) or a negative gp_status. On error, out-params
 *     are left untouched and nothing is leaked.
 *   - Ownership: input buffers stay the caller's and may be freed as soon as
 *     the call returns. Graph and plan handles are owned by the library until
 *     the matching gp_free_* call. Handles are immutable after creation, so
 *     concurrent counts on different streams with the same handles are legal.
 *   - Streams: a hipStream_t is passed as void* (0 = the null stream). Work is
 *     ordered on that stream; calls documented as blocking synchronise it.
 *   - Vertex ids and pattern vertices are zero-based.
 */
#ifndef GP_H
#define GP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gp_status;

enum {
    GP_OK = 0,
    GP_ERR_ARG = -1,             /* bad argument (null pointer, size out of range, bad option) */
    GP_ERR_CSR_UNSORTED = -2,    /* a neighbor list is not ascending, or row_ptr decreases */
    GP_ERR_CSR_ASYMMETRIC = -3,  /* (u,v) stored without (v,u) */
    GP_ERR_CSR_SELFLOOP = -4,    /* (v,v) stored */
    GP_ERR_CSR_DUPLICATE = -5,   /* a neighbor stored twice in one list */
    GP_ERR_PATTERN = -6,         /* pattern with k<2, k>GP_MAX_K, a self-loop, a repeated edge,
                                    a vertex id out of range, or not connected */
    GP_ERR_NOMEM = -7,           /* device or host allocation failed */
    GP_ERR_HIP = -8,             /* a HIP runtime call failed */
    GP_ERR_OVERFLOW = -9,        /* the true count does not fit in 64 bits */
    GP_ERR_BUDGET = -10,         /* predicted cost above the caller's cap */
    GP_ERR_CSR_RANGE = -11,      /* a column index outside [0, n) or row_ptr[0] != 0 */
    GP_ERR_UNSUPPORTED = -12,    /* option or shape not built into this library */
    GP_ERR_TIMEOUT = -13,        /* gp_server_wait: the query did not finish in time */
    GP_ERR_INTERNAL = -14        /* an internal consistency check failed (a bug) */
};

#define GP_MAX_K 8

/* ------------------------------------------------------------------ graph */

typedef struct gp_graph gp_graph;

/* gp_load_graph flags */
#define GP_IN_DEVICE 1u          /* row_ptr and col point to device memory (e.g. torch tensors) */
#define GP_NO_HUB_BITMAPS 2u     /* build no hub bitmaps (every membership test binary-searches) */
#define GP_DENSE_HUB_BITMAPS 4u  /* bitmaps for every non-isolated vertex that fits the budget
                                    (default: degree >= 64); for tests */

typedef struct {
    int64_t n;            /* vertices */
    int64_t m;            /* undirected edges (nnz / 2) */
    int64_t max_degree;
    uint64_t tri_cnt;     /* ordered triangles = 6 x triangles: the tri_cnt input of the
                             cardinality estimates (Section IV-C) */
    uint64_t hash;        /* 64-bit content hash of the input CSR (cache key) */
    double load_seconds;  /* wall time of gp_load_graph */
    int64_t hub_vertices; /* vertices with a dense neighbor bitmap (the highest-degree ones) */
    int64_t hub_bitmap_bytes;
} gp_stats;

/*
 * Load an undirected simple graph given as CSR (Section IV-E: each neighbor
 * list sorted and contiguous): row_ptr[n+1] (int64, row_ptr[0] == 0) and
 * col[nnz] (int32), with both directions of every edge stored, no self-loops
 * and no duplicates. Host pointers by default, device pointers with
 * GP_IN_DEVICE; either way the library copies what it needs.
 * On the device the graph is validated (GP_ERR_CSR_* on failure), relabelled
 * by descending degree (ties by ascending id), each list re-sorted, and its
 * triangle count computed for the cost model. The highest-degree vertices
 * (degree >= 64, at most 8 GiB in total) also get a dense n-bit neighbor
 * bitmap, so that a membership test in their lists is one bit read. Blocking
 * on `stream`.
 */
gp_status gp_load_graph(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz,
                        uint32_t flags, void* stream, gp_graph** out);

/* Options of gp_load_graph_opts (zero fields: the defaults of gp_load_graph). */
typedef struct {
    uint32_t flags;            /* as gp_load_graph's flags */
    int64_t hub_min_degree;    /* vertices of at least this degree get a dense neighbor bitmap
                                  (0 = 64) */
    int64_t hub_budget_bytes;  /* bitmaps of at most this many bytes in total, highest degrees
                                  first (0 = 8 GiB); each takes ceil(n/32) * 4 bytes */
} gp_load_opts;

void gp_load_opts_default(gp_load_opts* o);

/* gp_load_graph with the hub bitmap threshold and budget chosen by the
 * caller: more bitmaps turn more membership tests in long lists into one
 * bit read, at n/8 bytes of HBM each. */
gp_status gp_load_graph_opts(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz,
                             const gp_load_opts* opts, void* stream, gp_graph** out);

gp_status gp_graph_stats(const gp_graph* g, gp_stats* out);

/* Copy the relabelling to host memory: new_id[v] = id of original vertex v
 * in the device layout (n entries, caller-allocated). */
gp_status gp_graph_new_id(const gp_graph* g, int32_t* new_id);

/* Copy the device layout to host memory (caller-allocated, n+1 and nnz
 * entries): the relabelled CSR that the counting kernels read. */
gp_status gp_graph_layout(const gp_graph* g, int64_t* row_ptr, int32_t* col);

void gp_free_graph(gp_graph* g);

/* ----------------------------------------------------------------- launch */

/* Launch shape of the counting kernel. Zero fields mean "the plan's own"
 * (its tuned shape after gp_plan_tune, else the defaults). */
typedef struct {
    int32_t group;         /* lanes that share one search path: 64, 32, 16 or 8 (0 = auto) */
    int32_t waves_per_cu;  /* resident wavefronts per compute unit for the persistent grid
                              (0 = auto) */
    int32_t chunk;         /* root tasks taken per queue grab (0 = auto) */
    int32_t leaf_mode;     /* 0 auto, 1: lanes take different second-to-last candidates and
                              count the last level alone, 2: the group counts each one together,
                              3: the last two enumerated levels are flattened into one
                              load-balanced batch of (x, y) pairs (k >= 5; else as 1),
                              4: as 1, but where the last level is a group-uniform hub
                              bitmap intersected with N(x), a long N(x) is walked by the
                              whole group (coalesced loads; else as 1) */
    int32_t root_stride;   /* count only every root_stride-th root task (0 or 1 = all), */
    int32_t root_offset;   /* starting at root_offset: a seeded root sample for tuning */
    int32_t split_ways;    /* 0 auto, 1 none, else: each heavy root edge runs as split_ways
                              tasks that bind disjoint slices of its level-2 candidates
                              (shortens the tail that single hub roots leave; k >= 4) */
    int32_t split_vertices;/* heavy roots: those whose smaller endpoint in the degree-sorted
                              layout is below split_vertices, rounded down to a power of
                              two (0 = auto) */
    int32_t xcd_tasks;     /* task order over the XCDs, each with its own L2 (0 = the
                              plan's own, one cursor unless set): > 0 deals the task space
                              to the 8 XCDs in blocks of this many tasks (rounded up to a
                              multiple of chunk), so one XCD's groups work on neighbouring
                              root edges, which share their hub endpoint; an XCD that runs
                              out helps the others. -1: one task cursor for the whole
                              device (all XCDs walk the same stretch of root edges, which
                              the shared last-level cache then holds once) */
    int32_t batch_runs;    /* batches (gp_count_batch, gp_batch_create): 0 or 1 = consecutive
                              plans of one launch shape and pattern size share one persistent
                              launch with a task cursor each; 2 = every plan gets its own
                              launch in the batch (a plan over its whole task space then
                              runs as gp_count would). gp_batch_tune measures both */
} gp_launch;

void gp_launch_default(gp_launch* l);

/* ------------------------------------------------------------------- plan */

typedef struct gp_plan gp_plan;

typedef struct {
    int64_t max_states;          /* cap on distinct restriction sets visited by Algorithm 1
                                    (0 = default 4,000,000) */
    int32_t max_sets;            /* cap on valid restriction sets kept (0 = default 100,000) */
    int32_t force_order[GP_MAX_K]; /* if force_order[0] >= 0: use this schedule (must pass
                                    Phase 1; Phase 2 is not required) */
    int32_t force_set;           /* if >= 0: use the force_set-th valid set (emission order) */
    int32_t n_force_restr;       /* if > 0: use these pairs instead (validated) */
    int32_t force_restr[2 * GP_MAX_K * GP_MAX_K];
    double cost_cap;             /* if > 0: GP_ERR_BUDGET when the best predicted cost exceeds it */
    double max_seconds;          /* Algorithm 1 stops exploring after this long once a valid set
                                    exists (0 = 20 s) */
    int32_t iep;                 /* counting with inclusion-exclusion (Section IV-D) over the
                                    innermost pairwise non-adjacent levels of the schedule,
                                    when a configuration allows it (see gp_plan_info.iep):
                                    0 off; 1: as many levels as the schedule allows (at most
                                    4, and not the root edge); 2..4: at most that many */
} gp_plan_opts;

/* Fill opts with the defaults (nothing forced, no cap). */
void gp_plan_opts_default(gp_plan_opts* opts);

/*
 * Plan a pattern with k vertices and e edges (edges[2*i], edges[2*i+1]).
 * Host only. Steps: automorphisms (Section IV-A), restriction sets by
 * Algorithm 1 (each kept as its transitive closure; for complete patterns
 * with k >= 6 the k! total orders it reaches are emitted directly), efficient
 * schedules by the two phases of Section IV-B, then the configuration with
 * the lowest predicted cost under the model of Section IV-C (schedules that
 * an automorphism maps onto each other give the same searches, so one per
 * orbit is evaluated), evaluated with `stats`
 * (null: |V| = 1e6, |E| = 1e7, tri_cnt = 6e7). Ties of predicted cost go to
 * the set with more upper-bound cuts (a later vertex bounded above by an
 * earlier one), then the lexicographically smaller schedule, then the earlier
 * set. The result is compiled into a device-ready plan descriptor.
 */
gp_status gp_plan_create(const int32_t* edges, int32_t k, int32_t e, const gp_stats* stats,
                         const gp_plan_opts* opts, gp_plan** out);

typedef struct {
    int32_t k;
    int32_t order[GP_MAX_K];   /* schedule: pattern vertex searched at level i */
    int32_t n_restr;           /* pairs in the applied restriction set (transitive closure) */
    int32_t restr[2 * GP_MAX_K * GP_MAX_K]; /* (a, b) means id(a) > id(b), pattern vertices */
    uint64_t aut;              /* |Aut(P)| */
    double cost;               /* predicted cost_1 of the chosen configuration */
    int32_t n_sets;            /* valid restriction sets found by Algorithm 1 */
    int64_t n_states;          /* distinct sets visited by Algorithm 1 */
    int32_t n_schedules;       /* efficient schedules (Phase 1 + Phase 2) */
    int32_t k_eff;             /* Phase-2 k actually used */
    int32_t set_index;         /* index of the chosen set in emission order (-1 if forced pairs) */
    double plan_seconds;       /* host wall time of gp_plan_create (plus gp_plan_tune) */
    int32_t tuned;             /* 1 if the configuration and launch were measured by gp_plan_tune */
    int32_t iep;               /* number of innermost levels counted with inclusion-exclusion
                                  (0: none; 2..4): the best-ranked configuration whose last iep
                                  schedule vertices are pairwise non-adjacent and over which IEP
                                  counts every embedding the same number of times, iep_div
                                  (restrictions between two inner levels are dropped, and if
                                  needed all checked in them); for each binding of the outer
                                  levels the kernel adds the number of tuples of distinct
                                  elements of the inner levels' candidate sets, and divides the
                                  128-bit total by iep_div */
    int32_t iep_div;
    int32_t n_measured;        /* configurations timed by gp_plan_tune */
    gp_launch launch;          /* launch shape used when the caller passes none */
    double tuned_ms;           /* gp_plan_tune: full-run time of the chosen configuration and
                                  launch (measured, or estimated from samples); 0 if untuned.
                                  Batches run longer plans first */
} gp_plan_info;

gp_status gp_plan_get(const gp_plan* p, gp_plan_info* out);

/* The idx-th valid restriction set in emission order, as closure pairs
 * (restr must hold 2*GP_MAX_K*GP_MAX_K ints). */
gp_status gp_plan_get_set(const gp_plan* p, int32_t idx, int32_t* n_restr, int32_t* restr);

/* The idx-th efficient schedule (order must hold k ints). */
gp_status gp_plan_get_schedule(const gp_plan* p, int32_t idx, int32_t* order);

/* Predicted cost_1 of (schedule idx_s, restriction set idx_r) under `stats`. */
gp_status gp_plan_model_cost(const gp_plan* p, int32_t idx_s, int32_t idx_r,
                             const gp_stats* stats, double* cost);

typedef struct {
    int32_t max_configs;    /* distinct configurations to time (0 = 24) */
    int32_t sample_stride;  /* time every stride-th root task only (0 = auto, aiming at
                               about 8 ms of balanced work per sample) */
    int32_t tune_launch;    /* 1 (default): also pick lanes per group, leaf mode and, for
                               k >= 4 when the winner was timed in full, the ways heavy
                               roots are split (16, 4 or 1), the tasks taken per queue grab
                               (1, 2, 4, 8 or 16), the heavy-root threshold (64, 256, 1024
                               or 4096) and 16 or 24 resident wavefronts per CU; -1: keep
                               the defaults */
    double budget_seconds;  /* GPU time for timing sampled configurations (0 = 20 s); the
                               launch-shape, full-run and queue-grab stages that follow may
                               bring the total to at most about 4 times this */
    int32_t try_iep;        /* 1: for a plan that counts without IEP, also time each
                               candidate configuration counted with inclusion-exclusion
                               over its last 2, 3 or 4 levels (Section IV-D) where the
                               schedule allows it, and keep whichever is fastest. The tuned
                               plan may then be an IEP plan, which gp_list refuses
                               (GP_ERR_UNSUPPORTED). 0 (default): the plan's mode */
} gp_tune_opts;

void gp_tune_opts_default(gp_tune_opts* o);

/*
 * Measured configuration selection for graph g: the paper's model ranks the
 * (schedule, restriction set) configurations (Section IV-C) but sees only
 * |V|, |E| and tri_cnt, and the paper reports its choice 32% slower than the
 * best schedule on average (Section V-C). This call takes the best-ranked
 * configurations, adds each one's mirror (every pair reversed, also valid),
 * drops configurations that compile to the same search, times each on a
 * sparse strided sample of its root tasks on `stream`, times the four fastest
 * again on a denser sample, keeps the fastest, then times launch shapes for it. *out is a new plan (same pattern, same counts) whose
 * default launch is the measured best. Blocking.
 */
gp_status gp_plan_tune(const gp_graph* g, const gp_plan* p, const gp_tune_opts* opts, void* stream,
                       gp_plan** out);

/*
 * A copy of plan p (same configuration, counts and tuning record) whose
 * default launch shape takes every non-zero field of `launch` (root_stride
 * and root_offset excepted: they belong to a call). The shape a plan takes
 * in a batch is its default launch, so plans of one batch can run at
 * different shapes (Section IV-E's task partitioning across patterns).
 * GP_ERR_ARG on a field out of range (group not 64/32/16/8, leaf_mode not
 * 1..4, waves_per_cu not 1..32, negative chunk, split_ways or
 * split_vertices, xcd_tasks below -1, batch_runs not 0..2); *out is then
 * untouched. Free with gp_free_plan.
 */
gp_status gp_plan_with_launch(const gp_plan* p, const gp_launch* launch, gp_plan** out);

void gp_free_plan(gp_plan* p);

/* ------------------------------------------------------------------ count */


/*
 * Count the embeddings of plan p in graph g (exact, unsigned 64-bit).
 * One persistent kernel launch on `stream`: wavefront groups take root edges
 * (the first two schedule levels) from an atomic queue and search the
 * remaining levels depth first. Blocking: synchronises `stream` and writes
 * *out on the host. GP_ERR_OVERFLOW if the count does not fit in 64 bits.
 * `launch` may be null (auto). Device memory, allocated stream-ordered per
 * call and freed at its end: the groups' candidate buffers (at most 16 GiB;
 * the grid shrinks to fit) and, for plans that can use one, a memo table
 * (leaf mode 4: a word per hub per group, at most 4 GiB; inclusion-exclusion:
 * one table for the launch, at most 2 GiB). GP_ERR_NOMEM when an
 * allocation fails.
 */
gp_status gp_count(const gp_graph* g, const gp_plan* p, const gp_launch* launch, void* stream,
                   uint64_t* out);

/* As gp_count, without host synchronisation: dev_out (device memory, 2
 * uint64) receives {count, flags} when the stream reaches it; flag bit 0:
 * overflow, bit 1: internal check failed. */
gp_status gp_count_async(const gp_graph* g, const gp_plan* p, const gp_launch* launch,
                         void* stream, uint64_t* dev_out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): gp_count_async
 * that allocates nothing. The task cursor, the per-group candidate buffers
 * and, when room is left, the memo (leaf mode 4's per-root counts per group,
 * or an IEP plan's shared table of inner set sizes) come from one static device
 * workspace of 32 MiB that every GPU the library runs on holds until the
 * process ends; the grid shrinks so the buffers fit it. dev_out (device
 * memory, 2 uint64, caller-owned) receives {count, flags} as in
 * gp_count_async. GP_ERR_NOMEM when the plan's candidate buffers for one
 * block of groups alone exceed the workspace (a graph whose second-largest
 * degree is too high for the plan and group width). Every call on a GPU
 * shares that GPU's workspace: calls that overlap on one GPU (different
 * streams, threads) race and must be serialised by the caller. The first
 * call on a device looks the workspace up (no allocation). No host
 * synchronisation.
 */
gp_status gp_count_noalloc(const gp_graph* g, const gp_plan* p, const gp_launch* launch, void* stream,
                           uint64_t* dev_out);

/*
 * Per-root counts, for verification: dev_per_root (device memory, one uint64
 * per directed CSR entry of the device layout, nnz entries) receives, at the
 * index of the layout entry (v0, v1), the number of embeddings whose first
 * two schedule levels map to v0 and v1 (zero where the entry is not a root;
 * for an IEP plan, that number times iep_div). Blocking; *out receives the
 * total.
 */
gp_status gp_count_per_root(const gp_graph* g, const gp_plan* p, const gp_launch* launch,
                            void* stream, uint64_t* dev_per_root, uint64_t* out);

/*
 * Count and, alongside it, the algorithmic bytes of the run under the paper's
 * intersection cost model (Section IV-C: intersecting sorted sets A and B
 * costs |A| + |B|; Section IV-E: sorted contiguous lists): 4(|A'| + |B'|)
 * bytes per executed intersection of the range-cut operands A', B', 4 bytes
 * per enumerated candidate, 8 bytes per root edge, and 4 ceil(log2(|L|+1))
 * bytes per last-level binary search in a list L. Runs an instrumented copy
 * of the kernel: for measurement, never for timing. Blocking.
 */
gp_status gp_count_traffic(const gp_graph* g, const gp_plan* p, const gp_launch* launch,
                           void* stream, uint64_t* out, uint64_t* alg_bytes);

/*
 * Verification of the exact accumulation (Section II-A defines the count as
 * an integer; counts above 2^64 are reported, never wrapped): the n values
 * (host memory) are added on the device exactly as the counting kernels add
 * their lanes' counts (64-bit lane totals with carries counted, an exact
 * 128-bit wavefront sum, a 128-bit device total), then finished as every
 * count is: divided by div (>= 1; the IEP over-count of an IEP plan, 1
 * otherwise). *out = the quotient's low 64 bits; *flags bit 0: the quotient
 * does not fit in 64 bits (gp_count's GP_ERR_OVERFLOW), bit 1: div does not
 * divide the sum (GP_ERR_INTERNAL). Blocking. For tests of the carry and
 * division paths with values that no graph here reaches.
 */
gp_status gp_check_sum(const uint64_t* values, int64_t n, uint64_t div, void* stream, uint64_t* out,
                       uint32_t* flags);

/*
 * List the embeddings of plan p in graph g: every distinct subgraph that is
 * an image of the pattern (the problem as Section II-A states it; gp_count
 * returns how many there are). The search is gp_count's with its last level
 * enumerated; the restriction closure lets exactly one map reach each
 * subgraph (Section IV-A), and that map is written out. Two passes of the
 * search: one counts the embeddings of every root edge, the other writes
 * them at offsets from a scan of those counts.
 *   out       device memory, caller-owned: capacity rows of k int32. Row r
 *             is one embedding: out[r*k + u] = original id of the data vertex
 *             that pattern vertex u maps to. Rows are ordered by root edge
 *             (in the library's root order), then by search order: the same
 *             for the same graph, plan and launch.
 *   capacity  rows that out can hold (0: count only, out may be null).
 *   n_found   host: the number of embeddings (gp_count's value). When it
 *             exceeds capacity, the first capacity rows are written and the
 *             call still returns GP_OK: compare the two and call again with a
 *             larger buffer, or page.
 *   launch    waves_per_cu, chunk, root_stride and root_offset as in
 *             gp_count; the searches run in 64-lane groups whatever `group`
 *             says. Paging: calls with root_stride s and root_offset
 *             0 .. s-1 list disjoint sets of embeddings whose union is all of them.
 * Blocking (synchronises `stream`). GP_ERR_UNSUPPORTED for a plan counted
 * with inclusion-exclusion (its last two levels are never enumerated).
 */
gp_status gp_list(const gp_graph* g, const gp_plan* p, const gp_launch* launch, void* stream, int32_t* out,
                  uint64_t capacity, uint64_t* n_found);

/* Estimate the run time of a full gp_count before running it, from a strided
 * sample of about 4096 root tasks (every root_tasks/4096-th, starting with the
 * first, which is the heaviest): the summed active time of the wavefronts, scaled by the
 * stride and divided by the wavefronts the device keeps resident, or the
 * longest chunk of tasks, whichever is longer (one heavy hub root can decide
 * the run). launch as in gp_count. budget_ms > 0 stops the sample once a
 * wavefront has run that long; *est_ms is then 1e300 (the full run is at
 * least that slow). Writes the sample's count and stride when the pointers
 * are non-null: count * stride is a rough estimate of the full count (not
 * exact; for planning only; for an IEP plan the sample's total is divided by
 * iep_div without a divisibility check). Blocks on stream. Used for admission
 * by gp_server (max_query_ms) and for feasibility reports. */
gp_status gp_estimate(const gp_graph* g, const gp_plan* p, const gp_launch* launch, double budget_ms,
                      void* stream, double* est_ms, uint64_t* sample_count, int64_t* sample_stride);

/*
 * Count several plans (1..64, any pattern sizes, counted plainly or with
 * IEP) over one graph together (Section IV-E's task partitioning, across
 * patterns). Every plan keeps its own task cursor and its own launch shape:
 * lanes per group (64, 32, 16 or 8; IEP plans 64 or 32), leaf mode (1, 3 or
 * 4 where the plan allows it) and tasks per grab come from the plan's launch
 * (its tuned one after gp_plan_tune), with every non-zero field of `launch`
 * (may be null) overriding them for all plans. Plans of one shape and
 * pattern size (at most 8 at a time) share ONE persistent launch of the
 * kernel compiled for that shape: its wavefronts take the plans
 * longest-first by gp_plan_info.tuned_ms (untuned plans after, in the given
 * order) and move to the next plan when one's tasks are all handed out, so
 * the plans fill each other's tails. A plan alone in its shape (or every
 * plan, with launch->batch_runs = 2) runs as gp_count would. The shapes run
 * one after another on `stream`. Totals are exact 128-bit sums, divided by
 * each plan's IEP over-count on the host.
 * out[i] = count of plans[i] (host memory); GP_ERR_OVERFLOW if one does not
 * fit in 64 bits. Blocking. Counts equal gp_count's bit for bit.
 */
gp_status gp_count_batch(const gp_graph* g, const gp_plan* const* plans, int32_t np,
                         const gp_launch* launch, void* stream, uint64_t* out);

typedef struct gp_batch gp_batch;

/*
 * Prepare a batch for repeated counting: device descriptors, scratch, queue
 * and result buffers are allocated once, and the whole run (counter reset by
 * fill kernels, the batched kernel, the 8-bytes-per-plan readback into pinned
 * host memory) is captured into a hipGraph. The plans and graph must outlive
 * the batch. One gp_batch must not run concurrently with itself.
 */
gp_status gp_batch_create(const gp_graph* g, const gp_plan* const* plans, int32_t np,
                          const gp_launch* launch, void* stream, gp_batch** out);

/* Replay the captured graph on `stream` and wait; out[i] = count of plan i. */
gp_status gp_batch_run(gp_batch* b, void* stream, uint64_t* out);

/*
 * Point a prepared batch at a strided sample of every plan's root tasks:
 * the next gp_batch_run counts, for each plan, the roots
 * roots[root_offset + r * root_stride] (as gp_launch.root_stride and
 * root_offset do for gp_count), heavy roots split as before. root_stride 1,
 * offset 0 is the whole count again. Runs with offsets 0 .. s-1 of one
 * stride s partition every plan's embeddings (for an IEP plan with an
 * over-count above 1 a sample's raw total is divided with the quotient
 * rounded down, so its parts may add up to less, by under one per part).
 * Copies the new task table to the device before returning (waits
 * for `stream`); the captured graph is unchanged. Errors: GP_ERR_ARG.
 */
gp_status gp_batch_set_sample(gp_batch* b, int64_t root_stride, int64_t root_offset, void* stream);

/*
 * Pick the launch shape of a batch of these plans on g by measurement: one
 * full batched run with every plan at its own launch shape, then one per
 * common shape (64, 32 or 16 lanes per group x leaf mode 1, 3 or 4), timed
 * with HIP events on stream. *out receives the fastest (all fields zero:
 * each plan's own shape; else group and leaf_mode set) for gp_count_batch /
 * gp_batch_create; *best_ms (may be null) its time. Blocking; costs ten
 * full runs. Errors as gp_count_batch.
 */
gp_status gp_batch_tune(const gp_graph* g, const gp_plan* const* plans, int32_t np, void* stream,
                        gp_launch* out, double* best_ms);

void gp_free_batch(gp_batch* b);

/* ---------------------------------------------------------------- serving */

typedef struct gp_server gp_server;

typedef struct {
    int32_t max_active;     /* queries per graph sharing one launch (1..64; 0 = 64) */
    double target_ms;       /* wall time aimed at per iteration (0 = 25 ms) */
    double cost_cap;        /* reject queries whose predicted cost (Section IV-C model) exceeds
                               this with GP_ERR_BUDGET (0 = no cap) */
    int64_t initial_slice;  /* root tasks a query gets in its first iteration (0 = 8192) */
    int32_t group;          /* lanes per group of the batched kernel: 64, 32 or 16 (0 = 64) */
    int32_t leaf_mode;      /* 1, 3 or 4 (0 = 1) */
    int32_t waves_per_cu;   /* 0 = 32 */
    double max_query_ms;    /* > 0: the first query of each (graph, pattern) counts a strided
                               sample of its root tasks first; a query whose full run is then
                               estimated above max_query_ms (summed wavefront busy time scaled
                               to all tasks over the resident wavefronts, or the longest task
                               chunk if longer) is rejected with GP_ERR_BUDGET, and so is
                               one whose sample has a wavefront run past max_query_ms / 4
                               (0 = off) */
    int32_t iep;            /* queries are planned with gp_plan_opts.iep = iep: counting with
                               inclusion-exclusion (Section IV-D) where a configuration allows
                               it, which makes stars and trees cheap (default 1; 0 off) */
} gp_server_opts;

typedef struct {
    int64_t submitted, completed, rejected, failed;
    int64_t iterations, launches;
    double busy_seconds;      /* wall time spent in iterations with work on the GPU */
    int64_t joined_midflight; /* queries admitted while another query of their graph was
                                 part-way through its root tasks */
    int64_t max_batch;        /* most queries that shared one launch */
} gp_server_stats;

void gp_server_opts_default(gp_server_opts* o);

/*
 * A serving loop over resident graphs (all on one device; they must outlive
 * the server). A worker thread plans each submitted query (plans cached per
 * graph and edge list), rejects those whose predicted cost exceeds the cap,
 * and admits the rest as batch slots free up (at most 64 per graph per
 * launch). Work runs in iterations: per graph, one batched persistent launch
 * over a slice of every active query's remaining root tasks, graphs on their
 * own streams so their launches overlap. Queries that arrive while others run
 * join at the next iteration. Slices adapt to the target iteration time from
 * the per-query busy time the kernel reports. Counts are exact: the slices
 * partition each query's root tasks, so a count equals the query's solo
 * gp_count.
 */
gp_status gp_server_create(const gp_graph* const* graphs, int32_t ng, const gp_server_opts* opts,
                           gp_server** out);

/* Queue a count of the pattern (k vertices, e edges) on graphs[graph]; thread-safe. */
gp_status gp_server_submit(gp_server* s, int32_t graph, const int32_t* edges, int32_t k, int32_t e,
                           uint64_t* ticket);

/* Non-blocking. *done = 1 once the query has finished; then *status (GP_OK,
 * GP_ERR_BUDGET when rejected, GP_ERR_OVERFLOW, ...), *count and *latency_s
 * (submit to completion) are written (each may be null). */
gp_status gp_server_poll(gp_server* s, uint64_t ticket, int32_t* done, gp_status* status, uint64_t* count,
                         double* latency_s);

/* Block until the query finishes, or timeout_s passes (GP_ERR_TIMEOUT; <= 0 waits forever). */
gp_status gp_server_wait(gp_server* s, uint64_t ticket, double timeout_s, gp_status* status, uint64_t* count,
                         double* latency_s);

gp_status gp_server_stats_get(gp_server* s, gp_server_stats* out);

/* Stop accepting queries, finish the admitted ones, release everything. */
void gp_server_destroy(gp_server* s);

/* Human-readable name of a status code (static string). */
const char* gp_strerror(gp_status s);

/* Library version string (static). */
const char* gp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GP_H */
