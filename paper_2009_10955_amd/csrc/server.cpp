// Serving loop (gp_server_*): pattern-count queries against resident graphs,
// with continuous batching.
//
// A worker thread owns the device side. Queries are planned off the submit
// path (plans are cached per graph and edge list); a query whose predicted
// cost (the model of Section IV-C) exceeds the cap is rejected with
// GP_ERR_BUDGET. The model ranks configurations of one pattern well but
// predicts run time across patterns poorly (on power-law graphs it misses
// the hubs), so with max_query_ms the first query of each (graph, pattern)
// also counts a strided root sample whose wavefront busy time gives a
// full-run estimate, and queries estimated above the limit are rejected too.
// The sample stops once a wavefront has run a quarter of the limit (such a
// query is rejected): a sample of a heavy pattern would otherwise hold every
// wavefront of the device for the whole limit. Admitted queries join the active set of their graph as
// batch slots (at most 64 per launch: the batched kernel keeps per-plan
// counters in LDS) and HBM scratch allow.
//
// Work proceeds in iterations. Each iteration launches, per graph with active
// queries, ONE batched persistent kernel over a slice of every active query's
// remaining root tasks (graphs on their own streams, so their launches
// overlap on the device). Two launches per graph are kept in flight on two
// streams: the next is enqueued before the previous one is collected, so its
// wavefronts take the device as the previous launch's tail drains. A query
// finishes when its last slice has been collected; new queries join at the
// next launch, so a short query arriving behind a long one waits about one
// iteration. Slices adapt: the kernel reports the wall time its groups spent
// on each query, which gives each query's task rate, and the next slice aims
// at an equal share of the target iteration time.
// Counts are exact: slices partition each query's root tasks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "api_internal.hpp"

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

enum QState { Q_QUEUED = 0, Q_WAITING = 1, Q_ACTIVE = 2, Q_DONE = 3 };

struct Query {
    uint64_t ticket = 0;
    int graph = 0;
    int k = 0;
    std::vector<int32_t> edges;
    const gp_plan* plan = nullptr;  // owned by the plan cache
    int64_t n_tasks = 0, progress = 0, slice = 0;
    int64_t launched = 0;  // tasks handed to launches (progress: tasks collected)
    int inflight = 0;      // launches in flight that hold a slice of this query
    uint64_t count = 0;
    uint64_t raw_lo = 0, raw_hi = 0;  // 128-bit total of the collected slices (before the IEP division)
    QState state = Q_QUEUED;
    gp_status status = GP_OK;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int iterations = 0;
};

}  // namespace

struct gp_server {
    std::vector<const gp_graph*> graphs;
    gp_server_opts opts{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Query*> inbox;
    std::unordered_map<uint64_t, Query*> by_ticket;
    uint64_t next_ticket = 1;
    bool stop = false;
    gp_status fatal = GP_OK;
    gp_server_stats stats{};
    std::thread worker;
    // worker-owned. Two launch slots per graph (arena + stream each): the
    // next iteration is enqueued before the previous one is collected, so its
    // wavefronts fill the device while the previous launch's tail drains.
    std::vector<gpint::BatchArena> arenas;  // [graph * 2 + slot]
    std::vector<hipStream_t> streams;       // [graph * 2 + slot]
    struct Launch {
        int graph = 0, slot = 0;
        std::vector<Query*> qs;
        std::vector<int64_t> slices;
    };
    std::deque<Launch> inflight;
    std::vector<int> slot_busy;  // [graph * 2 + slot]
    std::vector<std::deque<Query*>> waiting;
    std::vector<std::vector<Query*>> active;
    std::map<std::pair<int, std::vector<int32_t>>, gp_plan*> plan_cache;
    std::map<const gp_plan*, double> est_ms;  // measured full-run estimates (max_query_ms)
    // estimates run on side streams while iterations go on; queries of a
    // (graph, pattern) whose estimate is not known yet wait on it
    struct Estimate {
        int graph = 0;
        const gp_plan* plan = nullptr;
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        unsigned long long* dev = nullptr;   // 5 words
        unsigned long long* host = nullptr;  // pinned, 5 words
        int64_t stride = 1;
        std::vector<Query*> queries;
    };
    std::vector<Estimate*> est_live, est_idle;
    std::deque<Estimate*> est_queue;
    std::map<const gp_plan*, Estimate*> est_by_plan;
};

namespace {

void finish(gp_server* S, Query* q, gp_status st) {
    std::lock_guard<std::mutex> lk(S->mu);
    q->status = st;
    q->state = Q_DONE;
    q->t_done = now_s();
    if (st == GP_OK) ++S->stats.completed;
    else if (st == GP_ERR_BUDGET) ++S->stats.rejected;
    else ++S->stats.failed;
    S->cv_done.notify_all();
}

// Launch shape of every batched launch of the server (its kernels, its task space).
gpint::LaunchCfg server_launch(const gp_server* S) {
    gpint::LaunchCfg cfg;
    cfg.group = S->opts.group;
    cfg.leaf = S->opts.leaf_mode;
    cfg.waves_per_cu = S->opts.waves_per_cu;
    cfg.chunk = 4;
    cfg.split_ways = 16;
    cfg.split_vertices = 256;
    return cfg;
}

gp_status plan_query(gp_server* S, Query* q) {
    std::vector<int32_t> key = q->edges;
    // canonical key: each edge (min, max), sorted
    std::vector<std::pair<int32_t, int32_t>> es;
    for (size_t i = 0; i + 1 < key.size(); i += 2)
        es.push_back({std::min(key[i], key[i + 1]), std::max(key[i], key[i + 1])});
    std::sort(es.begin(), es.end());
    key.clear();
    key.push_back(q->k);
    for (auto& e : es) {
        key.push_back(e.first);
        key.push_back(e.second);
    }
    auto ck = std::make_pair(q->graph, key);
    auto it = S->plan_cache.find(ck);
    if (it == S->plan_cache.end()) {
        gp_stats st;
        gp_graph_stats(S->graphs[q->graph], &st);
        gp_plan_opts o;
        gp_plan_opts_default(&o);
        o.cost_cap = S->opts.cost_cap;
        o.iep = S->opts.iep;
        gp_plan* p = nullptr;
        gp_status rc = gp_plan_create(q->edges.data(), q->k, (int32_t)(q->edges.size() / 2), &st, &o, &p);
        if (rc != GP_OK) return rc;
        it = S->plan_cache.emplace(ck, p).first;
    }
    q->plan = it->second;
    // slices cut the query's task space, in which a split root counts once per task
    q->n_tasks = gpint::task_count(S->graphs[q->graph]->dg, q->plan->desc, server_launch(S));
    return GP_OK;
}

constexpr size_t kMaxLiveEstimates = 8;

// Route a planned query: reject, wait for a batch slot, or wait for the
// estimate of its (graph, pattern).
void route_query(gp_server* S, Query* q) {
    if (q->n_tasks == 0) {
        finish(S, q, GP_OK);
        return;
    }
    if (S->opts.max_query_ms > 0) {
        auto e = S->est_ms.find(q->plan);
        if (e == S->est_ms.end()) {
            auto& slot = S->est_by_plan[q->plan];
            if (!slot) {
                if (!S->est_idle.empty()) {
                    slot = S->est_idle.back();
                    S->est_idle.pop_back();
                } else {
                    slot = new (std::nothrow) gp_server::Estimate;
                    if (!slot) {
                        S->est_by_plan.erase(q->plan);
                        finish(S, q, GP_ERR_NOMEM);
                        return;
                    }
                }
                slot->graph = q->graph;
                slot->plan = q->plan;
                slot->queries.clear();
                S->est_queue.push_back(slot);
            }
            slot->queries.push_back(q);
            return;
        }
        if (e->second > S->opts.max_query_ms) {
            finish(S, q, GP_ERR_BUDGET);
            return;
        }
    }
    q->state = Q_WAITING;
    S->waiting[q->graph].push_back(q);
}

void fail_estimate(gp_server* S, gp_server::Estimate* x, gp_status rc) {
    for (Query* q : x->queries) finish(S, q, rc);
    x->queries.clear();
    S->est_by_plan.erase(x->plan);
}

// Start queued estimates, collect finished ones, and route their queries.
void poll_estimates(gp_server* S) {
    while (!S->est_queue.empty() && S->est_live.size() < kMaxLiveEstimates) {
        gp_server::Estimate* x = S->est_queue.front();
        S->est_queue.pop_front();
        bool ok = true;
        if (!x->stream)
            ok = hipStreamCreateWithFlags(&x->stream, hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&x->done, hipEventDisableTiming) == hipSuccess &&
                 hipMalloc((void**)&x->dev, 5 * sizeof(unsigned long long)) == hipSuccess &&
                 hipHostMalloc((void**)&x->host, 5 * sizeof(unsigned long long), hipHostMallocDefault) ==
                     hipSuccess;
        gpint::LaunchCfg cfg = server_launch(S);
        cfg.waves_per_cu = 32;
        ok = ok &&
             gpint::estimate_begin(S->graphs[x->graph]->dg, x->plan->desc, cfg, S->opts.max_query_ms / 4.0,
                                   x->stream, x->dev, &x->stride) == GP_OK &&
             hipMemcpyAsync(x->host, x->dev, 5 * sizeof(unsigned long long), hipMemcpyDeviceToHost, x->stream) ==
                 hipSuccess &&
             hipEventRecord(x->done, x->stream) == hipSuccess;
        if (!ok) {
            fail_estimate(S, x, GP_ERR_HIP);
            S->est_idle.push_back(x);
            continue;
        }
        S->est_live.push_back(x);
    }
    std::vector<gp_server::Estimate*> still;
    for (gp_server::Estimate* x : S->est_live) {
        const hipError_t r = hipEventQuery(x->done);
        if (r == hipErrorNotReady) {
            still.push_back(x);
            continue;
        }
        if (r != hipSuccess) {
            fail_estimate(S, x, GP_ERR_HIP);
        } else {
            gpint::LaunchCfg cfg = server_launch(S);
            cfg.waves_per_cu = 32;
            const double est = gpint::estimate_end(S->graphs[x->graph]->dg, x->plan->desc, cfg, x->host, x->stride);
            S->est_ms[x->plan] = est;
            std::vector<Query*> qs;
            qs.swap(x->queries);
            S->est_by_plan.erase(x->plan);
            for (Query* q : qs) route_query(S, q);
        }
        S->est_idle.push_back(x);
    }
    S->est_live.swap(still);
}

bool arena_fits(const gp_server* S, int g, int nbuf) {
    const gpint::BatchArena& a = S->arenas[2 * g];
    return a.st.queues && a.nbuf_cap >= nbuf;
}

// Both launch slots of graph g with room for nbuf buffer slots per group.
// Only while neither slot is in flight.
gp_status ensure_arena(gp_server* S, int g, int nbuf) {
    if (arena_fits(S, g, nbuf)) return GP_OK;
    const int want = std::max(nbuf, std::max(S->arenas[2 * g].nbuf_cap * 2, 4));
    for (int slot = 0; slot < 2; ++slot) {
        gpint::BatchArena& a = S->arenas[2 * g + slot];
        gpint::arena_release(&a);
        const gpint::LaunchCfg lc = server_launch(S);
        gp_status rc =
            gpint::arena_create(S->graphs[g]->dg, std::min(want, GP_DESC_MAX_BUILDS), lc.waves_per_cu, lc.group, &a);
        if (rc != GP_OK) return rc;
    }
    return GP_OK;
}

void worker_main(gp_server* S) {
    (void)hipSetDevice(S->device);
    const int ng = (int)S->graphs.size();
    S->arenas.assign(2 * ng, gpint::BatchArena{});
    S->streams.assign(2 * ng, nullptr);
    S->slot_busy.assign(2 * ng, 0);
    S->waiting.assign(ng, {});
    S->active.assign(ng, {});
    for (int i = 0; i < 2 * ng; ++i) {
        if (hipStreamCreateWithFlags(&S->streams[i], hipStreamNonBlocking) != hipSuccess) {
            std::lock_guard<std::mutex> lk(S->mu);
            S->fatal = GP_ERR_HIP;
        }
    }
    const double target = S->opts.target_ms / 1e3;
    const gpint::LaunchCfg lcfg = server_launch(S);
    double busy_since = -1;  // wall time the device last went from idle to busy
    for (;;) {
        std::vector<Query*> fresh;
        bool idle = S->inflight.empty();
        for (int g = 0; g < ng; ++g)
            if (!S->active[g].empty() || !S->waiting[g].empty()) idle = false;
        const bool estimating = !S->est_live.empty() || !S->est_queue.empty();
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (idle && S->inbox.empty()) {
                if (S->stop && !estimating) break;
                S->cv_work.wait_for(lk, std::chrono::milliseconds(estimating ? 1 : 50));
            }
            fresh.assign(S->inbox.begin(), S->inbox.end());
            S->inbox.clear();
            if (S->fatal != GP_OK) {
                // fail everything still queued
                for (Query* q : fresh) {
                    q->status = S->fatal;
                    q->state = Q_DONE;
                    q->t_done = now_s();
                    ++S->stats.failed;
                }
                S->cv_done.notify_all();
                if (S->stop) break;
                continue;
            }
        }
        for (Query* q : fresh) {
            gp_status rc = plan_query(S, q);
            if (rc != GP_OK) {
                finish(S, q, rc);
                continue;
            }
            route_query(S, q);
        }
        poll_estimates(S);
        // admission: free slots and scratch
        bool any = false;
        for (int g = 0; g < ng; ++g) {
            while ((int)S->active[g].size() < S->opts.max_active && !S->waiting[g].empty()) {
                Query* q = S->waiting[g].front();
                if (!arena_fits(S, g, q->plan->desc.nbuf)) {
                    // growing the arenas waits until this graph has nothing in flight
                    if (S->slot_busy[2 * g] || S->slot_busy[2 * g + 1]) break;
                    if (ensure_arena(S, g, q->plan->desc.nbuf) != GP_OK) {
                        S->waiting[g].pop_front();
                        finish(S, q, GP_ERR_NOMEM);
                        continue;
                    }
                }
                S->waiting[g].pop_front();
                q->state = Q_ACTIVE;
                q->t_admit = now_s();
                q->slice = S->opts.initial_slice;
                // with a measured estimate, the first slice aims at a quarter of the target
                // iteration (tasks run heaviest first, so the first slice is the slowest)
                auto e = S->est_ms.find(q->plan);
                if (e != S->est_ms.end() && e->second > 0) {
                    const double share = S->opts.target_ms / std::max(e->second, S->opts.target_ms) / 4.0;
                    const double want = std::max(16.0, (double)q->n_tasks * share);
                    q->slice = std::min<int64_t>(S->opts.initial_slice, (int64_t)want);
                }
                bool midflight = false;
                for (Query* o : S->active[g])
                    if (o->launched > 0) midflight = true;
                S->active[g].push_back(q);
                std::lock_guard<std::mutex> lk(S->mu);
                if (midflight) ++S->stats.joined_midflight;
                S->stats.max_batch = std::max<int64_t>(S->stats.max_batch, (int64_t)S->active[g].size());
            }
            if (!S->active[g].empty()) any = true;
        }
        if (!any && S->inflight.empty()) continue;

        for (int g = 0; g < ng; ++g) {
            auto& act = S->active[g];
            act.erase(std::remove_if(act.begin(), act.end(), [](Query* q) { return q->state == Q_DONE; }),
                      act.end());
        }
        // launch: per graph, a slice of every active query's remaining tasks
        // into a free slot (at most one new launch per graph per pass)
        bool launched_any = false;
        for (int g = 0; g < ng; ++g) {
            int slot = !S->slot_busy[2 * g] ? 0 : (!S->slot_busy[2 * g + 1] ? 1 : -1);
            if (slot < 0) continue;
            gp_server::Launch L;
            L.graph = g;
            L.slot = slot;
            std::vector<GpPlanDesc> descs;
            std::vector<gpint::LaunchCfg> cfgs;
            std::vector<int64_t> offs;
            // queries of one launch shape side by side: each shape is one launch
            std::vector<Query*> ready;
            for (Query* q : S->active[g])
                if (q->launched < q->n_tasks && q->state != Q_DONE) ready.push_back(q);
            const int min_group = S->arenas[2 * g + slot].min_group;
            std::stable_sort(ready.begin(), ready.end(), [&](const Query* a, const Query* b) {
                return gpint::batch_shape_key(a->plan->desc, lcfg, min_group) <
                       gpint::batch_shape_key(b->plan->desc, lcfg, min_group);
            });
            for (Query* q : ready) {
                const int64_t c = std::min(q->slice, q->n_tasks - q->launched);
                descs.push_back(q->plan->desc);
                cfgs.push_back(lcfg);
                offs.push_back(q->launched);
                L.qs.push_back(q);
                L.slices.push_back(c);
            }
            if (L.qs.empty()) continue;
            const int idx = 2 * g + slot;
            gp_status rc = gpint::arena_launch(S->graphs[g]->dg, &S->arenas[idx], descs.data(), cfgs.data(),
                                               offs.data(), L.slices.data(), (int)L.qs.size(), S->streams[idx]);
            if (rc != GP_OK) {
                for (Query* q : L.qs) finish(S, q, rc);
                continue;
            }
            for (size_t i = 0; i < L.qs.size(); ++i) {
                L.qs[i]->launched += L.slices[i];
                ++L.qs[i]->inflight;
            }
            S->slot_busy[idx] = 1;
            if (S->inflight.empty()) busy_since = now_s();
            S->inflight.push_back(std::move(L));
            launched_any = true;
            std::lock_guard<std::mutex> lk(S->mu);
            ++S->stats.launches;
        }
        // collect the oldest launch once nothing more can be launched
        if (launched_any || S->inflight.empty()) continue;
        gp_server::Launch L = std::move(S->inflight.front());
        S->inflight.pop_front();
        const int idx = 2 * L.graph + L.slot;
        const bool ok = hipStreamSynchronize(S->streams[idx]) == hipSuccess;
        S->slot_busy[idx] = 0;
        if (S->inflight.empty() && busy_since >= 0) {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stats.busy_seconds += now_s() - busy_since;
            busy_since = -1;
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            ++S->stats.iterations;
        }
        const unsigned long long* r = S->arenas[idx].h_result;
        int n_active = 0;
        for (int g = 0; g < ng; ++g) n_active += (int)S->active[g].size();
        const double fair = target / std::max(1, n_active);
        // GPU seconds a query's slice used: its groups' busy clock ticks over
        // the groups the device keeps resident
        const double groups = (double)S->graphs[L.graph]->dg.num_cus * lcfg.waves_per_cu * (64.0 / lcfg.group);
        const double tick_s = 1.0 / (S->graphs[L.graph]->dg.wall_khz * 1e3);
        for (size_t i = 0; i < L.qs.size(); ++i) {
            Query* q = L.qs[i];
            --q->inflight;
            if (q->state == Q_DONE) continue;
            if (!ok) {
                finish(S, q, GP_ERR_HIP);
                continue;
            }
            // 128-bit sum of the slices' 128-bit totals; divided once at the end
            const uint64_t lo = q->raw_lo + r[4 * i];
            q->raw_hi += r[4 * i + 3] + (lo < q->raw_lo ? 1u : 0u);
            q->raw_lo = lo;
            q->progress += L.slices[i];
            ++q->iterations;
            if (q->progress >= q->n_tasks && q->inflight == 0) {
                const unsigned long long w[4] = {q->raw_lo, 0, 0, q->raw_hi};
                const gp_status fs = gpint::batch_result(q->plan->desc, w, &q->count, true);
                finish(S, q, fs);
                continue;
            }
            // next slice: this query's task rate times its fair share of the target
            const double t_q = std::max(1e-7, (double)r[4 * i + 2] * tick_s / groups);
            const double rate = (double)L.slices[i] / t_q;
            double next = rate * fair;
            next = std::min(next, 4.0 * (double)L.slices[i] + 1);
            next = std::max(next, 64.0);
            q->slice = (int64_t)std::min(next, 1e12);
        }
    }
    for (int i = 0; i < 2 * ng; ++i) {
        if (S->streams[i]) {
            (void)hipStreamSynchronize(S->streams[i]);
            (void)hipStreamDestroy(S->streams[i]);
        }
        gpint::arena_release(&S->arenas[i]);
    }
    for (gp_server::Estimate* x : S->est_live) S->est_idle.push_back(x);
    for (gp_server::Estimate* x : S->est_queue) S->est_idle.push_back(x);
    for (gp_server::Estimate* x : S->est_idle) {
        if (x->stream) {
            (void)hipStreamSynchronize(x->stream);
            (void)hipStreamDestroy(x->stream);
        }
        if (x->done) (void)hipEventDestroy(x->done);
        if (x->dev) (void)hipFree(x->dev);
        if (x->host) (void)hipHostFree(x->host);
        delete x;
    }
    S->est_live.clear();
    S->est_queue.clear();
    S->est_idle.clear();
}

}  // namespace

extern "C" {

void gp_server_opts_default(gp_server_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->max_active = 64;
    o->target_ms = 25.0;
    o->initial_slice = 8192;
    o->group = 64;
    o->leaf_mode = 1;
    o->waves_per_cu = 32;
    o->iep = 1;
}

gp_status gp_server_create(const gp_graph* const* graphs, int32_t ng, const gp_server_opts* opts,
                           gp_server** out) {
    if (!graphs || ng < 1 || !out) return GP_ERR_ARG;
    for (int i = 0; i < ng; ++i)
        if (!graphs[i]) return GP_ERR_ARG;
    gp_server_opts o;
    gp_server_opts_default(&o);
    if (opts) o = *opts;
    if (o.max_active <= 0) o.max_active = 64;
    if (o.max_active > 64) return GP_ERR_ARG;
    if (o.target_ms <= 0) o.target_ms = 25.0;
    if (o.initial_slice <= 0) o.initial_slice = 8192;
    if (o.group != 64 && o.group != 32 && o.group != 16) o.group = 64;
    if (o.leaf_mode != 1 && o.leaf_mode != 3 && o.leaf_mode != 4) o.leaf_mode = 1;
    if (o.waves_per_cu <= 0 || o.waves_per_cu > 32) o.waves_per_cu = 32;
    if (o.max_query_ms < 0 || o.cost_cap < 0 || o.iep < 0 || o.iep > GP_IEP_MAX_INNER) return GP_ERR_ARG;
    gp_server* S = new (std::nothrow) gp_server;
    if (!S) return GP_ERR_NOMEM;
    S->graphs.assign(graphs, graphs + ng);
    S->opts = o;
    S->device = graphs[0]->dg.device;
    for (int i = 1; i < ng; ++i)
        if (graphs[i]->dg.device != S->device) {
            delete S;
            return GP_ERR_ARG;
        }
    try {
        S->worker = std::thread(worker_main, S);
    } catch (...) {
        delete S;
        return GP_ERR_NOMEM;
    }
    *out = S;
    return GP_OK;
}

gp_status gp_server_submit(gp_server* S, int32_t graph, const int32_t* edges, int32_t k, int32_t e,
                           uint64_t* ticket) {
    if (!S || !edges || !ticket || graph < 0 || graph >= (int32_t)S->graphs.size() || k < 2 ||
        k > GP_MAX_K || e < 1 || e > k * (k - 1) / 2)
        return GP_ERR_ARG;
    Query* q = new (std::nothrow) Query;
    if (!q) return GP_ERR_NOMEM;
    q->graph = graph;
    q->k = k;
    q->edges.assign(edges, edges + 2 * e);
    q->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) {
            delete q;
            return GP_ERR_ARG;
        }
        q->ticket = S->next_ticket++;
        S->by_ticket[q->ticket] = q;
        S->inbox.push_back(q);
        ++S->stats.submitted;
        *ticket = q->ticket;
    }
    S->cv_work.notify_one();
    return GP_OK;
}

gp_status gp_server_poll(gp_server* S, uint64_t ticket, int32_t* done, gp_status* status, uint64_t* count,
                         double* latency_s) {
    if (!S || !done) return GP_ERR_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->by_ticket.find(ticket);
    if (it == S->by_ticket.end()) return GP_ERR_ARG;
    Query* q = it->second;
    *done = q->state == Q_DONE ? 1 : 0;
    if (*done) {
        if (status) *status = q->status;
        if (count) *count = q->count;
        if (latency_s) *latency_s = q->t_done - q->t_submit;
    }
    return GP_OK;
}

gp_status gp_server_wait(gp_server* S, uint64_t ticket, double timeout_s, gp_status* status, uint64_t* count,
                         double* latency_s) {
    if (!S) return GP_ERR_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->by_ticket.find(ticket);
    if (it == S->by_ticket.end()) return GP_ERR_ARG;
    Query* q = it->second;
    auto pred = [&] { return q->state == Q_DONE; };
    if (timeout_s > 0) {
        if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) return GP_ERR_TIMEOUT;
    } else {
        S->cv_done.wait(lk, pred);
    }
    if (status) *status = q->status;
    if (count) *count = q->count;
    if (latency_s) *latency_s = q->t_done - q->t_submit;
    return GP_OK;
}

gp_status gp_server_stats_get(gp_server* S, gp_server_stats* out) {
    if (!S || !out) return GP_ERR_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    return GP_OK;
}

void gp_server_destroy(gp_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (auto& kv : S->by_ticket) delete kv.second;
    for (auto& kv : S->plan_cache) gp_free_plan(kv.second);
    delete S;
}

}  // extern "C"
