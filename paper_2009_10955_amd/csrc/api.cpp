// C ABI (include/gp.h): argument checking, ownership, and the glue between
// the host planner and the device kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "gp.h"
#include "internal.hpp"
#include "planner.hpp"

namespace gpint {
gp_status build_layout(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz,
                       hipStream_t s, DeviceGraph* g);
gp_status build_hub_bitmaps(DeviceGraph* g, int64_t min_degree, int64_t budget_bytes, hipStream_t s);
}

#include "api_internal.hpp"

namespace {

double now_seconds() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
            changed = hipSetDevice(dev) == hipSuccess;
        }
    }
    ~DeviceGuard() {
        if (changed) (void)hipSetDevice(prev);
    }
};

void free_device_graph(gpint::DeviceGraph& g) {
    (void)hipFree(g.row_ptr);
    (void)hipFree(g.col);
    (void)hipFree(g.roots_all);
    (void)hipFree(g.roots_lower);
    (void)hipFree(g.roots_upper);
    (void)hipFree(g.new_id);
    (void)hipFree(g.hub_bits);
    g = gpint::DeviceGraph{};
}

// Triangle plan: schedule (0,1,2), restrictions id(0) > id(1) > id(2).
gp_status triangle_desc(GpPlanDesc* d) {
    const int32_t e[6] = {0, 1, 1, 2, 2, 0};
    gp::Pattern p;
    if (gp::parse_pattern(e, 3, 3, &p)) return GP_ERR_PATTERN;
    gp::Perm order{};
    for (int i = 0; i < 3; ++i) order[i] = uint8_t(i);
    gp::Rel r = gp::closure(gp::rel_bit(0, 1) | gp::rel_bit(1, 2), 3);
    return gp::compile_plan(p, order, r, d) == 0 ? GP_OK : GP_ERR_PATTERN;
}

// Algorithm 1's result depends on the pattern alone (its cost is per
// pattern, Table III): complete results are kept per (pattern edge set,
// caps) for the life of the process, so planning a pattern again (other
// schedules, forced sets, the tuner, the server) does not repeat it.
gp::RestrictionSets cached_restriction_sets(const gp::Pattern& pat, const std::vector<gp::Perm>& auts,
                                            int64_t max_states, int32_t max_sets, double max_seconds) {
    static std::mutex mu;
    static std::map<std::vector<int64_t>, gp::RestrictionSets> cache;
    std::vector<int64_t> key{pat.k, max_states, max_sets};
    for (int v = 0; v < pat.k; ++v) key.push_back(pat.adj[v]);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    gp::RestrictionSets rs = gp::restriction_sets(pat, auts, max_states, max_sets, max_seconds);
    if (!rs.truncated) {
        std::lock_guard<std::mutex> lk(mu);
        cache.emplace(key, rs);
    }
    return rs;
}

gp_status count_to_host(const gp_graph* g, const GpPlanDesc& d, const gpint::LaunchCfg& cfg,
                        hipStream_t s, unsigned long long* per_root, uint64_t* out,
                        uint64_t* alg_bytes = nullptr) {
    unsigned long long* res = nullptr;
    GP_HIP_TRY(hipMallocAsync((void**)&res, 3 * sizeof(unsigned long long), s));
    gp_status st = gpint::launch_count(g->dg, d, cfg, s, res, per_root, alg_bytes != nullptr);
    unsigned long long h[3] = {0, 0, 0};
    if (st == GP_OK) {
        if (hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, s) != hipSuccess) st = GP_ERR_HIP;
    }
    (void)hipFreeAsync(res, s);
    if (hipStreamSynchronize(s) != hipSuccess && st == GP_OK) st = GP_ERR_HIP;
    if (st != GP_OK) return st;
    if (h[1] & 2) return GP_ERR_INTERNAL;
    if (h[1]) return GP_ERR_OVERFLOW;
    *out = h[0];
    if (alg_bytes) *alg_bytes = h[2];
    return GP_OK;
}

}  // namespace

extern "C" {

const char* gp_version(void) { return "gp-mi355x 0.1 (gfx950)"; }

const char* gp_strerror(gp_status s) {
    switch (s) {
        case GP_OK: return "ok";
        case GP_ERR_ARG: return "invalid argument";
        case GP_ERR_CSR_UNSORTED: return "CSR neighbor list not ascending or row_ptr decreasing";
        case GP_ERR_CSR_ASYMMETRIC: return "CSR not symmetric";
        case GP_ERR_CSR_SELFLOOP: return "CSR has a self-loop";
        case GP_ERR_CSR_DUPLICATE: return "CSR has a duplicate entry";
        case GP_ERR_PATTERN: return "invalid pattern";
        case GP_ERR_NOMEM: return "out of memory";
        case GP_ERR_HIP: return "HIP runtime error";
        case GP_ERR_OVERFLOW: return "count does not fit in 64 bits";
        case GP_ERR_BUDGET: return "predicted cost above the cap";
        case GP_ERR_CSR_RANGE: return "CSR index out of range";
        case GP_ERR_UNSUPPORTED: return "unsupported option or shape";
        case GP_ERR_TIMEOUT: return "timed out";
        case GP_ERR_INTERNAL: return "internal consistency check failed";
        default: return "unknown status";
    }
}

void gp_load_opts_default(gp_load_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
}

gp_status gp_load_graph(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz,
                        uint32_t flags, void* stream, gp_graph** out) {
    gp_load_opts o;
    gp_load_opts_default(&o);
    o.flags = flags;
    return gp_load_graph_opts(row_ptr, col, n, nnz, &o, stream, out);
}

gp_status gp_load_graph_opts(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz,
                             const gp_load_opts* opts, void* stream, gp_graph** out) {
    if (!out || n < 0 || nnz < 0 || !row_ptr || (nnz > 0 && !col) || !opts) return GP_ERR_ARG;
    const uint32_t flags = opts->flags;
    if (flags & ~(GP_IN_DEVICE | GP_NO_HUB_BITMAPS | GP_DENSE_HUB_BITMAPS)) return GP_ERR_ARG;
    if (opts->hub_min_degree < 0 || opts->hub_budget_bytes < 0) return GP_ERR_ARG;
    if (n >= 0x7fffffff || nnz >= 0x7fffffff) return GP_ERR_UNSUPPORTED;
    const double t0 = now_seconds();
    hipStream_t s = (hipStream_t)stream;
    gp_graph* g = new (std::nothrow) gp_graph;
    if (!g) return GP_ERR_NOMEM;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        delete g;
        return GP_ERR_HIP;
    }
    g->dg.device = dev;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        delete g;
        return GP_ERR_HIP;
    }
    g->dg.num_cus = cus;
    int wall_khz = 0;
    if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || wall_khz <= 0)
        wall_khz = 100000;
    g->dg.wall_khz = wall_khz;

    const int64_t* d_row = row_ptr;
    const int32_t* d_col = col;
    int64_t* own_row = nullptr;
    int32_t* own_col = nullptr;
    gp_status st = GP_OK;
    int64_t ends[2] = {0, 0};
    if (!(flags & GP_IN_DEVICE)) {
        ends[0] = row_ptr[0];
        ends[1] = row_ptr[n];
        if (hipMalloc((void**)&own_row, sizeof(int64_t) * (n + 1)) != hipSuccess ||
            hipMalloc((void**)&own_col, sizeof(int32_t) * (nnz > 0 ? nnz : 1)) != hipSuccess) {
            st = GP_ERR_NOMEM;
        } else if (hipMemcpyAsync(own_row, row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s) !=
                       hipSuccess ||
                   (nnz > 0 && hipMemcpyAsync(own_col, col, sizeof(int32_t) * nnz, hipMemcpyHostToDevice,
                                              s) != hipSuccess)) {
            st = GP_ERR_HIP;
        }
        d_row = own_row;
        d_col = own_col;
    } else {
        if (hipMemcpyAsync(&ends[0], row_ptr, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&ends[1], row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = GP_ERR_HIP;
    }
    if (st == GP_OK && (ends[0] != 0 || ends[1] != nnz)) st = GP_ERR_CSR_RANGE;
    if (st == GP_OK) st = gpint::build_layout(d_row, d_col, n, nnz, s, &g->dg);
    if (st == GP_OK && !(flags & GP_NO_HUB_BITMAPS)) {
        const int64_t min_deg =
            (flags & GP_DENSE_HUB_BITMAPS) ? 1 : (opts->hub_min_degree > 0 ? opts->hub_min_degree : 64);
        const int64_t budget = opts->hub_budget_bytes > 0 ? opts->hub_budget_bytes : (int64_t(8) << 30);
        st = gpint::build_hub_bitmaps(&g->dg, min_deg, budget, s);
    }
    if (own_row || own_col) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(own_row);
        (void)hipFree(own_col);
    }
    if (st == GP_OK && nnz > 0) {
        GpPlanDesc tri;
        st = triangle_desc(&tri);
        if (st == GP_OK) {
            gpint::LaunchCfg cfg;
            cfg.group = 16;
            cfg.waves_per_cu = 16;
            cfg.chunk = 256;
            cfg.leaf = 1;
            uint64_t t = 0;
            st = count_to_host(g, tri, cfg, s, nullptr, &t);
            g->dg.stats.tri_cnt = 6 * t;
        }
    }
    if (st != GP_OK) {
        (void)hipStreamSynchronize(s);
        free_device_graph(g->dg);
        delete g;
        return st;
    }
    g->dg.stats.load_seconds = now_seconds() - t0;
    *out = g;
    return GP_OK;
}

gp_status gp_graph_stats(const gp_graph* g, gp_stats* out) {
    if (!g || !out) return GP_ERR_ARG;
    *out = g->dg.stats;
    return GP_OK;
}

gp_status gp_graph_new_id(const gp_graph* g, int32_t* new_id) {
    if (!g || !new_id) return GP_ERR_ARG;
    if (g->dg.n == 0) return GP_OK;
    DeviceGuard dgd(g->dg.device);
    GP_HIP_TRY(hipMemcpy(new_id, g->dg.new_id, sizeof(int32_t) * g->dg.n, hipMemcpyDeviceToHost));
    return GP_OK;
}

gp_status gp_graph_layout(const gp_graph* g, int64_t* row_ptr, int32_t* col) {
    if (!g || !row_ptr || (g->dg.nnz > 0 && !col)) return GP_ERR_ARG;
    DeviceGuard dgd(g->dg.device);
    GP_HIP_TRY(hipMemcpy(row_ptr, g->dg.row_ptr, sizeof(int64_t) * (g->dg.n + 1), hipMemcpyDeviceToHost));
    if (g->dg.nnz > 0)
        GP_HIP_TRY(hipMemcpy(col, g->dg.col, sizeof(int32_t) * g->dg.nnz, hipMemcpyDeviceToHost));
    return GP_OK;
}

void gp_free_graph(gp_graph* g) {
    if (!g) return;
    DeviceGuard dgd(g->dg.device);
    (void)hipDeviceSynchronize();
    free_device_graph(g->dg);
    delete g;
}

void gp_plan_opts_default(gp_plan_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->force_order[0] = -1;
    o->force_set = -1;
}

gp_status gp_plan_create(const int32_t* edges, int32_t k, int32_t e, const gp_stats* stats,
                         const gp_plan_opts* opts, gp_plan** out) {
    if (!out) return GP_ERR_ARG;
    const double t0 = now_seconds();
    gp_plan_opts o;
    gp_plan_opts_default(&o);
    if (opts) o = *opts;
    gp::Pattern pat;
    int rc = gp::parse_pattern(edges, k, e, &pat);
    if (rc) return rc;
    if (o.max_states < 0 || o.max_sets < 0 || o.iep < 0 || o.iep > GP_IEP_MAX_INNER) return GP_ERR_ARG;
    const int64_t max_states = o.max_states ? o.max_states : 4000000;
    const int32_t max_sets = o.max_sets ? o.max_sets : 100000;

    gp_plan* p = new (std::nothrow) gp_plan;
    if (!p) return GP_ERR_NOMEM;
    p->pattern = pat;
    auto auts = gp::automorphisms(pat);
    p->aut = auts.size();
    gp::RestrictionSets rs = cached_restriction_sets(pat, auts, max_states, max_sets,
                                                     o.max_seconds > 0 ? o.max_seconds : 20.0);
    p->sets = rs.sets;
    gp::Schedules sc = gp::efficient_schedules(pat);
    p->schedules = sc.orders;

    // candidate schedules
    std::vector<gp::Perm> cand_orders;
    if (o.force_order[0] >= 0) {
        gp::Perm ord{};
        unsigned seen = 0;
        for (int i = 0; i < k; ++i) {
            int v = o.force_order[i];
            if (v < 0 || v >= k || (seen & (1u << v))) {
                delete p;
                return GP_ERR_ARG;
            }
            seen |= 1u << v;
            ord[i] = uint8_t(v);
        }
        if (!gp::phase1_ok(pat, ord)) {
            delete p;
            return GP_ERR_ARG;
        }
        cand_orders.push_back(ord);
    } else {
        // one schedule per automorphism orbit: same costs, same argmin
        cand_orders = gp::orbit_representatives(p->schedules, auts, k);
    }
    // candidate restriction sets
    std::vector<gp::Rel> cand_sets;
    std::vector<int> cand_index;
    if (o.n_force_restr > 0) {
        if (o.n_force_restr > GP_MAX_K * GP_MAX_K) {
            delete p;
            return GP_ERR_ARG;
        }
        gp::Rel r = 0;
        for (int i = 0; i < o.n_force_restr; ++i) {
            int a = o.force_restr[2 * i], b = o.force_restr[2 * i + 1];
            if (a < 0 || a >= k || b < 0 || b >= k) {
                delete p;
                return GP_ERR_ARG;
            }
            r |= gp::rel_bit(a, b);
        }
        r = gp::closure(r, k);
        if (!gp::acyclic(r, k) || !gp::validate(r, k, p->aut)) {
            delete p;
            return GP_ERR_ARG;
        }
        // Also require that every non-identity automorphism is eliminated.
        for (size_t i = 1; i < auts.size(); ++i)
            if (gp::no_conflict(auts[i], r, k)) {
                delete p;
                return GP_ERR_ARG;
            }
        cand_sets.push_back(r);
        cand_index.push_back(-1);
    } else if (o.force_set >= 0) {
        if (o.force_set >= (int32_t)p->sets.size()) {
            delete p;
            return GP_ERR_ARG;
        }
        cand_sets.push_back(p->sets[o.force_set]);
        cand_index.push_back(o.force_set);
    } else {
        for (size_t i = 0; i < p->sets.size(); ++i) {
            cand_sets.push_back(p->sets[i]);
            cand_index.push_back(int(i));
        }
    }
    if (cand_sets.empty() || cand_orders.empty()) {
        delete p;
        return GP_ERR_UNSUPPORTED;
    }

    gp::GraphStats gs{1e6, 1e7, 6e7};
    if (stats && stats->n > 0 && stats->m > 0) {
        gs.n_v = double(stats->n);
        gs.n_e = double(stats->m);
        gs.tri_cnt = double(stats->tri_cnt);
    }
    double best = 0;
    int best_cuts = -1;
    size_t bo = 0, bs = 0;
    bool have = false;
    gp::Rel best_kept = 0;
    int best_div = 0, best_nin = 0;
    for (size_t i = 0; i < cand_orders.size(); ++i) {
        for (size_t j = 0; j < cand_sets.size(); ++j) {
            double c = gp::model_cost(pat, cand_orders[i], cand_sets[j], gs);
            int cuts = gp::upper_cuts(cand_orders[i], cand_sets[j], k);
            bool better;
            if (!have) {
                better = true;
            } else {
                double tol = 1e-9 * std::max(std::abs(best), std::abs(c));
                if (c < best - tol) better = true;
                else if (c > best + tol) better = false;
                else better = cuts > best_cuts;  // schedules/sets visited in order: earlier wins ties
            }
            gp::Rel kept = 0;
            int div = 0, nin = 0;
            if (better && o.iep) {
                // IEP over as many innermost levels as asked for and the
                // schedule allows, fewer if needed: only configurations whose
                // over-count is the same for every embedding
                const int want = o.iep == 1 ? GP_IEP_MAX_INNER : o.iep;
                for (int n = std::min(want, gp::iep_max_inner(pat, cand_orders[i])); n >= 2 && div <= 0; --n) {
                    div = gp::iep_setup(pat, auts, cand_orders[i], cand_sets[j], n, &kept);
                    nin = n;
                }
                if (div <= 0) better = false;
            }
            if (better) {
                best = c;
                best_cuts = cuts;
                bo = i;
                bs = j;
                best_kept = kept;
                best_div = div;
                best_nin = nin;
                have = true;
            }
        }
    }
    if (o.iep && !have) {
        // no configuration can be counted with IEP: plain enumeration
        o.iep = 0;
        for (size_t i = 0; i < cand_orders.size(); ++i)
            for (size_t j = 0; j < cand_sets.size(); ++j) {
                double c = gp::model_cost(pat, cand_orders[i], cand_sets[j], gs);
                int cuts = gp::upper_cuts(cand_orders[i], cand_sets[j], k);
                double tol = 1e-9 * std::max(std::abs(best), std::abs(c));
                if (!have || c < best - tol || (c <= best + tol && cuts > best_cuts)) {
                    best = c;
                    best_cuts = cuts;
                    bo = i;
                    bs = j;
                    have = true;
                }
            }
    }
    if (o.cost_cap > 0 && best > o.cost_cap) {
        delete p;
        return GP_ERR_BUDGET;
    }
    p->order = cand_orders[bo];
    p->set = cand_sets[bs];
    rc = gp::compile_plan(pat, p->order, p->set, &p->desc, best_kept, best_div, best_nin);
    if (rc) {
        delete p;
        return rc;
    }
    p->launch = gpint::default_launch(p->desc);
    gp_plan_info& in = p->info;
    std::memset(&in, 0, sizeof in);
    in.k = k;
    for (int i = 0; i < k; ++i) in.order[i] = p->order[i];
    int nr = 0;
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b)
            if (gp::rel_has(p->set, a, b)) {
                in.restr[2 * nr] = a;
                in.restr[2 * nr + 1] = b;
                ++nr;
            }
    in.n_restr = nr;
    in.aut = p->aut;
    in.cost = best;
    in.n_sets = (int32_t)p->sets.size();
    in.n_states = rs.states;
    in.n_schedules = (int32_t)p->schedules.size();
    in.k_eff = sc.k_eff;
    in.set_index = cand_index[bs];
    in.plan_seconds = now_seconds() - t0;
    in.tuned = 0;
    in.iep = p->desc.iep;
    in.iep_div = p->desc.iep_div;
    *out = p;
    return GP_OK;
}

gp_status gp_plan_get(const gp_plan* p, gp_plan_info* out) {
    if (!p || !out) return GP_ERR_ARG;
    *out = p->info;
    out->launch.group = p->launch.group;
    out->launch.waves_per_cu = p->launch.waves_per_cu;
    out->launch.chunk = p->launch.chunk;
    out->launch.leaf_mode = p->launch.leaf;
    out->launch.root_stride = 0;
    out->launch.root_offset = 0;
    out->launch.split_ways = p->launch.split_ways;
    out->launch.split_vertices = (int32_t)std::min<int64_t>(p->launch.split_vertices, INT32_MAX);
    out->launch.xcd_tasks = (int32_t)std::max<int64_t>(-1, std::min<int64_t>(p->launch.xcd, INT32_MAX));
    out->launch.batch_runs = p->launch.batch_runs;
    return GP_OK;
}

gp_status gp_plan_get_set(const gp_plan* p, int32_t idx, int32_t* n_restr, int32_t* restr) {
    if (!p || !n_restr || !restr || idx < 0 || idx >= (int32_t)p->sets.size()) return GP_ERR_ARG;
    int nr = 0;
    const int k = p->pattern.k;
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b)
            if (gp::rel_has(p->sets[idx], a, b)) {
                restr[2 * nr] = a;
                restr[2 * nr + 1] = b;
                ++nr;
            }
    *n_restr = nr;
    return GP_OK;
}

gp_status gp_plan_get_schedule(const gp_plan* p, int32_t idx, int32_t* order) {
    if (!p || !order || idx < 0 || idx >= (int32_t)p->schedules.size()) return GP_ERR_ARG;
    for (int i = 0; i < p->pattern.k; ++i) order[i] = p->schedules[idx][i];
    return GP_OK;
}

gp_status gp_plan_model_cost(const gp_plan* p, int32_t idx_s, int32_t idx_r, const gp_stats* stats,
                             double* cost) {
    if (!p || !cost || idx_s < 0 || idx_s >= (int32_t)p->schedules.size() || idx_r < 0 ||
        idx_r >= (int32_t)p->sets.size())
        return GP_ERR_ARG;
    gp::GraphStats gs{1e6, 1e7, 6e7};
    if (stats && stats->n > 0 && stats->m > 0) {
        gs.n_v = double(stats->n);
        gs.n_e = double(stats->m);
        gs.tri_cnt = double(stats->tri_cnt);
    }
    *cost = gp::model_cost(p->pattern, p->schedules[idx_s], p->sets[idx_r], gs);
    return GP_OK;
}

gp_status gp_plan_with_launch(const gp_plan* p, const gp_launch* launch, gp_plan** out) {
    if (!p || !launch || !out) return GP_ERR_ARG;
    const gp_launch& l = *launch;
    if ((l.group && l.group != 64 && l.group != 32 && l.group != 16 && l.group != 8) ||
        (l.leaf_mode && (l.leaf_mode < 1 || l.leaf_mode > 4)) || (l.waves_per_cu && (l.waves_per_cu < 1 || l.waves_per_cu > 32)) ||
        l.chunk < 0 || l.split_ways < 0 || l.split_vertices < 0 || l.xcd_tasks < -1 || l.batch_runs < 0 ||
        l.batch_runs > 2)
        return GP_ERR_ARG;
    gp_plan* q = new (std::nothrow) gp_plan(*p);
    if (!q) return GP_ERR_NOMEM;
    gp_launch f = l;
    f.root_stride = 0;
    f.root_offset = 0;
    q->launch = gpint::apply_launch(q->launch, &f);
    *out = q;
    return GP_OK;
}

void gp_free_plan(gp_plan* p) { delete p; }

void gp_launch_default(gp_launch* l) {
    if (l) std::memset(l, 0, sizeof *l);
}

gp_status gp_count(const gp_graph* g, const gp_plan* p, const gp_launch* launch, void* stream,
                   uint64_t* out) {
    if (!g || !p || !out) return GP_ERR_ARG;
    DeviceGuard dgd(g->dg.device);
    gpint::LaunchCfg cfg = gpint::launch_for_plan(p, launch, g->dg);
    return count_to_host(g, p->desc, cfg, (hipStream_t)stream, nullptr, out);
}

gp_status gp_count_async(const gp_graph* g, const gp_plan* p, const gp_launch* launch, void* stream,
                         uint64_t* dev_out) {
    if (!g || !p || !dev_out) return GP_ERR_ARG;
    DeviceGuard dgd(g->dg.device);
    gpint::LaunchCfg cfg = gpint::launch_for_plan(p, launch, g->dg);
    return gpint::launch_count(g->dg, p->desc, cfg, (hipStream_t)stream,
                               reinterpret_cast<unsigned long long*>(dev_out), nullptr);
}

gp_status gp_count_noalloc(const gp_graph* g, const gp_plan* p, const gp_launch* launch, void* stream,
                           uint64_t* dev_out) {
    if (!g || !p || !dev_out) return GP_ERR_ARG;
    DeviceGuard dgd(g->dg.device);
    gpint::LaunchCfg cfg = gpint::launch_for_plan(p, launch, g->dg);
    return gpint::launch_count_noalloc(g->dg, p->desc, cfg, (hipStream_t)stream,
                                       reinterpret_cast<unsigned long long*>(dev_out));
}

gp_status gp_count_per_root(const gp_graph* g, const gp_plan* p, const gp_launch* launch, void* stream,
                            uint64_t* dev_per_root, uint64_t* out) {
    if (!g || !p || !dev_per_root || !out) return GP_ERR_ARG;
    DeviceGuard dgd(g->dg.device);
    hipStream_t s = (hipStream_t)stream;
    if (g->dg.nnz > 0) GP_HIP_TRY(hipMemsetAsync(dev_per_root, 0, sizeof(uint64_t) * g->dg.nnz, s));
    gpint::LaunchCfg cfg = gpint::launch_for_plan(p, launch, g->dg);
    return count_to_host(g, p->desc, cfg, s, reinterpret_cast<unsigned long long*>(dev_per_root), out);
}

gp_status gp_count_traffic(const gp_graph* g, const gp_plan* p, const gp_launch* launch, void* stream,
                           uint64_t* out, uint64_t* alg_bytes) {
    if (!g || !p || !out || !alg_bytes) return GP_ERR_ARG;
    DeviceGuard dgd(g->dg.device);
    gpint::LaunchCfg cfg = gpint::launch_for_plan(p, launch, g->dg);
    return count_to_host(g, p->desc, cfg, (hipStream_t)stream, nullptr, out, alg_bytes);
}

gp_status gp_check_sum(const uint64_t* values, int64_t n, uint64_t div, void* stream, uint64_t* out,
                       uint32_t* flags) {
    if (!out || !flags) return GP_ERR_ARG;
    return gpint::check_sum(values, n, div, (hipStream_t)stream, out, flags);
}

gp_status gp_list(const gp_graph* g, const gp_plan* p, const gp_launch* launch, void* stream, int32_t* out,
                  uint64_t capacity, uint64_t* n_found) {
    if (!g || !p || !n_found || (capacity > 0 && !out)) return GP_ERR_ARG;
    const int k = p->desc.k;
    if (k < 2 || k > GP_MAX_K || capacity > (uint64_t)INT64_MAX / (uint64_t)k) return GP_ERR_ARG;
    if (p->desc.iep) return GP_ERR_UNSUPPORTED;
    DeviceGuard dgd(g->dg.device);
    hipStream_t s = (hipStream_t)stream;
    gpint::LaunchCfg cfg = gpint::launch_for_plan(p, launch, g->dg);
    int32_t order[GP_MAX_K] = {};
    for (int i = 0; i < k; ++i) order[i] = p->order[i];
    unsigned long long* res = nullptr;
    GP_HIP_TRY(hipMallocAsync((void**)&res, 2 * sizeof(unsigned long long), s));
    gp_status st = gpint::launch_list(g->dg, p->desc, order, cfg, s, res, out, (int64_t)capacity);
    unsigned long long h[2] = {0, 0};
    if (st == GP_OK && hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, s) != hipSuccess) st = GP_ERR_HIP;
    (void)hipFreeAsync(res, s);
    if (hipStreamSynchronize(s) != hipSuccess && st == GP_OK) st = GP_ERR_HIP;
    if (st != GP_OK) return st;
    *n_found = h[0];
    return GP_OK;
}

namespace {
// Device descriptors and per-plan launch shapes of a batch, in the order the
// batch runs them. Plans of one launch shape run together in one launch
// (shapes in the order of their longest measured plan); within a shape, by
// measured (tuned) run time, longest first, so the light plans fill the tail
// of the heavy ones; untimed plans keep their order after the timed ones.
// slot[i] is where the caller's plan i runs.
gp_status batch_inputs(const gp_graph* g, const gp_plan* const* plans, int32_t np, const gp_launch* launch,
                       std::vector<GpPlanDesc>* descs, std::vector<gpint::LaunchCfg>* cfgs,
                       std::vector<int>* slot, int* waves_per_cu) {
    if (!plans || np < 1 || np > 64) return GP_ERR_ARG;
    std::vector<int> ord(np);
    std::vector<gpint::LaunchCfg> cfg(np);
    std::vector<int> key(np);
    for (int i = 0; i < np; ++i) {
        if (!plans[i]) return GP_ERR_ARG;
        ord[i] = i;
        cfg[i] = gpint::launch_for_plan(plans[i], launch, g->dg);
        key[i] = gpint::batch_shape_key(plans[i]->desc, cfg[i], 8);
    }
    // a shape's rank: its longest plan
    std::map<int, double> shape_ms;
    for (int i = 0; i < np; ++i) {
        auto it = shape_ms.find(key[i]);
        if (it == shape_ms.end()) shape_ms[key[i]] = plans[i]->tuned_ms;
        else it->second = std::max(it->second, plans[i]->tuned_ms);
    }
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
        if (key[a] != key[b]) {
            const double ma = shape_ms[key[a]], mb = shape_ms[key[b]];
            return ma != mb ? ma > mb : key[a] < key[b];
        }
        return plans[a]->tuned_ms > plans[b]->tuned_ms;
    });
    descs->resize(np);
    cfgs->resize(np);
    slot->resize(np);
    for (int r = 0; r < np; ++r) {
        const int i = ord[r];
        (*descs)[r] = plans[i]->desc;
        (*cfgs)[r] = cfg[i];
        (*slot)[i] = r;
    }
    *waves_per_cu = launch && launch->waves_per_cu ? launch->waves_per_cu : 32;
    if (*waves_per_cu < 1 || *waves_per_cu > 32) return GP_ERR_ARG;
    return GP_OK;
}

// Counts of a finished batch from its result words (4 per plan, batch order).
// A plan whose launch counts a root sample (stride above 1 or an offset) is
// not whole: its IEP quotient is rounded down, not checked.
gp_status batch_counts(const std::vector<GpPlanDesc>& descs, const std::vector<gpint::LaunchCfg>& cfgs,
                       const std::vector<int>& slot, const unsigned long long* res, uint64_t* out) {
    const int np = (int)slot.size();
    std::vector<uint64_t> tmp(np);
    for (int i = 0; i < np; ++i) {
        const int r = slot[i];
        const bool whole = cfgs[r].root_stride <= 1 && cfgs[r].root_offset == 0;
        gp_status st = gpint::batch_result(descs[r], res + 4 * r, &tmp[i], whole);
        if (st != GP_OK) return st;
    }
    for (int i = 0; i < np; ++i) out[i] = tmp[i];
    return GP_OK;
}
}  // namespace

gp_status gp_count_batch(const gp_graph* g, const gp_plan* const* plans, int32_t np,
                         const gp_launch* launch, void* stream, uint64_t* out) {
    if (!g || !out) return GP_ERR_ARG;
    std::vector<GpPlanDesc> descs;
    std::vector<gpint::LaunchCfg> cfgs;
    std::vector<int> slot;
    int wpc = 32;
    gp_status st = batch_inputs(g, plans, np, launch, &descs, &cfgs, &slot, &wpc);
    if (st != GP_OK) return st;
    DeviceGuard dgd(g->dg.device);
    hipStream_t s = (hipStream_t)stream;
    gpint::BatchState bs;
    st = gpint::batch_prepare(g->dg, descs.data(), cfgs.data(), nullptr, nullptr, np, wpc, s, &bs);
    if (st != GP_OK) return st;
    std::vector<unsigned long long> h(4 * np, 0);
    st = gpint::batch_enqueue(g->dg, bs, s);
    if (st == GP_OK &&
        hipMemcpyAsync(h.data(), bs.result, sizeof(unsigned long long) * 4 * np, hipMemcpyDeviceToHost, s) !=
            hipSuccess)
        st = GP_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess && st == GP_OK) st = GP_ERR_HIP;
    gpint::batch_release(&bs);
    if (st != GP_OK) return st;
    return batch_counts(descs, cfgs, slot, h.data(), out);
}

namespace {
// Capture the batch's work into its hipGraph (replacing an earlier one):
// counter and memo reset (fill kernels, no memset nodes) -> the runs' launches
// -> D2H of the result words.
bool capture_batch(gp_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
    gp_status est = gpint::batch_enqueue(b->g->dg, b->st, b->cap_stream);
    hipError_t ce = hipMemcpyAsync(b->host_res, b->st.result, 4 * sizeof(unsigned long long) * b->np,
                                   hipMemcpyDeviceToHost, b->cap_stream);
    hipError_t ee = hipStreamEndCapture(b->cap_stream, &b->graph);
    return est == GP_OK && ce == hipSuccess && ee == hipSuccess &&
           hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess;
}
}  // namespace

gp_status gp_batch_create(const gp_graph* g, const gp_plan* const* plans, int32_t np,
                          const gp_launch* launch, void* stream, gp_batch** out) {
    if (!g || !out) return GP_ERR_ARG;
    std::vector<GpPlanDesc> descs;
    std::vector<gpint::LaunchCfg> cfgs;
    std::vector<int> slot;
    int wpc = 32;
    gp_status st = batch_inputs(g, plans, np, launch, &descs, &cfgs, &slot, &wpc);
    if (st != GP_OK) return st;
    DeviceGuard dgd(g->dg.device);
    hipStream_t s = (hipStream_t)stream;
    gp_batch* b = new (std::nothrow) gp_batch;
    if (!b) return GP_ERR_NOMEM;
    b->g = g;
    b->np = np;
    b->descs = descs;
    b->cfgs = cfgs;
    b->slot = slot;
    st = gpint::batch_prepare(g->dg, descs.data(), cfgs.data(), nullptr, nullptr, np, wpc, s, &b->st);
    if (st != GP_OK) {
        delete b;
        return st;
    }
    bool ok = hipHostMalloc((void**)&b->host_res, 4 * sizeof(unsigned long long) * np,
                            hipHostMallocDefault) == hipSuccess &&
              hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) == hipSuccess &&
              capture_batch(b);
    if (!ok) {
        gp_free_batch(b);
        return GP_ERR_HIP;
    }
    *out = b;
    return GP_OK;
}

gp_status gp_batch_run(gp_batch* b, void* stream, uint64_t* out) {
    if (!b || !out) return GP_ERR_ARG;
    DeviceGuard dgd(b->g->dg.device);
    hipStream_t s = (hipStream_t)stream;
    GP_HIP_TRY(hipGraphLaunch(b->exec, s));
    GP_HIP_TRY(hipStreamSynchronize(s));
    return batch_counts(b->descs, b->cfgs, b->slot, b->host_res, out);
}

gp_status gp_batch_set_sample(gp_batch* b, int64_t root_stride, int64_t root_offset, void* stream) {
    if (!b || root_stride < 1 || root_offset < 0) return GP_ERR_ARG;
    DeviceGuard dgd(b->g->dg.device);
    hipStream_t s = (hipStream_t)stream;
    GP_HIP_TRY(hipStreamSynchronize(s));
    if (b->cap_stream) GP_HIP_TRY(hipStreamSynchronize(b->cap_stream));
    std::vector<gpint::LaunchCfg> cfgs = b->cfgs;
    for (auto& c : cfgs) {
        c.root_stride = root_stride;
        c.root_offset = root_offset;
    }
    gp_status st = gpint::batch_update(b->g->dg, &b->st, b->descs.data(), cfgs.data(), s);
    if (st == GP_OK) {
        b->cfgs = cfgs;
        if (!capture_batch(b)) st = GP_ERR_HIP;
    }
    return st;
}

gp_status gp_batch_tune(const gp_graph* g, const gp_plan* const* plans, int32_t np, void* stream,
                        gp_launch* out, double* best_ms) {
    if (!g || !out) return GP_ERR_ARG;
    DeviceGuard dgd(g->dg.device);
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        return GP_ERR_HIP;
    }
    gp_status st = GP_OK;
    double best = -1;
    gp_launch pick{};
    // each plan at its own shape (all fields zero), sharing launches by shape
    // and each in a launch of its own, then one shape for all
    std::vector<gp_launch> shapes(2, gp_launch{});
    shapes[1].batch_runs = 2;
    for (int grp : {64, 32, 16})
        for (int lm : {1, 3, 4}) {
            gp_launch l{};
            l.group = grp;
            l.leaf_mode = lm;
            shapes.push_back(l);
        }
    for (const gp_launch& l : shapes) {
        std::vector<GpPlanDesc> descs;
        std::vector<gpint::LaunchCfg> cfgs;
        std::vector<int> slot;
        int wpc = 32;
        st = batch_inputs(g, plans, np, &l, &descs, &cfgs, &slot, &wpc);
        if (st != GP_OK) break;
        gpint::BatchState bs;
        st = gpint::batch_prepare(g->dg, descs.data(), cfgs.data(), nullptr, nullptr, np, wpc, s, &bs);
        if (st != GP_OK) break;
        float ms = 0;
        if (hipEventRecord(a, s) != hipSuccess || gpint::batch_enqueue(g->dg, bs, s) != GP_OK ||
            hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
            hipEventElapsedTime(&ms, a, b) != hipSuccess)
            st = GP_ERR_HIP;
        gpint::batch_release(&bs);
        if (st != GP_OK) break;
        if (best < 0 || ms < best) {
            best = ms;
            pick = l;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != GP_OK) return st;
    *out = pick;
    if (best_ms) *best_ms = best;
    return GP_OK;
}

void gp_free_batch(gp_batch* b) {
    if (!b) return;
    DeviceGuard dgd(b->g->dg.device);
    if (b->cap_stream) (void)hipStreamSynchronize(b->cap_stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    (void)hipDeviceSynchronize();
    if (b->host_res) (void)hipHostFree(b->host_res);
    gpint::batch_release(&b->st);
    delete b;
}

}  // extern "C"
