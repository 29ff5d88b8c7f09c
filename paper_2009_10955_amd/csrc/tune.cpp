// Measured configuration selection (gp_plan_tune).
//
// The paper picks one (schedule, restriction set) by its cost model
// (Section IV-C), which sees only |V|, |E| and tri_cnt, and reports the pick
// 32% slower than the best schedule on average (Section V-C). On a
// degree-sorted layout the direction of each restriction also decides whether
// the search walks hub lists or short ones, which the model cannot see. So the
// best-ranked configurations and their mirrors are timed on a strided sample
// of their own root tasks, and the fastest wins; then the launch shape is
// timed for it. Results are cached per (graph hash, pattern).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "api_internal.hpp"

namespace {
// Sampling strides are odd: the all-orientations root array interleaves (u, v)
// and (v, u), so an even stride would sample one orientation only.
int64_t odd_stride(int64_t s) {
    return s <= 1 ? 1 : (s | 1);
}

}  // namespace

namespace gpint {

LaunchCfg launch_for_plan(const gp_plan* p, const gp_launch* l, const DeviceGraph& g) {
    (void)g;
    return apply_launch(p->launch, l);
}

gp_status estimate_begin(const DeviceGraph& g, const GpPlanDesc& d, LaunchCfg cfg, double budget_ms,
                         hipStream_t s, unsigned long long* res, int64_t* stride_out) {
    const int64_t roots = std::max<int64_t>(1, root_task_count(g, d));
    const int64_t stride = odd_stride(std::max<int64_t>(1, roots / 4096));
    *stride_out = stride;
    cfg.root_stride = stride;
    cfg.root_offset = 0;  // the first root is the heaviest: its tail shows
    cfg.budget_ms = budget_ms;
    return launch_count(g, d, cfg, s, res, nullptr, false, res + 2);
}

double estimate_end(const DeviceGraph& g, const GpPlanDesc& d, const LaunchCfg& cfg,
                    const unsigned long long* h, int64_t stride) {
    if (h[1] & 4ull) return 1e300;  // a wavefront of the sample alone ran past the budget
    const double busy = (double)h[2] / g.wall_khz, chunk = (double)h[4] / g.wall_khz;
    const double resident = (double)g.num_cus * resident_waves_per_cu(g, d, cfg);
    return std::max(busy * (double)stride / resident, chunk);
}

double estimate_full_ms(const DeviceGraph& g, const GpPlanDesc& d, LaunchCfg cfg, double budget_ms,
                        hipStream_t s, unsigned long long* res, uint64_t* sample_count, int64_t* sample_stride) {
    int64_t stride = 1;
    unsigned long long h[5] = {0, 0, 0, 0, 0};
    if (estimate_begin(g, d, cfg, budget_ms, s, res, &stride) != GP_OK ||
        hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return -1;
    if (sample_stride) *sample_stride = stride;
    if (sample_count) *sample_count = h[0];
    return estimate_end(g, d, cfg, h, stride);
}

}  // namespace gpint

namespace {

double now_seconds() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

gp::Rel mirror(gp::Rel r, int k) {
    gp::Rel m = 0;
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b)
            if (gp::rel_has(r, a, b)) m |= gp::rel_bit(b, a);
    return m;
}

struct Cfg {
    gp::Perm order;
    gp::Rel rel;
    GpPlanDesc desc;
};

struct Cached {
    gp::Perm order;
    gp::Rel rel;
    GpPlanDesc desc;
    gpint::LaunchCfg launch;
    int measured;
    double ms;
};

std::mutex g_cache_mu;
std::map<std::tuple<uint64_t, int64_t, int, std::vector<std::pair<int, int>>>, Cached> g_cache;

// One measured launch of a root sample. The kernel reports the summed
// active time of its wavefronts and the longest chunk of tasks any of them
// ran; with the sample's stride these give the full run's time as
//   max(busy * stride / resident wavefronts, longest chunk):
// the balanced share of the work, or the tail of the heaviest task, whichever
// is longer. Wall time of a small sample alone mostly measures that tail.
struct Timing {
    double wall = -1;   // ms, negative on failure
    double busy = 0;    // wavefront-ms
    double chunk = 0;   // ms
    long long waves = 0;
    bool stopped = false;  // hit the time budget: slower than the budget allows
};

Timing time_launch(const gpint::DeviceGraph& g, const GpPlanDesc& d, const gpint::LaunchCfg& cfg,
                   hipStream_t s, unsigned long long* res) {
    Timing out;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return out;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return out;
    }
    unsigned long long h[5] = {0, 0, 0, 0, 0};
    if (hipEventRecord(a, s) == hipSuccess &&
        gpint::launch_count(g, d, cfg, s, res, nullptr, false, res + 2) == GP_OK &&
        hipEventRecord(b, s) == hipSuccess &&
        hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, s) == hipSuccess &&
        hipStreamSynchronize(s) == hipSuccess) {
        float f = 0;
        if (hipEventElapsedTime(&f, a, b) == hipSuccess) {
            out.wall = f;
            out.stopped = (h[1] & 4ull) != 0;
            out.busy = (double)h[2] / g.wall_khz;
            out.waves = (long long)h[3];
            out.chunk = (double)h[4] / g.wall_khz;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return out;
}

bool verbose() {
    static const bool v = [] {
        const char* e = std::getenv("GP_TUNE_VERBOSE");
        return e && *e && *e != '0';
    }();
    return v;
}

}  // namespace

extern "C" {

void gp_tune_opts_default(gp_tune_opts* o) {
    if (o) std::memset(o, 0, sizeof *o);
}

gp_status gp_plan_tune(const gp_graph* g, const gp_plan* p, const gp_tune_opts* opts, void* stream,
                       gp_plan** out) {
    if (!g || !p || !out) return GP_ERR_ARG;
    gp_tune_opts o;
    gp_tune_opts_default(&o);
    if (opts) o = *opts;
    if (o.max_configs < 0 || o.sample_stride < 0 || o.budget_seconds < 0) return GP_ERR_ARG;
    const int max_configs = o.max_configs ? o.max_configs : 24;
    const double budget_ms = 1e3 * (o.budget_seconds > 0 ? o.budget_seconds : 20.0);
    const double t0 = now_seconds();
    const int k = p->pattern.k;
    hipStream_t s = (hipStream_t)stream;
    int prev_dev = -1;
    (void)hipGetDevice(&prev_dev);
    if (prev_dev != g->dg.device) (void)hipSetDevice(g->dg.device);

    gp_plan* np = new (std::nothrow) gp_plan(*p);
    if (!np) return GP_ERR_NOMEM;

    auto edges = p->pattern.edges;
    for (auto& e : edges)
        if (e.first > e.second) std::swap(e.first, e.second);
    std::sort(edges.begin(), edges.end());
    const bool try_iep = o.try_iep > 0 && !p->desc.iep;
    auto key = std::make_tuple(g->dg.stats.hash,
                               (int64_t)g->dg.n_hubs * 4 + (p->desc.iep ? 1 : 0) + (try_iep ? 2 : 0), k, edges);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            np->order = it->second.order;
            np->set = it->second.rel;
            np->launch = it->second.launch;
            np->tuned = true;
            np->desc = it->second.desc;
            np->info.n_measured = it->second.measured;
            np->tuned_ms = it->second.ms;
        }
    }

    gp_status st = GP_OK;
    unsigned long long* res = nullptr;
    if (!np->tuned) {
        if (hipMallocAsync((void**)&res, 5 * sizeof(unsigned long long), s) != hipSuccess) {  // {count, flags, busy[3]}
            delete np;
            return GP_ERR_HIP;
        }
        // 1. candidates: model ranking, each followed by its mirror, distinct searches only
        gp::GraphStats gs{double(std::max<int64_t>(1, g->dg.stats.n)),
                          double(std::max<int64_t>(1, g->dg.stats.m)),
                          double(g->dg.stats.tri_cnt)};
        struct Ranked {
            double cost;
            size_t i, j;
        };
        std::vector<Ranked> ranked;
        std::vector<gp::Perm> auts0 = gp::automorphisms(p->pattern);
        std::vector<gp::Perm> reps = gp::orbit_representatives(p->schedules, auts0, k);
        for (size_t i = 0; i < reps.size(); ++i)
            for (size_t j = 0; j < p->sets.size(); ++j)
                ranked.push_back({gp::model_cost(p->pattern, reps[i], p->sets[j], gs), i, j});
        std::stable_sort(ranked.begin(), ranked.end(),
                         [](const Ranked& a, const Ranked& b) { return a.cost < b.cost; });
        std::vector<Cfg> cands;
        std::vector<gp::Perm> auts = gp::automorphisms(p->pattern);
        // with try_iep every configuration may come several times: counted
        // plainly and with inclusion-exclusion over its 2, 3 or 4 last levels
        const int cap = try_iep ? 3 * max_configs : max_configs;
        auto add_one = [&](const gp::Perm& order, gp::Rel rel, int n_in) {
            if ((int)cands.size() >= cap) return;
            Cfg c;
            c.order = order;
            c.rel = rel;
            gp::Rel kept = 0;
            int div = 0;
            if (n_in > 0) {
                div = gp::iep_setup(p->pattern, auts, order, rel, n_in, &kept);
                if (div <= 0) return;
            }
            if (gp::compile_plan(p->pattern, order, rel, &c.desc, kept, div, n_in) != 0) return;
            for (auto& x : cands)
                if (std::memcmp(&x.desc, &c.desc, sizeof c.desc) == 0) return;
            cands.push_back(c);
        };
        auto add = [&](const gp::Perm& order, gp::Rel rel) {
            if ((int)cands.size() >= cap) return;
            // a mirrored set is valid whenever the original is; check anyway
            if (!gp::acyclic(rel, k) || !gp::validate(rel, k, p->aut)) return;
            for (size_t q = 1; q < auts.size(); ++q)
                if (gp::no_conflict(auts[q], rel, k)) return;
            // the plan's own mode (its number of IEP levels, where this
            // configuration allows as many), then with try_iep every IEP depth
            const int nmax = gp::iep_max_inner(p->pattern, order);
            add_one(order, rel, p->desc.iep ? std::min<int>(p->desc.iep, nmax) : 0);
            if (try_iep)
                for (int n = nmax; n >= 2; --n) add_one(order, rel, n);
        };
        add(p->order, p->set);
        add(p->order, mirror(p->set, k));
        for (auto& r : ranked) {
            if ((int)cands.size() >= cap) break;
            add(reps[r.i], p->sets[r.j]);
            add(reps[r.i], mirror(p->sets[r.j], k));
        }

        double spent = 0;
        const double inf = 1e300;
        double best_est = inf;  // best full-run estimate so far (ms)
        // full-run estimate (ms) of one sampled launch; inf if it failed or stopped
        auto measure = [&](const GpPlanDesc& d, gpint::LaunchCfg cfg, int64_t str, const char* what,
                           size_t c, bool saturate = false) -> double {
            if (saturate) {
                // comparing launch shapes: the sample must keep every resident
                // group of this shape busy (about two tasks each, one per grab),
                // or narrower groups run with less contention than they will
                const int64_t groups = (int64_t)g->dg.num_cus * gpint::resident_waves_per_cu(g->dg, d, cfg) *
                                       (64 / std::max(1, cfg.group));
                const int64_t roots = gpint::root_task_count(g->dg, d);
                str = std::max<int64_t>(1, std::min<int64_t>(str, roots / std::max<int64_t>(1, 2 * groups)));
                cfg.chunk = 1;
            }
            str = odd_stride(str);
            cfg.root_stride = str;
            cfg.root_offset = 0;  // the first root is the heaviest: its tail shows
            cfg.budget_ms = best_est < inf ? std::max(20.0, 3.0 * best_est) : 0.0;
            Timing t = time_launch(g->dg, d, cfg, s, res);
            if (t.wall < 0) {
                st = GP_ERR_HIP;
                return -1;
            }
            spent += t.wall;
            const double resident = (double)g->dg.num_cus * gpint::resident_waves_per_cu(g->dg, d, cfg);
            // a sample of stride 1 is the full run: its wall time is the answer
            const double est = t.stopped ? inf
                               : str == 1 ? t.wall
                                          : std::max(t.busy * (double)str / resident, t.chunk);
            if (verbose())
                std::fprintf(stderr,
                             "gp_plan_tune %s cand %zu stride %lld group %d leaf %d waves %d split %dx%lld: "
                             "wall %.3f ms, busy %.1f wave-ms over %lld wavefronts, longest chunk %.3f ms%s, "
                             "estimate %.3f ms\n",
                             what, c, (long long)str, cfg.group, cfg.leaf, cfg.waves_per_cu, cfg.split_ways,
                             (long long)cfg.split_vertices, t.wall, t.busy, t.waves, t.chunk,
                             t.stopped ? " (stopped)" : "", est < inf ? est : -1.0);
            if (est < best_est) best_est = est;
            return est;
        };

        // 2. sample stride: the planner's configuration gives the work; the
        //    sample keeps a balanced share of about 8 ms of it
        const gpint::LaunchCfg base = gpint::default_launch(p->desc);
        int64_t stride = o.sample_stride;
        if (stride <= 0) {
            const int64_t roots = std::max<int64_t>(1, gpint::root_task_count(g->dg, p->desc));
            const int64_t s0 = odd_stride(std::max<int64_t>(1, roots / 4096));
            gpint::LaunchCfg cfg = base;
            cfg.root_stride = s0;
            cfg.root_offset = 0;
            cfg.budget_ms = budget_ms;  // a sample that runs past it still gives a lower bound
            Timing t = time_launch(g->dg, p->desc, cfg, s, res);
            if (t.wall < 0) st = GP_ERR_HIP;
            spent += std::max(0.0, t.wall);
            const double resident = (double)g->dg.num_cus * gpint::resident_waves_per_cu(g->dg, p->desc, base);
            const double full_ms = t.busy * (double)s0 / resident;
            stride = std::max<int64_t>(1, (int64_t)(full_ms / 8.0));
            stride = std::min(stride, s0);
            if (verbose())
                std::fprintf(stderr, "gp_plan_tune calibration: %lld roots, balanced full run ~%.1f ms, stride %lld\n",
                             (long long)roots, full_ms, (long long)stride);
        }

        // 3. every configuration on a sample 4x sparser, then the four best
        //    again on the full sample, all with the default launch shape
        std::vector<std::pair<double, size_t>> coarse;
        int measured = 0;
        for (size_t c = 0; st == GP_OK && c < cands.size(); ++c) {
            if (spent > budget_ms && measured > 0) break;
            double t = measure(cands[c].desc, base, stride * 4, "coarse", c);
            if (t < 0) break;
            ++measured;
            coarse.push_back({t, c});
        }
        std::stable_sort(coarse.begin(), coarse.end());
        std::vector<std::pair<double, size_t>> fine;
        best_est = inf;
        for (size_t r = 0; st == GP_OK && r < coarse.size() && r < 4; ++r) {
            if (spent > 1.5 * budget_ms && !fine.empty()) break;
            if (coarse[r].first >= inf && !fine.empty()) break;
            size_t c = coarse[r].second;
            double t = measure(cands[c].desc, base, stride, "fine", c);
            if (t < 0) break;
            fine.push_back({t, c});
        }
        std::stable_sort(fine.begin(), fine.end());

        // 4. launch shape for the two best configurations: group width and
        //    leaf mode change which configuration is fastest. Root splitting
        //    stays at its default here: the tail it removes comes from the few
        //    heaviest roots, which a strided sample mostly misses; the last
        //    stage sets it from full runs
        struct Pick {
            double est;
            size_t c;
            gpint::LaunchCfg launch;
        };
        std::vector<Pick> picks;
        std::vector<Pick> tried;  // every (configuration, shape) measured on the full sample
        const int n_shape = o.tune_launch >= 0 ? 2 : 1;
        // the two best, and the planner's own configuration (candidate 0) as well
        std::vector<std::pair<double, size_t>> shape_set(fine.begin(),
                                                         fine.begin() + std::min<size_t>(fine.size(), n_shape));
        bool has0 = false;
        for (auto& f : shape_set) has0 |= f.second == 0;
        if (!has0 && o.tune_launch >= 0)
            for (auto& f : coarse)
                if (f.second == 0) shape_set.push_back({f.first, 0});
        auto leaf_ok = [&](const GpPlanDesc& bd, int lm) {
            if (lm == 2) return !bd.iep && (k <= 3 || bd.lv[k - 1].last_list >= 0);
            if (lm == 3) return k >= 5 && !bd.iep && bd.build_begin[k - 3] == bd.build_end[k - 3];
            if (lm == 4) return k >= 4 && !bd.iep && bd.lv[k - 1].last_list == k - 2;
            return true;
        };
        // pass A: every leaf mode with 64-lane groups, for each configuration
        for (size_t r = 0; st == GP_OK && r < shape_set.size(); ++r) {
            const size_t c = shape_set[r].second;
            Pick pk{shape_set[r].first, c, base};
            if (o.tune_launch >= 0) {
                const GpPlanDesc& bd = cands[c].desc;
                best_est = inf;
                pk.est = measure(bd, base, stride, "shape", c, true);
                if (pk.est < 0) break;
                tried.push_back(pk);
                // leaf 2 (a group walk per candidate) last: it rarely wins for
                // k >= 5, and its samples are the slowest, so the budget that
                // remains goes to it
                for (int lm : {3, 4, 2}) {
                    if (!leaf_ok(bd, lm) || spent > 2.5 * budget_ms) continue;
                    gpint::LaunchCfg cfg = base;
                    cfg.leaf = lm;
                    double t = measure(bd, cfg, stride, "shape", c, true);
                    if (t < 0) break;
                    tried.push_back(Pick{t, c, cfg});
                    if (t < pk.est) {
                        pk.est = t;
                        pk.launch = cfg;
                    }
                }
            }
            picks.push_back(pk);
        }
        std::stable_sort(picks.begin(), picks.end(), [](const Pick& a, const Pick& b) { return a.est < b.est; });
        // pass B: narrower groups for the two best, while they stay within 1.5x
        for (size_t r = 0; st == GP_OK && o.tune_launch >= 0 && r < picks.size() && r < 2; ++r) {
            Pick& pk = picks[r];
            const GpPlanDesc& bd = cands[pk.c].desc;
            best_est = pk.est;
            for (int grp : {32, 16, 8}) {
                if (bd.iep && grp < 32) continue;
                double best_g = inf;
                for (int lm : {1, 2, 3, 4}) {
                    if (!leaf_ok(bd, lm) || spent > 2.5 * budget_ms) continue;
                    gpint::LaunchCfg cfg = base;
                    cfg.group = grp;
                    cfg.leaf = lm;
                    double t = measure(bd, cfg, stride, "shape", pk.c, true);
                    if (t < 0) break;
                    tried.push_back(Pick{t, pk.c, cfg});
                    best_g = std::min(best_g, t);
                    if (t < pk.est) {
                        pk.est = t;
                        pk.launch = cfg;
                    }
                }
                if (st != GP_OK || best_g > 1.5 * pk.est) break;
            }
        }
        // 5. the finalists once more on a sample 4x denser; then, when the
        //    two best fit the budget, in full: estimates miss tails that the
        //    sample did not contain, a full run does not
        if (st == GP_OK && picks.size() > 1 && spent < 3.0 * budget_ms && stride >= 4) {
            best_est = inf;
            for (auto& pk : picks) {
                double t = measure(cands[pk.c].desc, pk.launch, std::max<int64_t>(1, stride / 4), "final", pk.c,
                                   true);
                if (t < 0) break;
                pk.est = t;
            }
        }
        // full runs of the best (configuration, shape) pairs while they fit
        // twice the budget, no pair twice
        std::stable_sort(picks.begin(), picks.end(), [](const Pick& a, const Pick& b) { return a.est < b.est; });
        std::stable_sort(tried.begin(), tried.end(), [](const Pick& a, const Pick& b) { return a.est < b.est; });
        // the best configuration at its best leaf mode for every group width
        // measured (sample estimates rank widths within their noise) and at its
        // best width for every leaf mode, then the runner-up configuration's
        // best pair
        std::vector<Pick> full;
        auto add_full = [&](const Pick& pk) {
            for (const Pick& f : full)
                if (f.c == pk.c && f.launch.group == pk.launch.group && f.launch.leaf == pk.launch.leaf) return;
            if (pk.est < inf) full.push_back(pk);
        };
        if (!picks.empty()) {
            add_full(picks[0]);
            for (int grp : {64, 32, 16, 8})
                for (const Pick& pk : tried)  // sorted: the first of a width is its best
                    if (pk.c == picks[0].c && pk.launch.group == grp) {
                        add_full(pk);
                        break;
                    }
            // and at its best width for every leaf mode measured (the samples
            // rank leaf modes within their noise as well)
            for (int lm : {1, 2, 3, 4})
                for (const Pick& pk : tried)
                    if (pk.c == picks[0].c && pk.launch.leaf == lm) {
                        add_full(pk);
                        break;
                    }
            for (const Pick& pk : picks)
                if (pk.c != picks[0].c) {
                    add_full(pk);
                    break;
                }
            // the other finalists, at their best measured shape or the default
            // one: sample estimates rank configurations only within their noise
            for (const auto& f : fine) {
                const Pick* bp = nullptr;
                for (const Pick& pk : tried)  // sorted: the first of a configuration is its best
                    if (pk.c == f.second) {
                        bp = &pk;
                        break;
                    }
                add_full(bp ? *bp : Pick{f.first, f.second, base});
            }
        }
        bool timed_full = stride == 1;  // picks hold full-run times
        if (st == GP_OK && stride > 1 && full.size() > 1) {
            std::stable_sort(full.begin(), full.end(), [](const Pick& a, const Pick& b) { return a.est < b.est; });
            double planned = 0;
            size_t n_full = 0;
            while (n_full < full.size() && planned + full[n_full].est < 2.0 * budget_ms) planned += full[n_full++].est;
            if (n_full > 1) {
                best_est = inf;
                for (size_t r = 0; r < n_full && st == GP_OK; ++r) {
                    double t = measure(cands[full[r].c].desc, full[r].launch, 1, "full", full[r].c);
                    if (t < 0) break;
                    full[r].est = t;
                }
                full.resize(n_full);
                picks = full;
                timed_full = true;
            }
        }
        // 5b. finalists too slow to time in full: the best one, the runner-up
        //     configuration (if within 2x) and the best one's other counting
        //     mode (plain vs inclusion-exclusion, same schedule and set) once
        //     more on a dense sample of about a quarter of the budget each.
        //     On skewed graphs a sparse sample holds few of the roots that
        //     carry the work and runs with less contention than a full run,
        //     and it misjudges configurations by different factors; IEP and
        //     plain counting differ most in how they treat those roots.
        if (st == GP_OK && !timed_full && stride > 1 && !picks.empty() && spent < 4.0 * budget_ms) {
            std::stable_sort(picks.begin(), picks.end(), [](const Pick& a, const Pick& b) { return a.est < b.est; });
            std::vector<Pick> dense;
            if (picks[0].est < inf) dense.push_back(picks[0]);
            for (const Pick& pk : picks)
                if (!dense.empty() && pk.c != dense[0].c && pk.est < 2.0 * dense[0].est) {
                    dense.push_back(pk);
                    break;
                }
            if (try_iep && !dense.empty()) {
                const Cfg& w = cands[dense[0].c];
                size_t other = cands.size();
                for (size_t c = 0; c < cands.size(); ++c)
                    if (cands[c].order == w.order && cands[c].rel == w.rel && (cands[c].desc.iep > 0) != (w.desc.iep > 0) &&
                        (other == cands.size() || cands[c].desc.iep > cands[other].desc.iep))
                        other = c;
                if (other < cands.size()) {
                    gpint::LaunchCfg cfg = dense[0].launch;
                    if (cands[other].desc.iep) {
                        cfg.group = cfg.group >= 64 ? 64 : 32;
                        cfg.leaf = 1;
                    }
                    dense.push_back(Pick{inf, other, cfg});
                }
            }
            const int64_t sd =
                dense.empty() ? 0 : std::max<int64_t>(1, (int64_t)std::ceil(dense[0].est / (0.25 * budget_ms)));
            if (dense.size() > 1 && sd < stride / 4) {
                best_est = inf;
                bool ok = true;
                for (Pick& pk : dense) {
                    const double t = measure(cands[pk.c].desc, pk.launch, sd, "dense", pk.c);
                    if (t < 0) {
                        ok = false;
                        break;
                    }
                    pk.est = t;
                }
                if (ok) picks = dense;
            }
        }
        size_t best = fine.empty() ? 0 : fine[0].second;
        gpint::LaunchCfg best_launch = base;
        double best_ms = inf;
        if (!picks.empty()) {
            const Pick* bp = &picks[0];
            for (auto& pk : picks)
                if (pk.est < bp->est) bp = &pk;
            best = bp->c;
            best_launch = bp->launch;
            best_ms = bp->est;
        }
        // 6. root splitting, then tasks per grab of the queue counter, in full
        //    runs of the winner, one change at a time. Splitting shortens the
        //    tail that single hub roots leave, but the split tasks of a root
        //    then run in different groups, which cannot share leaf mode 4's
        //    per-root memo. Single roots per grab shorten the tail of long
        //    patterns; longer grabs keep neighbouring roots (and the split
        //    tasks of one root) in one group. A change must win by 2% to count
        //    as more than noise.
        if (st == GP_OK && timed_full && k >= 4 && best_ms < inf && o.tune_launch >= 0) {
            auto try_cfg = [&](const gpint::LaunchCfg& cfg) {
                if (st != GP_OK || spent + best_ms > 4.0 * budget_ms) return;
                best_est = best_ms;  // a run past three times the winner stops
                const double t = measure(cands[best].desc, cfg, 1, "grab", best);
                if (t >= 0 && t < 0.98 * best_ms) {
                    best_ms = t;
                    best_launch = cfg;
                }
            };
            const gpint::LaunchCfg won = best_launch;
            for (int ways : {4, 1}) {
                if (ways == won.split_ways) continue;
                gpint::LaunchCfg cfg = best_launch;
                cfg.split_ways = ways;
                try_cfg(cfg);
            }
            const int chunk0 = best_launch.chunk;
            for (int ch : {2, 1, 8, 16}) {
                if (ch == chunk0) continue;
                gpint::LaunchCfg cfg = best_launch;
                cfg.chunk = ch;
                try_cfg(cfg);
            }
            // the heavy-root threshold T (roots whose hub endpoint is below it
            // are split), where roots are split at all
            if (best_launch.split_ways > 1) {
                const int64_t t0v = best_launch.split_vertices;
                for (int64_t tv : {64, 1024, 4096}) {
                    if (tv == t0v) continue;
                    gpint::LaunchCfg cfg = best_launch;
                    cfg.split_vertices = tv;
                    try_cfg(cfg);
                }
            }
            // fewer resident wavefronts per compute unit: less contention for
            // the caches on graphs larger than them
            const int w0 = best_launch.waves_per_cu;
            for (int w : {16, 24}) {
                if (w >= w0) continue;
                gpint::LaunchCfg cfg = best_launch;
                cfg.waves_per_cu = w;
                try_cfg(cfg);
            }
        }
        best_launch.root_stride = 1;
        best_launch.root_offset = 0;
        best_launch.budget_ms = 0;
        if (st == GP_OK) {
            np->order = cands[best].order;
            np->set = cands[best].rel;
            np->desc = cands[best].desc;
            np->launch = best_launch;
            np->tuned = true;
            np->tuned_ms = best_ms < inf ? best_ms : 0;
            np->info.n_measured = measured;
            std::lock_guard<std::mutex> lk(g_cache_mu);
            g_cache[key] = Cached{np->order, np->set, np->desc, np->launch, measured, np->tuned_ms};
        }
        (void)hipFreeAsync(res, s);
        (void)hipStreamSynchronize(s);
    }
    if (prev_dev >= 0 && prev_dev != g->dg.device) (void)hipSetDevice(prev_dev);
    if (st != GP_OK) {
        delete np;
        return st;
    }
    // refresh the reported configuration
    gp_plan_info& in = np->info;
    for (int i = 0; i < k; ++i) in.order[i] = np->order[i];
    int nr = 0;
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b)
            if (gp::rel_has(np->set, a, b)) {
                in.restr[2 * nr] = a;
                in.restr[2 * nr + 1] = b;
                ++nr;
            }
    in.n_restr = nr;
    in.set_index = -1;
    for (size_t j = 0; j < np->sets.size(); ++j)
        if (np->sets[j] == np->set) in.set_index = (int32_t)j;
    gp::GraphStats gs{double(std::max<int64_t>(1, g->dg.stats.n)),
                      double(std::max<int64_t>(1, g->dg.stats.m)), double(g->dg.stats.tri_cnt)};
    in.cost = gp::model_cost(np->pattern, np->order, np->set, gs);
    in.tuned = 1;
    in.iep = np->desc.iep;
    in.iep_div = np->desc.iep_div;
    in.tuned_ms = np->tuned_ms;
    in.plan_seconds = p->info.plan_seconds + (now_seconds() - t0);
    *out = np;
    return GP_OK;
}

gp_status gp_estimate(const gp_graph* g, const gp_plan* p, const gp_launch* launch, double budget_ms,
                      void* stream, double* est_ms, uint64_t* sample_count, int64_t* sample_stride) {
    if (!g || !p || !est_ms || budget_ms < 0) return GP_ERR_ARG;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != g->dg.device) (void)hipSetDevice(g->dg.device);
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* res = nullptr;
    gp_status st = GP_OK;
    if (hipMallocAsync((void**)&res, 5 * sizeof(unsigned long long), s) != hipSuccess) {
        st = GP_ERR_NOMEM;
    } else {
        gpint::LaunchCfg cfg = gpint::launch_for_plan(p, launch, g->dg);
        cfg.root_stride = 1;
        cfg.root_offset = 0;
        const double e = gpint::estimate_full_ms(g->dg, p->desc, cfg, budget_ms, s, res, sample_count,
                                                 sample_stride);
        if (e < 0) st = GP_ERR_HIP;
        else *est_ms = e;
        (void)hipFreeAsync(res, s);
        (void)hipStreamSynchronize(s);
    }
    if (prev >= 0 && prev != g->dg.device) (void)hipSetDevice(prev);
    return st;
}

}  // extern "C"
