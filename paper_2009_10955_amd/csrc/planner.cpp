// Host-side configuration generation and selection.
//
//   automorphisms        Section IV-A (all permutations preserving the edge set)
//   restriction_sets     Section IV-A, Algorithm 1 (2-cycle based automorphism
//                        elimination: sets grown by 2-cycle pairs, no_conflict,
//                        validate)
//   efficient_schedules  Section IV-B (Phase 1: prefix-connected orders;
//                        Phase 2: last k searched vertices pairwise non-adjacent)
//   model_cost           Section IV-C (nested cost model with the cardinality
//                        estimates p1, p2 and the filter fractions f_i)
//   compile_plan         lowers (schedule, restriction closure) to GpPlanDesc
//
// Readings where the paper is silent or garbled:
//   * 2-cycle test: perm[perm[v]] == v and perm[v] != v; the pair added is
//     (v, perm[v]), meaning id(v) > id(perm[v]).
//   * each restriction set is explored once per transitive closure (sound:
//     conflicts and the validate count depend only on the closure); results
//     are closures, sorted by size, then by their sorted pairs.
//   * validate uses the closed form of the paper's K_k check: on the complete
//     graph K_k every bijection is a map, so the restricted count is the
//     number of rank vectors obeying the set; valid iff that times |Aut| = k!.
//   * Phase 2 with no satisfying order: the largest k' <= alpha(P) that some
//     Phase-1 order admits.
//   * Model: tri_cnt counts ordered triangles; a restriction is charged to the
//     loop of its later-bound vertex; an intersection is charged to the loop of
//     its last-bound parent, starting from the largest earlier candidate set
//     with a subset of its parents bound no later, else the first parent's
//     neighborhood, then the remaining parents in schedule order.
#include "planner.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <unordered_map>
#include <unordered_set>

#include "gp.h"

namespace gp {

int parse_pattern(const int32_t* edges, int k, int e, Pattern* out) {
    if (k < 2 || k > kMaxK || e < 1 || e > k * (k - 1) / 2 || !edges) return GP_ERR_PATTERN;
    Pattern p;
    p.k = k;
    for (int i = 0; i < e; ++i) {
        int a = edges[2 * i], b = edges[2 * i + 1];
        if (a < 0 || a >= k || b < 0 || b >= k || a == b) return GP_ERR_PATTERN;
        if (p.adj[a] & (1u << b)) return GP_ERR_PATTERN;  // repeated edge
        p.adj[a] |= uint8_t(1u << b);
        p.adj[b] |= uint8_t(1u << a);
        p.edges.emplace_back(a, b);
    }
    // connected?
    unsigned seen = 1, frontier = 1;
    while (frontier) {
        unsigned next = 0;
        for (int v = 0; v < k; ++v)
            if (frontier & (1u << v)) next |= p.adj[v];
        next &= ~seen;
        seen |= next;
        frontier = next;
    }
    if (seen != (1u << k) - 1) return GP_ERR_PATTERN;
    *out = p;
    return 0;
}

std::vector<Perm> automorphisms(const Pattern& p) {
    std::vector<Perm> out;
    Perm perm{};
    for (int i = 0; i < p.k; ++i) perm[i] = uint8_t(i);
    do {
        bool ok = true;
        for (auto& e : p.edges)
            if (!(p.adj[perm[e.first]] & (1u << perm[e.second]))) { ok = false; break; }
        if (ok) out.push_back(perm);
    } while (std::next_permutation(perm.begin(), perm.begin() + p.k));
    return out;
}

Rel closure(Rel r, int k) {
    uint8_t row[kMaxK];
    for (int a = 0; a < k; ++a) row[a] = uint8_t(r >> (a * 8));
    for (int m = 0; m < k; ++m)
        for (int a = 0; a < k; ++a)
            if (row[a] & (1u << m)) row[a] |= row[m];
    Rel out = 0;
    for (int a = 0; a < k; ++a) out |= Rel(row[a]) << (a * 8);
    return out;
}

bool acyclic(Rel r, int k) {
    Rel c = closure(r, k);
    for (int a = 0; a < k; ++a)
        if (rel_has(c, a, a)) return false;
    return true;
}

// Algorithm 1, no_conflict: the digraph with every restriction (a,b) and its
// image (perm[a], perm[b]); perm survives iff the digraph is acyclic.
bool no_conflict(const Perm& perm, Rel r, int k) {
    Rel g = r;
    Rel rest = r;
    while (rest) {
        int bit = __builtin_ctzll(rest);
        rest &= rest - 1;
        int a = bit >> 3, b = bit & 7;
        g |= rel_bit(perm[a], perm[b]);
    }
    return acyclic(g, k);
}

uint64_t linear_extensions(Rel r, int k) {
    // below[x] = elements that must rank lower than x (pairs (x, b)).
    uint8_t below[kMaxK];
    for (int x = 0; x < k; ++x) below[x] = uint8_t(r >> (x * 8));
    // Place elements from the lowest rank upward; x may take the next rank
    // once everything that must be below it is placed.
    uint64_t dp[1 << kMaxK];
    const int full = (1 << k) - 1;
    std::fill(dp, dp + (full + 1), 0);
    dp[0] = 1;
    for (int s = 0; s < full; ++s) {
        if (!dp[s]) continue;
        for (int x = 0; x < k; ++x) {
            if (s & (1 << x)) continue;
            if ((below[x] & ~s) != 0) continue;
            dp[s | (1 << x)] += dp[s];
        }
    }
    return dp[full];
}

static uint64_t factorial(int k) {
    uint64_t f = 1;
    for (int i = 2; i <= k; ++i) f *= uint64_t(i);
    return f;
}

bool validate(Rel r, int k, uint64_t aut) {
    return linear_extensions(r, k) * aut == factorial(k);
}

namespace {
double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Lexicographic order of the sorted (a, b) pair lists of two relations.
bool pairs_less(Rel x, Rel y) {
    while (x && y) {
        const int bx = __builtin_ctzll(x), by = __builtin_ctzll(y);  // bit a*8+b: ascending (a, b)
        if (bx != by) return bx < by;
        x &= x - 1;
        y &= y - 1;
    }
    return !x && y;
}

// The valid closures first by size, then by their sorted pairs.
void sort_sets(std::vector<Rel>* sets) {
    std::sort(sets->begin(), sets->end(), [](Rel a, Rel b) {
        const int na = __builtin_popcountll(a), nb = __builtin_popcountll(b);
        if (na != nb) return na < nb;
        return pairs_less(a, b);
    });
}
}  // namespace

RestrictionSets restriction_sets(const Pattern& p, const std::vector<Perm>& auts,
                                 int64_t max_states, int32_t max_sets, double max_seconds) {
    const int k = p.k;
    // Complete pattern, k >= 6: every valid set is a total order (one orbit,
    // one obeying order per orbit) and Algorithm 1 reaches all k! of them, so
    // emit them directly (then sorted like every other result).
    bool complete = true;
    for (int v = 0; v < k; ++v)
        if (__builtin_popcount(p.adj[v]) != k - 1) complete = false;
    if (complete && k >= 6) {
        RestrictionSets out;
        Perm rank{};
        for (int i = 0; i < k; ++i) rank[i] = uint8_t(i);
        do {
            if ((int32_t)out.sets.size() >= max_sets) {
                out.truncated = true;
                break;
            }
            Rel r = 0;  // id(rank[0]) > id(rank[1]) > ...
            for (int i = 0; i < k; ++i)
                for (int j = i + 1; j < k; ++j) r |= rel_bit(rank[i], rank[j]);
            out.sets.push_back(r);
        } while (std::next_permutation(rank.begin(), rank.begin() + k));
        sort_sets(&out.sets);
        out.states = (int64_t)out.sets.size();
        return out;
    }
    // Worklist over closures: a closure grows by one pair (v, perm[v]) per
    // automorphism perm it does not yet eliminate and vertex v on a 2-cycle
    // of perm; a closure at which the identity alone survives is kept if
    // valid. A grown closure's survivors are its parent's survivors that do
    // not conflict with it (a conflict persists in every superset, so this
    // equals filtering all automorphisms).
    RestrictionSets out;
    const double deadline = max_seconds > 0 ? now_s() + max_seconds : 0;
    std::unordered_set<Rel> seen;
    std::unordered_set<Rel> valid;
    struct Item {
        Rel rel;
        std::vector<int> alive;
    };
    std::vector<Item> work;
    Item start;
    start.rel = 0;
    for (size_t i = 0; i < auts.size(); ++i) start.alive.push_back(int(i));
    seen.insert(0);
    work.push_back(std::move(start));
    while (!work.empty()) {
        if ((int32_t)valid.size() >= max_sets ||
            (deadline > 0 && (seen.size() & 1023) == 0 && now_s() > deadline && !valid.empty())) {
            out.truncated = true;
            break;
        }
        Item it = std::move(work.back());
        work.pop_back();
        if (it.alive.size() <= 1) {
            // the identity alone survives (or nothing: a cyclic set)
            if (!it.alive.empty() && validate(it.rel, k, auts.size())) valid.insert(it.rel);
            continue;
        }
        for (int pi : it.alive) {
            const Perm& perm = auts[pi];
            for (int v = 0; v < k; ++v) {
                if (perm[v] == v || perm[perm[v]] != v) continue;  // v is not on a 2-cycle
                const Rel grown = closure(it.rel | rel_bit(v, perm[v]), k);
                if (seen.count(grown)) continue;
                if ((int64_t)seen.size() >= max_states) {
                    out.truncated = true;
                    continue;
                }
                seen.insert(grown);
                Item next;
                next.rel = grown;
                for (int qi : it.alive)
                    if (no_conflict(auts[qi], grown, k)) next.alive.push_back(qi);
                work.push_back(std::move(next));
            }
        }
    }
    out.sets.assign(valid.begin(), valid.end());
    sort_sets(&out.sets);
    out.states = int64_t(seen.size());
    return out;
}

bool phase1_ok(const Pattern& p, const Perm& order) {
    unsigned placed = 1u << order[0];
    for (int i = 1; i < p.k; ++i) {
        if (!(p.adj[order[i]] & placed)) return false;
        placed |= 1u << order[i];
    }
    return true;
}

static int independence_number(const Pattern& p) {
    int best = 0;
    for (unsigned s = 1; s < (1u << p.k); ++s) {
        bool ok = true;
        for (int v = 0; v < p.k && ok; ++v)
            if ((s & (1u << v)) && (p.adj[v] & s)) ok = false;
        if (ok) best = std::max(best, __builtin_popcount(s));
    }
    return best;
}

Schedules efficient_schedules(const Pattern& p) {
    const int k = p.k;
    std::vector<Perm> p1;
    Perm perm{};
    for (int i = 0; i < k; ++i) perm[i] = uint8_t(i);
    do {
        if (phase1_ok(p, perm)) p1.push_back(perm);
    } while (std::next_permutation(perm.begin(), perm.begin() + k));
    Schedules out;
    int alpha = independence_number(p);
    for (int keff = alpha; keff >= 1; --keff) {
        for (auto& o : p1) {
            bool ok = true;
            for (int a = k - keff; a < k && ok; ++a)
                for (int b = a + 1; b < k && ok; ++b)
                    if (p.adj[o[a]] & (1u << o[b])) ok = false;
            if (ok) out.orders.push_back(o);
        }
        if (!out.orders.empty()) {
            out.k_eff = keff;
            return out;
        }
    }
    out.orders = p1;
    out.k_eff = 0;
    return out;
}

std::vector<Perm> orbit_representatives(const std::vector<Perm>& orders, const std::vector<Perm>& auts,
                                        int k) {
    // (order, R) and (pi o order, pi(R)) compile to the same search for every
    // automorphism pi; keep the lexicographically smallest schedule per orbit.
    std::vector<Perm> reps;
    for (const Perm& o : orders) {
        bool smallest = true;
        for (const Perm& pi : auts) {
            Perm img{};
            for (int i = 0; i < k; ++i) img[i] = pi[o[i]];
            if (std::lexicographical_compare(img.begin(), img.begin() + k, o.begin(), o.begin() + k)) {
                smallest = false;
                break;
            }
        }
        if (smallest) reps.push_back(o);
    }
    return reps;
}

double model_cost(const Pattern& p, const Perm& order, Rel r, const GraphStats& s) {
    const int k = p.k;
    int pos[kMaxK];
    for (int i = 0; i < k; ++i) pos[order[i]] = i;
    const double p1 = 2.0 * s.n_e / (s.n_v * s.n_v);
    const double p2 = s.tri_cnt * s.n_v / std::pow(2.0 * s.n_e, 2.0);
    auto card = [&](int nsets) { return s.n_v * p1 * std::pow(p2, double(nsets - 1)); };

    // parents as level lists (ascending)
    int npar[kMaxK];
    unsigned parmask[kMaxK];
    for (int i = 0; i < k; ++i) {
        parmask[i] = 0;
        for (int j = 0; j < i; ++j)
            if (p.adj[order[i]] & (1u << order[j])) parmask[i] |= 1u << j;
        npar[i] = __builtin_popcount(parmask[i]);
    }

    // f_i: survivors among the k! relative magnitudes, filtered loop by loop.
    double f[kMaxK] = {0};
    Rel upto = 0;
    uint64_t before = factorial(k);
    for (int i = 0; i < k; ++i) {
        Rel here = 0;
        Rel rest = r;
        while (rest) {
            int bit = __builtin_ctzll(rest);
            rest &= rest - 1;
            int a = bit >> 3, b = bit & 7;
            if (std::max(pos[a], pos[b]) == i) here |= rel_bit(a, b);
        }
        if (!here) continue;
        upto |= here;
        uint64_t after = linear_extensions(upto, k);
        f[i] = before ? double(before - after) / double(before) : 0.0;
        before = after;
    }

    double loop[kMaxK];
    loop[0] = s.n_v;
    for (int i = 1; i < k; ++i) loop[i] = card(npar[i]);

    double c[kMaxK] = {0};
    int built[kMaxK];
    int nbuilt = 0;
    for (int i = 0; i < k; ++i) {
        if (npar[i] < 2) continue;
        int h = 31 - __builtin_clz(parmask[i]);
        int base = -1;
        for (int t = 0; t < nbuilt; ++t) {
            int m = built[t];
            unsigned pm = parmask[m];
            int hm = 31 - __builtin_clz(pm);
            bool subset = (pm & ~parmask[i]) == 0 && pm != parmask[i];
            if (hm <= h && subset) {
                if (base < 0 || npar[m] > npar[base]) base = m;
            }
        }
        int have, nrest;
        if (base < 0) {
            have = 1;
            nrest = npar[i] - 1;
        } else {
            have = npar[base];
            nrest = npar[i] - npar[base];
        }
        for (int t = 0; t < nrest; ++t) {
            c[h] += card(have) + card(1);
            ++have;
        }
        built[nbuilt++] = i;
    }

    double cost = loop[k - 1] * (1.0 - f[k - 1]);
    for (int i = k - 2; i >= 0; --i) cost = loop[i] * (1.0 - f[i]) * (c[i] + cost);
    return cost;
}

int upper_cuts(const Perm& order, Rel r, int k) {
    int pos[kMaxK];
    for (int i = 0; i < k; ++i) pos[order[i]] = i;
    int n = 0;
    Rel rest = r;
    while (rest) {
        int bit = __builtin_ctzll(rest);
        rest &= rest - 1;
        int a = bit >> 3, b = bit & 7;
        if (pos[a] < pos[b]) ++n;  // b searched later and bounded above by a
    }
    return n;
}

// How many relative orders of each Aut-orbit obey `kept`, if the same for
// every orbit; else 0.
static int orbit_multiplicity(const std::vector<Perm>& auts, Rel kept, int k) {
    // pairs of kept as (a, b) lists
    int pa[64], pb[64], np = 0;
    Rel rest = kept;
    while (rest) {
        int bit = __builtin_ctzll(rest);
        rest &= rest - 1;
        pa[np] = bit >> 3;
        pb[np] = bit & 7;
        ++np;
    }
    Perm r{};
    for (int i = 0; i < k; ++i) r[i] = uint8_t(i);
    int mult = -1;
    do {
        int c = 0;
        for (const Perm& q : auts) {
            // member r o q: rank of vertex v is r[q[v]]
            bool ok = true;
            for (int t = 0; t < np && ok; ++t) ok = r[q[pa[t]]] > r[q[pb[t]]];
            c += ok;
        }
        if (mult < 0) mult = c;
        else if (c != mult) return 0;
    } while (std::next_permutation(r.begin(), r.begin() + k));
    return mult < 0 ? 0 : mult;
}

int iep_max_inner(const Pattern& p, const Perm& order) {
    const int k = p.k;
    // inner levels come after the root edge (levels 0 and 1)
    const int cap = std::min(GP_IEP_MAX_INNER, k - 2);
    int n = 0;
    unsigned inner = 0;
    while (n < cap) {
        const int u = order[k - 1 - n];
        if (p.adj[u] & inner) break;
        inner |= 1u << u;
        ++n;
    }
    return n >= 2 ? n : 0;
}

int iep_setup(const Pattern& p, const std::vector<Perm>& auts, const Perm& order, Rel r, int n_in, Rel* kept) {
    const int k = p.k;
    if (n_in < 2 || n_in > iep_max_inner(p, order)) return 0;
    unsigned inner = 0;
    for (int i = k - n_in; i < k; ++i) inner |= 1u << order[i];
    // 1) drop only the restrictions between two inner levels
    Rel k1 = 0, k2 = 0;
    Rel rest = r;
    while (rest) {
        int bit = __builtin_ctzll(rest);
        rest &= rest - 1;
        const int u = bit >> 3, w = bit & 7;
        const bool iu = (inner >> u) & 1u, iw = (inner >> w) & 1u;
        if (!(iu && iw)) k1 |= rel_bit(u, w);
        if (!iu && !iw) k2 |= rel_bit(u, w);
    }
    int m = orbit_multiplicity(auts, k1, k);
    if (m > 0) {
        *kept = k1;
        return m;
    }
    // 2) drop every restriction checked in the inner levels
    m = orbit_multiplicity(auts, k2, k);
    if (m > 0) {
        *kept = k2;
        return m;
    }
    return 0;
}

int compile_plan(const Pattern& p, const Perm& order, Rel r, GpPlanDesc* out, Rel iep_kept, int iep_div,
                 int iep_n) {
    const int k = p.k;
    if (!phase1_ok(p, order)) return GP_ERR_ARG;
    const bool iep = iep_div > 0;
    if (iep && (iep_n < 2 || iep_n > iep_max_inner(p, order))) return GP_ERR_ARG;
    const int first_inner = iep ? k - iep_n : k;
    const unsigned inner_mask = iep ? ((1u << k) - 1) & ~((1u << first_inner) - 1) : 0u;
    GpPlanDesc d;
    std::memset(&d, 0, sizeof d);
    d.k = k;
    int pos[kMaxK];
    for (int i = 0; i < k; ++i) pos[order[i]] = i;

    unsigned par[kMaxK], hi[kMaxK], lo[kMaxK];
    for (int i = 0; i < k; ++i) {
        par[i] = hi[i] = lo[i] = 0;
        int u = order[i];
        // the inner IEP levels are bounded only by the restrictions that remain
        const Rel rr = i >= first_inner ? iep_kept : r;
        for (int j = 0; j < i; ++j) {
            int w = order[j];
            if (p.adj[u] & (1u << w)) par[i] |= 1u << j;
            if (rel_has(rr, w, u)) hi[i] |= 1u << j;  // id(w) > id(u): v_i < v_j
            if (rel_has(rr, u, w)) lo[i] |= 1u << j;  // id(u) > id(w): v_i > v_j
        }
        if (i >= first_inner) {
            // the other inner levels are never bound: not bound sources
            hi[i] &= ~inner_mask;
            lo[i] &= ~inner_mask;
        }
    }
    d.root_cut = (hi[1] & 1u) ? 1 : ((lo[1] & 1u) ? 2 : 0);

    struct Key {
        unsigned q, h, l;
        bool operator==(const Key& o) const { return q == o.q && h == o.h && l == o.l; }
    };
    std::vector<std::pair<Key, int>> slots;
    std::vector<GpBuild> builds;

    // Chain of two-operand steps over the given parent levels (ascending);
    // returns the slot holding the full intersection.
    auto ensure_chain = [&](unsigned pmask, int target) -> int {
        int lv[kMaxK], n = 0;
        for (int j = 0; j < k; ++j)
            if (pmask & (1u << j)) lv[n++] = j;
        unsigned prefix = 1u << lv[0];
        int slot = -1;
        for (int s = 1; s < n; ++s) {
            int h = lv[s];
            prefix |= 1u << h;
            unsigned lim = (2u << h) - 1;
            Key key{prefix, hi[target] & lim, lo[target] & lim};
            int found = -1;
            for (auto& kv : slots)
                if (kv.first == key) { found = kv.second; break; }
            if (found >= 0) { slot = found; continue; }
            GpBuild b;
            b.h = int8_t(h);
            b.dst = int8_t(slots.size());
            b.src_buf = int8_t(slot);
            b.src_list = int8_t(slot < 0 ? lv[0] : -1);
            b.with_list = int8_t(h);
            b.hi_src = uint8_t(key.h);
            b.lo_src = uint8_t(key.l);
            b.pad = 0;
            slots.push_back({key, int(b.dst)});
            builds.push_back(b);
            slot = b.dst;
        }
        return slot;
    };

    for (int i = 0; i < k; ++i) {
        GpLevel& L = d.lv[i];
        L.parents = uint8_t(par[i]);
        L.hi_src = uint8_t(hi[i]);
        L.lo_src = uint8_t(lo[i]);
        L.inj = uint8_t(((1u << i) - 1) & ~par[i] & ~hi[i] & ~lo[i]);
        if (i >= first_inner) L.inj &= uint8_t(~inner_mask);  // distinct inner images: the IEP sum
        L.list = L.buf = L.pre_buf = L.pre_list = L.last_list = -1;
        if (i == 0) continue;
        int np = __builtin_popcount(par[i]);
        int h = 31 - __builtin_clz(par[i]);
        if (np == 1) {
            L.list = int8_t(h);
        } else if (i >= first_inner && h == first_inner - 1) {
            // an IEP inner set whose last parent is the last outer level: left
            // unbuilt as pre & N(v_h), counted where it is used
            unsigned prefix = par[i] & ~(1u << h);
            if (__builtin_popcount(prefix) == 1) {
                L.pre_list = int8_t(__builtin_ctz(prefix));
            } else {
                L.pre_buf = int8_t(ensure_chain(prefix, i));
            }
            L.last_list = int8_t(h);
        } else if (i < k - 1 || h < k - 2) {
            L.buf = int8_t(ensure_chain(par[i], i));
        } else {
            // last level whose last parent is level k-2: count-only final step
            unsigned prefix = par[i] & ~(1u << h);
            if (__builtin_popcount(prefix) == 1) {
                L.pre_list = int8_t(__builtin_ctz(prefix));
            } else {
                L.pre_buf = int8_t(ensure_chain(prefix, i));
            }
            L.last_list = int8_t(h);
        }
    }
    if (builds.size() > GP_DESC_MAX_BUILDS) return GP_ERR_UNSUPPORTED;
    std::stable_sort(builds.begin(), builds.end(),
                     [](const GpBuild& a, const GpBuild& b) { return a.h < b.h; });
    d.nbuild = int32_t(builds.size());
    d.nbuf = int32_t(slots.size());
    for (size_t t = 0; t < builds.size(); ++t) d.b[t] = builds[t];
    for (int h = 0; h < k; ++h) {
        int b0 = 0;
        while (b0 < d.nbuild && d.b[b0].h < h) ++b0;
        int b1 = b0;
        while (b1 < d.nbuild && d.b[b1].h == h) ++b1;
        d.build_begin[h] = uint8_t(b0);
        d.build_end[h] = uint8_t(b1);
    }
    d.iep = iep ? iep_n : 0;
    d.iep_div = iep ? iep_div : 0;
    *out = d;
    return 0;
}

}  // namespace gp
