// Host-side configuration generation and selection (GraphPi Sections IV-A..C).
#pragma once
#include <array>
#include <cstdint>
#include <vector>

#include "plan_desc.h"

namespace gp {

constexpr int kMaxK = GP_DESC_MAX_K;

// Relation over pattern vertices as an 8x8 bit matrix: bit (a*8+b) set means
// the restriction id(a) > id(b).
using Rel = uint64_t;
inline Rel rel_bit(int a, int b) { return Rel(1) << (a * 8 + b); }
inline bool rel_has(Rel r, int a, int b) { return (r >> (a * 8 + b)) & 1; }

using Perm = std::array<uint8_t, kMaxK>;

struct Pattern {
    int k = 0;
    uint8_t adj[kMaxK] = {0};                 // adjacency bitmask per vertex
    std::vector<std::pair<int, int>> edges;
};

// Returns 0 or GP_ERR_PATTERN.
int parse_pattern(const int32_t* edges, int k, int e, Pattern* out);

std::vector<Perm> automorphisms(const Pattern& p);

Rel closure(Rel r, int k);
bool acyclic(Rel r, int k);
bool no_conflict(const Perm& perm, Rel r, int k);
// Number of rank vectors r (permutations of 0..k-1) with r[a] > r[b] for all pairs.
uint64_t linear_extensions(Rel r, int k);
bool validate(Rel r, int k, uint64_t aut);

struct RestrictionSets {
    std::vector<Rel> sets;   // distinct valid closures, emission order
    int64_t states = 0;      // distinct closures visited
    bool truncated = false;
};
// max_seconds > 0: stop exploring once that long has passed and a valid set
// exists (the output is then a prefix of the full emission order).
RestrictionSets restriction_sets(const Pattern& p, const std::vector<Perm>& auts,
                                 int64_t max_states, int32_t max_sets, double max_seconds = 0);

// Lexicographically smallest schedule of each orbit under the automorphisms.
std::vector<Perm> orbit_representatives(const std::vector<Perm>& orders, const std::vector<Perm>& auts,
                                        int k);

struct Schedules {
    std::vector<Perm> orders;  // lexicographic order
    int k_eff = 0;
};
bool phase1_ok(const Pattern& p, const Perm& order);
Schedules efficient_schedules(const Pattern& p);

struct GraphStats {
    double n_v, n_e, tri_cnt;
};
double model_cost(const Pattern& p, const Perm& order, Rel r, const GraphStats& s);
// Number of restriction pairs that cut a later vertex from above.
int upper_cuts(const Perm& order, Rel r, int k);

// Compile (schedule, closure) into the kernel descriptor. Returns 0 or an error.
// With iep_div > 0 the last iep_n levels (pairwise non-adjacent) are compiled
// for counting with inclusion-exclusion: their bounds come from iep_kept (the
// restrictions that remain), they are neither bound sources nor injectivity
// partners of each other, and iep_div is the over-count.
int compile_plan(const Pattern& p, const Perm& order, Rel r, GpPlanDesc* out, Rel iep_kept = 0,
                 int iep_div = 0, int iep_n = 0);

// The most innermost levels of `order` that IEP may count: the longest run
// of pairwise non-adjacent pattern vertices at the end of the schedule, at
// most GP_IEP_MAX_INNER and at most k - 2 (the root edge is enumerated); 0
// if fewer than 2.
int iep_max_inner(const Pattern& p, const Perm& order);

// IEP over the last n_in levels of (order, r): the restrictions that remain
// and the exact over-count (how many relative orders of each Aut-orbit obey
// them; it must be the same for every orbit). First try dropping only the
// restrictions between two inner levels, then every restriction checked in
// the inner levels. Returns the over-count (and *kept), or 0 when the
// configuration cannot be counted with IEP over n_in levels.
int iep_setup(const Pattern& p, const std::vector<Perm>& auts, const Perm& order, Rel r, int n_in, Rel* kept);

}  // namespace gp
