// Device-ready plan descriptor: the compiled form of one configuration
// (schedule + restriction set) that the counting kernel interprets.
//
// Levels are schedule positions: level i binds the data vertex v_i that the
// i-th searched pattern vertex maps to (Section II-B: a schedule is the order
// in which pattern vertices are searched). Levels 0 and 1 come from one root
// edge (v0, v1); the last level is never enumerated, only counted.
//
// A candidate set is either one neighbor list N(v_p) (single parent) or an
// intersection of the parents' neighbor lists (Section IV-B). Intersections
// are built as a chain of two-operand steps in ascending parent level; each
// step runs right after its last operand is bound (the hoisting that puts
// intersections in outer loops, Section IV-B Phase 2 and the tmp sets of the
// generated code) and writes a buffer slot that later steps and levels read.
//
// Restrictions (id(a) > id(b), Section II-B) become bounds on v_i: hi_src
// lists levels j with v_i < v_j, lo_src levels j with v_i > v_j. The kernel
// applies them as binary-search cuts on sorted sets (the paper's `break`).
// With IEP, restrictions between two inner levels are dropped (and, when
// needed, every restriction checked in them), so those levels' bounds come
// from the restrictions that remain.
#pragma once
#include <stdint.h>

#define GP_DESC_MAX_K 8
#define GP_DESC_MAX_BUILDS 24
// inclusion-exclusion over at most this many innermost levels
#define GP_IEP_MAX_INNER 4

struct GpBuild {
    int8_t h;          // runs right after level h is bound
    int8_t dst;        // buffer slot written
    int8_t src_buf;    // base operand: buffer slot, or -1 for N(v[src_list])
    int8_t src_list;
    int8_t with_list;  // second operand: N(v[with_list])
    uint8_t hi_src;    // result cut to values < v_j for j in mask (all j <= h)
    uint8_t lo_src;    // result cut to values > v_j
    int8_t pad;
};

struct GpLevel {
    uint8_t parents;   // levels adjacent in the pattern (bitmask)
    uint8_t hi_src;    // v_i < v_j for j in mask
    uint8_t lo_src;    // v_i > v_j for j in mask
    uint8_t inj;       // earlier levels v_i must differ from explicitly
    int8_t list;       // single parent: level whose neighbor list is the candidate set
    int8_t buf;        // several parents, fully built before level i: buffer slot
    // the last level when its last parent is the level just before it, or an
    // IEP inner level whose last parent is the last outer level: the set
    // pre & N(v[last_list]) & cuts is counted where it is used, never built.
    int8_t pre_buf;    // prefix operand: buffer slot, or -1 for N(v[pre_list])
    int8_t pre_list;
    int8_t last_list;  // -1 when the last level reads `list` or `buf`
    int8_t pad[3];
};

struct GpPlanDesc {
    int32_t k;
    int32_t root_cut;  // 0: every directed edge, 1: only v1 < v0, 2: only v1 > v0
    int32_t nbuild;
    int32_t nbuf;
    // Counting with inclusion-exclusion (Section IV-D): iep > 0 is the number
    // of innermost levels (2 .. GP_IEP_MAX_INNER, pairwise non-adjacent) that
    // are not enumerated; for each binding of the outer levels the kernel adds
    // the number of tuples of distinct elements of their candidate sets, and
    // the total is divided by iep_div, the number of times IEP counts every
    // embedding.
    int32_t iep;
    int32_t iep_div;
    GpLevel lv[GP_DESC_MAX_K];
    GpBuild b[GP_DESC_MAX_BUILDS];
    uint8_t build_begin[GP_DESC_MAX_K];  // builds with h == level are b[begin, end)
    uint8_t build_end[GP_DESC_MAX_K];
};
