/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct counting of pattern embeddings, written from
 * the problem definition (Section II-A): an embedding is a bijection id from
 * the pattern's vertices onto a subgraph of the data graph such that every
 * pattern edge (u_i, u_j) maps onto a data-graph edge. The number of distinct
 * subgraphs equals the number of injective edge-preserving maps divided by the
 * number of automorphisms of the pattern (Section II-B: automorphic maps give
 * the same subgraph). This file counts MAPS; the division is done by the
 * caller (oracle/__init__.py), which also computes the automorphisms.
 *
 * Optional extras, each still a plain definition:
 *   - restriction pairs (a, b): keep only maps with id(a) > id(b)
 *     (Section II-B, "restriction");
 *   - pinned vertices: fix id(u) = x for given pattern vertices, so that a
 *     count can be split into independently checkable parts.
 *
 * Method: backtracking over pattern vertices, the most-constrained vertex
 * (most already-placed pattern neighbors) first. A candidate for a vertex is
 * any neighbor of the image of one earlier pattern neighbor -- the one with
 * the shortest list -- or any data vertex if it has none. Every candidate is checked against every
 * pattern edge to an earlier vertex (binary search in the sorted adjacency
 * list), against injectivity, and against every restriction pair. There are
 * no set intersections, no schedules and no restriction-derived bounds here.
 * Counts accumulate in unsigned 128-bit integers.
 *
 * Shares no code with the GPU library. Only tests/, the smoke check and the
 * benchmark's CPU-baseline leg may load it.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_K 12

typedef unsigned __int128 u128;

typedef struct {
    const int64_t *row_ptr;
    const int32_t *col;
    int32_t n;
    int32_t k;
    int32_t order[ORACLE_MAX_K];     /* pattern vertex searched at position t */
    int32_t anchor[ORACLE_MAX_K];    /* earlier position whose image's neighbors are scanned; -1: all */
    int32_t nback[ORACLE_MAX_K];     /* earlier positions adjacent in the pattern */
    int32_t back[ORACLE_MAX_K][ORACLE_MAX_K];
    int32_t ngt[ORACLE_MAX_K];       /* earlier positions s with required img[s] > img[t] */
    int32_t gt[ORACLE_MAX_K][ORACLE_MAX_K];
    int32_t nlt[ORACLE_MAX_K];       /* earlier positions s with required img[s] < img[t] */
    int32_t lt[ORACLE_MAX_K][ORACLE_MAX_K];
    int32_t npin;                    /* positions 0..npin-1 are pinned */
    int32_t pin_value[ORACLE_MAX_K];
    /* work distribution over the first position's candidates */
    int64_t next_first;
    int64_t first_count;
} job_t;

static int adjacent(const job_t *J, int32_t a, int32_t b) {
    int64_t lo = J->row_ptr[a], hi = J->row_ptr[a + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int32_t v = J->col[mid];
        if (v == b) return 1;
        if (v < b) lo = mid + 1; else hi = mid;
    }
    return 0;
}

/* Is x a valid image for position t given images img[0..t-1]? */
static int acceptable(const job_t *J, int t, const int32_t *img, int32_t x) {
    for (int s = 0; s < t; ++s)
        if (img[s] == x) return 0;
    for (int q = 0; q < J->nback[t]; ++q)
        if (!adjacent(J, img[J->back[t][q]], x)) return 0;
    for (int q = 0; q < J->ngt[t]; ++q)
        if (!(img[J->gt[t][q]] > x)) return 0;
    for (int q = 0; q < J->nlt[t]; ++q)
        if (!(img[J->lt[t][q]] < x)) return 0;
    return 1;
}

static u128 extend(const job_t *J, int t, int32_t *img) {
    if (t == J->k) return 1;
    u128 total = 0;
    if (t < J->npin) {
        int32_t x = J->pin_value[t];
        if (acceptable(J, t, img, x)) {
            img[t] = x;
            total += extend(J, t + 1, img);
        }
        return total;
    }
    if (J->anchor[t] < 0) {
        for (int32_t x = 0; x < J->n; ++x) {
            if (!acceptable(J, t, img, x)) continue;
            img[t] = x;
            total += extend(J, t + 1, img);
        }
    } else {
        /* scan the shortest neighbor list among the placed pattern neighbors;
         * acceptable() still checks every pattern edge */
        int32_t a = img[J->anchor[t]];
        for (int q = 0; q < J->nback[t]; ++q) {
            int32_t b = img[J->back[t][q]];
            if (J->row_ptr[b + 1] - J->row_ptr[b] < J->row_ptr[a + 1] - J->row_ptr[a]) a = b;
        }
        for (int64_t e = J->row_ptr[a]; e < J->row_ptr[a + 1]; ++e) {
            int32_t x = J->col[e];
            if (!acceptable(J, t, img, x)) continue;
            img[t] = x;
            total += extend(J, t + 1, img);
        }
    }
    return total;
}

typedef struct {
    job_t *J;
    u128 result;
} worker_t;

/* Threads split the candidates of position 0 (all data vertices). */
static void *worker(void *arg) {
    worker_t *W = (worker_t *)arg;
    job_t *J = W->J;
    int32_t img[ORACLE_MAX_K];
    u128 total = 0;
    for (;;) {
        int64_t x = __atomic_fetch_add(&J->next_first, 1, __ATOMIC_RELAXED);
        if (x >= J->first_count) break;
        if (!acceptable(J, 0, img, (int32_t)x)) continue;
        img[0] = (int32_t)x;
        total += extend(J, 1, img);
    }
    W->result = total;
    return NULL;
}

/*
 * Count injective edge-preserving maps of the pattern (k vertices, ne edges
 * given as 2*ne vertex ids) into the graph, keeping only maps that satisfy
 * every restriction pair (restr[2q], restr[2q+1]) meaning id(a) > id(b), and
 * that send pattern vertex pin_vertex[q] to pin_value[q].
 * Returns 0 on success, -1 on a bad argument. The 128-bit count is split into
 * *out_lo / *out_hi.
 */
int oracle_count_maps(const int64_t *row_ptr, const int32_t *col, int32_t n,
                      int32_t k, const int32_t *edges, int32_t ne,
                      const int32_t *restr, int32_t nr,
                      const int32_t *pin_vertex, const int32_t *pin_value, int32_t npin,
                      int32_t nthreads, uint64_t *out_lo, uint64_t *out_hi) {
    if (k < 1 || k > ORACLE_MAX_K || n < 0 || ne < 0 || nr < 0 || npin < 0 || npin > k)
        return -1;
    int adj[ORACLE_MAX_K][ORACLE_MAX_K];
    memset(adj, 0, sizeof adj);
    for (int q = 0; q < ne; ++q) {
        int a = edges[2 * q], b = edges[2 * q + 1];
        if (a < 0 || a >= k || b < 0 || b >= k || a == b) return -1;
        adj[a][b] = adj[b][a] = 1;
    }
    for (int q = 0; q < nr; ++q) {
        int a = restr[2 * q], b = restr[2 * q + 1];
        if (a < 0 || a >= k || b < 0 || b >= k) return -1;
    }

    job_t *J = (job_t *)calloc(1, sizeof(job_t));
    if (!J) return -1;
    J->row_ptr = row_ptr;
    J->col = col;
    J->n = n;
    J->k = k;

    /* Search order: pinned vertices first, then repeatedly the smallest
     * unplaced vertex adjacent to a placed one (else the smallest unplaced). */
    int placed[ORACLE_MAX_K] = {0};
    int pos_of[ORACLE_MAX_K];
    int t = 0;
    for (int q = 0; q < npin; ++q) {
        int u = pin_vertex[q];
        if (u < 0 || u >= k || placed[u]) { free(J); return -1; }
        placed[u] = 1;
        pos_of[u] = t;
        J->order[t] = u;
        J->pin_value[t] = pin_value[q];
        if (pin_value[q] < 0 || pin_value[q] >= n) { free(J); return -1; }
        ++t;
    }
    J->npin = npin;
    while (t < k) {
        /* the unplaced vertex with the most placed neighbors (smallest id on
         * ties); with none adjacent, the smallest unplaced vertex */
        int pick = -1, best = 0;
        for (int u = 0; u < k; ++u) {
            if (placed[u]) continue;
            int c = 0;
            for (int w = 0; w < k; ++w)
                if (placed[w] && adj[u][w]) ++c;
            if (c > best) { best = c; pick = u; }
        }
        if (pick < 0)
            for (int u = 0; u < k; ++u)
                if (!placed[u]) { pick = u; break; }
        placed[pick] = 1;
        pos_of[pick] = t;
        J->order[t] = pick;
        ++t;
    }
    for (t = 0; t < k; ++t) {
        int u = J->order[t];
        J->anchor[t] = -1;
        J->nback[t] = J->ngt[t] = J->nlt[t] = 0;
        for (int s = 0; s < t; ++s) {
            int w = J->order[s];
            if (adj[u][w]) {
                if (J->anchor[t] < 0) J->anchor[t] = s;
                J->back[t][J->nback[t]++] = s;
            }
        }
        for (int q = 0; q < nr; ++q) {
            int a = restr[2 * q], b = restr[2 * q + 1];  /* id(a) > id(b) */
            if (a == b) continue;  /* handled below: unsatisfiable */
            if (b == u && pos_of[a] < t) J->gt[t][J->ngt[t]++] = pos_of[a];
            if (a == u && pos_of[b] < t) J->lt[t][J->nlt[t]++] = pos_of[b];
        }
    }
    /* A pair id(a) > id(a) can never hold: no map survives. */
    for (int q = 0; q < nr; ++q)
        if (restr[2 * q] == restr[2 * q + 1]) {
            free(J);
            *out_lo = 0;
            *out_hi = 0;
            return 0;
        }

    u128 total = 0;
    if (npin > 0 || n == 0 || nthreads <= 1) {
        int32_t img[ORACLE_MAX_K];
        if (npin > 0) {
            total = extend(J, 0, img);
        } else {
            J->next_first = 0;
            J->first_count = n;
            worker_t W = {J, 0};
            worker(&W);
            total = W.result;
        }
    } else {
        J->next_first = 0;
        J->first_count = n;
        pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
        worker_t *ws = (worker_t *)malloc(sizeof(worker_t) * (size_t)nthreads);
        if (!th || !ws) { free(th); free(ws); free(J); return -1; }
        int started = 0;
        for (int i = 0; i < nthreads; ++i) {
            ws[i].J = J;
            ws[i].result = 0;
            if (pthread_create(&th[i], NULL, worker, &ws[i]) != 0) break;
            ++started;
        }
        if (started == 0) {
            worker(&ws[0]);
            total = ws[0].result;
        } else {
            for (int i = 0; i < started; ++i) {
                pthread_join(th[i], NULL);
                total += ws[i].result;
            }
        }
        free(th);
        free(ws);
    }
    *out_lo = (uint64_t)total;
    *out_hi = (uint64_t)(total >> 64);
    free(J);
    return 0;
}
