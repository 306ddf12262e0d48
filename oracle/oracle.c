/*
 * CPU oracle for subgraph-embedding enumeration.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or helper with
 * the HIP path.
 *
 * What it computes (paper, Sec. III-A "Preliminaries"): for a data graph
 * G_d = (V_d, E_d) and a connected pattern graph G_p = (V_p, E_p), all
 * undirected and unlabeled, the set
 *
 *     Emb(G_p, G_d) = { f : V_p -> V_d  injective  :
 *                       for every {u,v} in E_p, {f(u), f(v)} in E_d }.
 *
 * This is the non-induced reading of the definition: it is exactly what the
 * method's join (edge preservation) plus its filter (no vertex used twice,
 * Sec. III-B, the "filter" step) enforces.  Data-graph self-loops are dropped
 * and both orientations of every edge are present (Sec. III-D: Res(M2) is
 * E_d without self-loops); duplicate edges are merged.
 *
 * Induced variant (flag `induced`): the definition in Sec. III-A also states
 * the converse, {u,v} in E_p exactly when {f(u), f(v)} in E_d; with the flag
 * set, a candidate is also rejected when it is adjacent to the image of an
 * earlier-mapped pattern vertex that is NOT its pattern neighbour, so the
 * result is the set of induced embeddings (the subgraph of G_d spanned by
 * f(V_p) equals f(G_p)).
 *
 * Scored variant (layout scoring, Sec. VI-D): with non-negative integer costs
 * c(x) per data vertex and c({x,y}) per data edge, the cost of f is
 *     cost(f) = sum_{v in V_p} c(f(v)) + sum_{{u,v} in E_p} c({f(u), f(v)})
 * (uint64, so the sum is exact and independent of evaluation order: the
 * paper's per-join product of fidelities, taken in the log domain with
 * fixed-point terms).  Rows are ordered by (cost ascending, row
 * lexicographically ascending) and the first top_k kept.
 *
 * The result is a table with one row per f, column j holding f(j), rows in
 * ascending lexicographic order, int32 values and an int64 count.  A cap keeps
 * the lexicographically first `cap` rows.
 *
 * Method: plain depth-first backtracking, written for clarity, not speed.
 *   1. Normalize G_d into sorted, duplicate-free adjacency lists.
 *   2. Check G_p: ids in range, no self-loop, connected (multi-edges merge).
 *   3. Order the pattern vertices by BFS from vertex 0 (neighbours ascending);
 *      every later vertex has an earlier neighbour, its parent.
 *   4. Position 0 tries every data vertex in ascending order; position i
 *      tries the neighbours of f(parent) in ascending order, rejecting a
 *      vertex already used and any vertex not adjacent to the image of an
 *      earlier-mapped pattern neighbour (binary search in the sorted list).
 *   5. At full depth, record (f(0), ..., f(k-1)) in pattern-vertex order.
 *   6. Sort rows lexicographically; assert that no two rows are equal.
 *
 * Streaming variant (outputs too large to store): instead of rows, it keeps
 * the count, the sum mod 2^64 and the XOR of a per-row hash:
 *     inner(f) = sum_j mix(((uint64)j << 32) | (uint32)f(j))  (mod 2^64)
 *     h(f)     = mix(inner(f))
 * where mix is SplitMix64's output step (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014): z = x + 0x9E3779B97F4A7C15,
 * z = (z ^ z>>30) * 0xBF58476D1CE4E5B9, z = (z ^ z>>27) * 0x94D049BB133111EB,
 * return z ^ z>>31.
 *
 * Return codes: 0 ok, -1 invalid argument, -2 vertex id out of range,
 * -3 pattern disconnected, -4 pattern self-loop, -5 out of memory,
 * -9 duplicate rows (impossible by construction; checked anyway).
 *
 * Mutation builds (-DORACLE_MUTANT=n) plant one plausible mistake each; the
 * test suite compiles them to show that its pins would catch such a mistake.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

enum { OR_OK = 0, OR_INVALID = -1, OR_RANGE = -2, OR_DISCONNECTED = -3,
       OR_SELF_LOOP = -4, OR_NOMEM = -5, OR_DUPLICATE = -9 };

/* ---------------------------------------------------------------- graphs */

typedef struct {
    int32_t n;
    int32_t *row_ptr; /* n + 1 */
    int32_t *col;     /* row_ptr[n] entries, each list ascending, no repeats */
} adj_t;

static int cmp_pair(const void *a, const void *b) {
    const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
    return 0;
}

static void adj_free(adj_t *g) {
    free(g->row_ptr);
    free(g->col);
    g->row_ptr = NULL;
    g->col = NULL;
}

/* Build sorted, duplicate-free, loop-free adjacency lists holding both
 * orientations of every input edge.  drop_loops = 0 reports a self-loop as an
 * error instead of dropping it (used for patterns). */
static int build_adj(int32_t n, int64_t m, const int32_t *edges, int drop_loops, adj_t *out) {
    out->n = n;
    out->row_ptr = NULL;
    out->col = NULL;
    if (n < 0 || m < 0 || (m > 0 && !edges)) return OR_INVALID;
    int32_t *pairs = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(2 * m + 1));
    if (!pairs) return OR_NOMEM;
    int64_t np = 0;
    for (int64_t e = 0; e < m; e++) {
        int32_t u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || v < 0 || u >= n || v >= n) { free(pairs); return OR_RANGE; }
        if (u == v) {
            if (!drop_loops) { free(pairs); return OR_SELF_LOOP; }
            continue;
        }
        pairs[2 * np] = u; pairs[2 * np + 1] = v; np++;
#if ORACLE_MUTANT != 6
        pairs[2 * np] = v; pairs[2 * np + 1] = u; np++;
#endif
    }
    qsort(pairs, (size_t)np, sizeof(int32_t) * 2, cmp_pair);
    out->row_ptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    out->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(np + 1));
    if (!out->row_ptr || !out->col) { free(pairs); adj_free(out); return OR_NOMEM; }
    int64_t w = 0;
    for (int64_t i = 0; i < np; i++) {
        if (i > 0 && pairs[2 * i] == pairs[2 * i - 2] && pairs[2 * i + 1] == pairs[2 * i - 1])
            continue; /* merge duplicate edge */
        out->col[w++] = pairs[2 * i + 1];
        out->row_ptr[pairs[2 * i] + 1]++;
    }
    for (int32_t v = 0; v < n; v++) out->row_ptr[v + 1] += out->row_ptr[v];
    free(pairs);
    return OR_OK;
}

static int adjacent(const adj_t *g, int32_t u, int32_t v) {
    int32_t lo = g->row_ptr[u], hi = g->row_ptr[u + 1];
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (g->col[mid] == v) return 1;
        if (g->col[mid] < v) lo = mid + 1; else hi = mid;
    }
    return 0;
}

/* ------------------------------------------------------------- row hash */

static uint64_t mix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static uint64_t row_hash(const int32_t *f, int32_t k) {
    uint64_t inner = 0;
    for (int32_t j = 0; j < k; j++) {
#if ORACLE_MUTANT == 8
        uint64_t key = ((uint64_t)(uint32_t)(j + 1) << 32) | (uint32_t)f[j];
#else
        uint64_t key = ((uint64_t)(uint32_t)j << 32) | (uint32_t)f[j];
#endif
        inner += mix64(key);
    }
    return mix64(inner);
}

/* --------------------------------------------------------- the search */

typedef struct {
    const adj_t *gd;
    const adj_t *gp;
    int32_t k;
    int32_t *order;   /* position -> pattern vertex */
    int32_t *parent;  /* pattern vertex -> parent pattern vertex (-1 for root) */
    int32_t *back;    /* flattened earlier-mapped neighbour lists */
    int32_t *back_ptr;
    int induced;      /* 1: also reject data edges between images of pattern non-neighbours */
    int32_t *nonback; /* flattened earlier-mapped non-neighbour lists (induced only) */
    int32_t *nonback_ptr;
    int32_t *f;       /* pattern vertex -> data vertex */
    uint8_t *used;    /* data vertex -> in use */
    int32_t root_lo, root_hi; /* images allowed for pattern vertex 0 */
    /* output */
    int stream;       /* 1: only count + hash */
    int32_t *rows;
    int64_t n_rows, cap_rows;
    int64_t count;
    uint64_t hsum, hxor;
    int oom;
} search_t;

static void emit(search_t *s) {
    s->count++;
    if (s->stream) {
        uint64_t h = row_hash(s->f, s->k);
        s->hsum += h;
        s->hxor ^= h;
        return;
    }
    if (s->n_rows == s->cap_rows) {
        int64_t nc = s->cap_rows ? 2 * s->cap_rows : 1024;
        int32_t *nr = (int32_t *)realloc(s->rows, sizeof(int32_t) * (size_t)(nc * s->k));
        if (!nr) { s->oom = 1; return; }
        s->rows = nr;
        s->cap_rows = nc;
    }
    int32_t *dst = s->rows + s->n_rows * s->k;
    for (int32_t j = 0; j < s->k; j++) {
#if ORACLE_MUTANT == 4
        dst[j] = s->f[s->order[j]]; /* wrong: search order instead of vertex order */
#else
        dst[j] = s->f[j];
#endif
    }
    s->n_rows++;
}

static void dfs(search_t *s, int32_t pos) {
    if (s->oom) return;
    if (pos == s->k) { emit(s); return; }
    int32_t p = s->order[pos];
    int32_t lo, hi;
    const int32_t *cand;
    if (pos == 0) {
        lo = s->root_lo;
#if ORACLE_MUTANT == 3
        hi = s->root_hi - 1; /* wrong: skips the last data vertex */
#else
        hi = s->root_hi;
#endif
        cand = NULL;
    } else {
        int32_t fp = s->f[s->parent[p]];
        lo = s->gd->row_ptr[fp];
        hi = s->gd->row_ptr[fp + 1];
        cand = s->gd->col;
    }
    for (int32_t i = lo; i < hi; i++) {
        int32_t c = cand ? cand[i] : i;
#if ORACLE_MUTANT != 1
        if (s->used[c]) continue;
#endif
        int ok = 1;
#if ORACLE_MUTANT != 2
        for (int32_t b = s->back_ptr[p]; b < s->back_ptr[p + 1] && ok; b++)
            if (!adjacent(s->gd, c, s->f[s->back[b]])) ok = 0;
#endif
        if (s->induced) {
#if ORACLE_MUTANT == 10
            if (pos + 1 < s->k) /* wrong: the last vertex skips the non-edge check */
#endif
            for (int32_t b = s->nonback_ptr[p]; b < s->nonback_ptr[p + 1] && ok; b++)
                if (adjacent(s->gd, c, s->f[s->nonback[b]])) ok = 0;
        }
        if (!ok) continue;
        s->f[p] = c;
        s->used[c] = 1;
        dfs(s, pos + 1);
        s->used[c] = 0;
        s->f[p] = -1;
    }
}

static int32_t g_sort_k; /* row width for the qsort comparator */

static int cmp_row(const void *a, const void *b) {
    const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
    for (int32_t j = 0; j < g_sort_k; j++) {
        if (x[j] != y[j]) {
#if ORACLE_MUTANT == 5
            return x[j] < y[j] ? 1 : -1; /* wrong: descending */
#else
            return x[j] < y[j] ? -1 : 1;
#endif
        }
    }
    return 0;
}

/* Shared driver: stream = 0 fills rows (caller frees with oracle_free),
 * stream = 1 fills count/hsum/hxor only. */
static int run(int32_t nd, int64_t md, const int32_t *ed,
               int32_t np, int64_t mp, const int32_t *ep,
               int stream, int64_t cap, int32_t root_lo, int32_t root_hi, int induced,
               int32_t **rows_out, int64_t *rows_n_out, int64_t *total_out,
               uint64_t *hsum_out, uint64_t *hxor_out) {
    if (rows_out) *rows_out = NULL;
    if (rows_n_out) *rows_n_out = 0;
    if (total_out) *total_out = 0;
    if (hsum_out) *hsum_out = 0;
    if (hxor_out) *hxor_out = 0;
    if (np <= 0 || nd < 0) return OR_INVALID;

    adj_t gd, gp;
    int rc = build_adj(nd, md, ed, 1, &gd);
    if (rc) return rc;
    rc = build_adj(np, mp, ep, 0, &gp);
    if (rc) { adj_free(&gd); return rc; }

    search_t s;
    memset(&s, 0, sizeof s);
    s.gd = &gd;
    s.gp = &gp;
    s.k = np;
    s.stream = stream;
    /* images of pattern vertex 0 restricted to [root_lo, root_hi) within [0, nd) */
    s.root_lo = root_lo < 0 ? 0 : root_lo;
    s.root_hi = root_hi > nd ? nd : root_hi;
    if (s.root_hi < s.root_lo) s.root_hi = s.root_lo;
    s.order = (int32_t *)malloc(sizeof(int32_t) * (size_t)np);
    s.parent = (int32_t *)malloc(sizeof(int32_t) * (size_t)np);
    s.back_ptr = (int32_t *)calloc((size_t)np + 1, sizeof(int32_t));
    s.back = (int32_t *)malloc(sizeof(int32_t) * (size_t)(gp.row_ptr[np] + 1));
    s.f = (int32_t *)malloc(sizeof(int32_t) * (size_t)np);
    s.used = (uint8_t *)calloc((size_t)(nd > 0 ? nd : 1), 1);
    s.induced = induced;
    s.nonback_ptr = (int32_t *)calloc((size_t)np + 1, sizeof(int32_t));
    s.nonback = (int32_t *)malloc(sizeof(int32_t) * ((size_t)np * (size_t)np + 1));
    int32_t *pos_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)np);
    if (!s.order || !s.parent || !s.back_ptr || !s.back || !s.f || !s.used || !pos_of || !s.nonback_ptr ||
        !s.nonback) {
        rc = OR_NOMEM;
        goto done;
    }

    /* BFS order from pattern vertex 0, neighbours ascending. */
    for (int32_t v = 0; v < np; v++) { pos_of[v] = -1; s.parent[v] = -1; s.f[v] = -1; }
    int32_t head = 0, tail = 0;
    s.order[tail++] = 0;
    pos_of[0] = 0;
    while (head < tail) {
        int32_t u = s.order[head++];
        for (int32_t i = gp.row_ptr[u]; i < gp.row_ptr[u + 1]; i++) {
            int32_t w = gp.col[i];
            if (pos_of[w] < 0) {
                pos_of[w] = tail;
                s.order[tail++] = w;
                s.parent[w] = u;
            }
        }
    }
    if (tail != np) { rc = OR_DISCONNECTED; goto done; }

    /* For each pattern vertex: its neighbours that are placed earlier. */
    for (int32_t v = 0; v < np; v++) {
        s.back_ptr[v + 1] = s.back_ptr[v];
        for (int32_t i = gp.row_ptr[v]; i < gp.row_ptr[v + 1]; i++)
            if (pos_of[gp.col[i]] < pos_of[v]) s.back[s.back_ptr[v + 1]++] = gp.col[i];
    }
    /* For each pattern vertex: the earlier-placed vertices that are not its
     * neighbours (every pattern non-edge is checked once, at its later end). */
    for (int32_t v = 0; v < np; v++) {
        s.nonback_ptr[v + 1] = s.nonback_ptr[v];
        for (int32_t w = 0; w < np; w++)
            if (w != v && pos_of[w] < pos_of[v] && !adjacent(&gp, v, w))
                s.nonback[s.nonback_ptr[v + 1]++] = w;
    }

    if (np <= nd) dfs(&s, 0);
    if (s.oom) { rc = OR_NOMEM; goto done; }

    if (!stream) {
        g_sort_k = np;
#if ORACLE_MUTANT != 9
        if (s.n_rows > 1) qsort(s.rows, (size_t)s.n_rows, sizeof(int32_t) * (size_t)np, cmp_row);
#endif
        for (int64_t r = 1; r < s.n_rows; r++)
            if (memcmp(s.rows + (r - 1) * np, s.rows + r * np, sizeof(int32_t) * (size_t)np) == 0) {
                rc = OR_DUPLICATE;
                goto done;
            }
        int64_t keep = s.n_rows;
        if (cap >= 0 && cap < keep) keep = cap;
#if ORACLE_MUTANT == 7
        if (cap > 0 && keep == cap) keep = cap - 1; /* wrong: off by one */
#endif
        if (rows_out) { *rows_out = s.rows; s.rows = NULL; }
        if (rows_n_out) *rows_n_out = keep;
    }
    if (total_out) *total_out = s.count;
    if (hsum_out) *hsum_out = s.hsum;
    if (hxor_out) *hxor_out = s.hxor;
    rc = OR_OK;

done:
    free(s.rows);
    free(s.order);
    free(s.parent);
    free(s.back_ptr);
    free(s.back);
    free(s.f);
    free(s.used);
    free(s.nonback);
    free(s.nonback_ptr);
    free(pos_of);
    adj_free(&gd);
    adj_free(&gp);
    return rc;
}

/* ------------------------------------------------------------ exports */

/* Normalized adjacency of a data graph: row_ptr[n+1], col[row_ptr[n]]
 * (caller provides col with room for 2*m entries).  Returns the number of
 * directed entries, or a negative code. */
int64_t oracle_normalize(int32_t n, int64_t m, const int32_t *edges,
                         int32_t *row_ptr, int32_t *col) {
    adj_t g;
    int rc = build_adj(n, m, edges, 1, &g);
    if (rc) return rc;
#if ORACLE_MUTANT == 12
    memcpy(row_ptr, g.row_ptr, sizeof(int32_t) * (size_t)n); /* last offset left out */
#else
    memcpy(row_ptr, g.row_ptr, sizeof(int32_t) * ((size_t)n + 1));
#endif
    int64_t nnz = g.row_ptr[n];
#if ORACLE_MUTANT == 13
    if (nnz > 1) memcpy(col, g.col + 1, sizeof(int32_t) * (size_t)(nnz - 1)); /* lists shifted by one */
#else
    if (nnz) memcpy(col, g.col, sizeof(int32_t) * (size_t)nnz);
#endif
    adj_free(&g);
    return nnz;
}

/* All embeddings as a sorted row-major table (malloc'd; free with
 * oracle_free).  *n_rows = min(cap, total) (cap < 0: all); *total = count. */
int oracle_enumerate(int32_t nd, int64_t md, const int32_t *ed,
                     int32_t np, int64_t mp, const int32_t *ep, int64_t cap,
                     int32_t **rows, int64_t *n_rows, int64_t *total) {
    return run(nd, md, ed, np, mp, ep, 0, cap, 0, nd, 0, rows, n_rows, total, NULL, NULL);
}

/* As oracle_enumerate, keeping only embeddings with f(0) in [root_lo, root_hi). */
int oracle_enumerate_range(int32_t nd, int64_t md, const int32_t *ed,
                           int32_t np, int64_t mp, const int32_t *ep, int64_t cap,
                           int32_t root_lo, int32_t root_hi,
                           int32_t **rows, int64_t *n_rows, int64_t *total) {
    return run(nd, md, ed, np, mp, ep, 0, cap, root_lo, root_hi, 0, rows, n_rows, total, NULL, NULL);
}

/* As oracle_enumerate_range, with induced = 1 selecting induced embeddings. */
int oracle_enumerate_ex(int32_t nd, int64_t md, const int32_t *ed,
                        int32_t np, int64_t mp, const int32_t *ep, int64_t cap,
                        int32_t root_lo, int32_t root_hi, int32_t induced,
                        int32_t **rows, int64_t *n_rows, int64_t *total) {
    return run(nd, md, ed, np, mp, ep, 0, cap, root_lo, root_hi, induced != 0, rows, n_rows, total, NULL, NULL);
}

/* Streaming count + order-independent multiset hash (see header). */
int oracle_count_hash(int32_t nd, int64_t md, const int32_t *ed,
                      int32_t np, int64_t mp, const int32_t *ep,
                      int64_t *count, uint64_t *hsum, uint64_t *hxor) {
    return run(nd, md, ed, np, mp, ep, 1, -1, 0, nd, 0, NULL, NULL, count, hsum, hxor);
}

/* As oracle_count_hash, counting only embeddings with f(0) in
 * [root_lo, root_hi) (the sums and XORs of a partition of the roots combine
 * into the full result). */
int oracle_count_hash_range(int32_t nd, int64_t md, const int32_t *ed,
                            int32_t np, int64_t mp, const int32_t *ep,
                            int32_t root_lo, int32_t root_hi,
                            int64_t *count, uint64_t *hsum, uint64_t *hxor) {
    return run(nd, md, ed, np, mp, ep, 1, -1, root_lo, root_hi, 0, NULL, NULL, count, hsum, hxor);
}

/* As oracle_count_hash, with induced = 1 selecting induced embeddings. */
int oracle_count_hash_ex(int32_t nd, int64_t md, const int32_t *ed,
                         int32_t np, int64_t mp, const int32_t *ep, int32_t induced,
                         int64_t *count, uint64_t *hsum, uint64_t *hxor) {
    return run(nd, md, ed, np, mp, ep, 1, -1, 0, nd, induced != 0, NULL, NULL, count, hsum, hxor);
}

/* Scored enumeration (see the header): all embeddings (induced != 0: the
 * induced ones), each with its cost, ordered by (cost, row) ascending; the
 * first top_k rows (top_k < 0: all).  vcost: nd entries (NULL = zeros);
 * cedges/ecost: mc data edges and their costs (each edge of G_d at most
 * once; unlisted edges cost 0).  *rows and *costs are malloc'd (free with
 * oracle_free).  Returns OR_INVALID for a listed pair that is not an edge of
 * G_d or is listed twice. */
static const int32_t *g_rows_k_base;
static const uint64_t *g_costs_base;

static int cmp_scored(const void *a, const void *b) {
    const int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    if (g_costs_base[x] != g_costs_base[y]) return g_costs_base[x] < g_costs_base[y] ? -1 : 1;
    const int32_t *rx = g_rows_k_base + x * g_sort_k, *ry = g_rows_k_base + y * g_sort_k;
    for (int32_t j = 0; j < g_sort_k; j++)
        if (rx[j] != ry[j]) return rx[j] < ry[j] ? -1 : 1;
    return 0;
}

int oracle_enumerate_scored(int32_t nd, int64_t md, const int32_t *ed,
                            int32_t np, int64_t mp, const int32_t *ep,
                            const uint32_t *vcost, int64_t mc, const int32_t *cedges, const uint32_t *ecost,
                            int64_t top_k, int32_t induced,
                            int32_t **rows_out, uint64_t **costs_out, int64_t *n_rows, int64_t *total) {
    *rows_out = NULL;
    *costs_out = NULL;
    *n_rows = 0;
    *total = 0;
    if (mc < 0 || (mc > 0 && (!cedges || !ecost))) return OR_INVALID;
    adj_t gd;
    int rc = build_adj(nd, md, ed, 1, &gd);
    if (rc) return rc;
    /* cost of each directed entry of the adjacency lists */
    int64_t nnz = gd.row_ptr[nd];
    uint32_t *ec = (uint32_t *)calloc((size_t)(nnz + 1), sizeof(uint32_t));
    uint8_t *seen = (uint8_t *)calloc((size_t)(nnz + 1), 1);
    if (!ec || !seen) { free(ec); free(seen); adj_free(&gd); return OR_NOMEM; }
    for (int64_t e = 0; e < mc && rc == OR_OK; e++) {
        for (int o = 0; o < 2 && rc == OR_OK; o++) {
            int32_t x = cedges[2 * e + o], y = cedges[2 * e + 1 - o];
            if (x < 0 || y < 0 || x >= nd || y >= nd) { rc = OR_INVALID; break; }
            int32_t lo = gd.row_ptr[x], hi = gd.row_ptr[x + 1], at = -1;
            while (lo < hi) {
                int32_t mid = lo + (hi - lo) / 2;
                if (gd.col[mid] == y) { at = mid; break; }
                if (gd.col[mid] < y) lo = mid + 1; else hi = mid;
            }
            if (at < 0 || seen[at]) { rc = OR_INVALID; break; }
            seen[at] = 1;
            ec[at] = ecost[e];
        }
    }
    int32_t *rows = NULL;
    int64_t nr = 0, tot = 0;
    if (rc == OR_OK)
        rc = run(nd, md, ed, np, mp, ep, 0, -1, 0, nd, induced != 0, &rows, &nr, &tot, NULL, NULL);
    uint64_t *cost = NULL;
    int64_t *ord = NULL;
    if (rc == OR_OK) {
        cost = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nr + 1));
        ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nr + 1));
        if (!cost || !ord) rc = OR_NOMEM;
    }
    if (rc == OR_OK) {
        /* pattern edges once each (u < v) */
        adj_t gp;
        rc = build_adj(np, mp, ep, 0, &gp);
        for (int64_t r = 0; r < nr && rc == OR_OK; r++) {
            const int32_t *f = rows + r * np;
            uint64_t c = 0;
#if ORACLE_MUTANT == 11
            for (int32_t v = 1; v < np; v++) /* wrong: the root's vertex cost is skipped */
#else
            for (int32_t v = 0; v < np; v++)
#endif
                c += vcost ? vcost[f[v]] : 0;
            for (int32_t u = 0; u < np; u++)
                for (int32_t i = gp.row_ptr[u]; i < gp.row_ptr[u + 1]; i++) {
                    int32_t v = gp.col[i];
                    if (v < u) continue;
                    int32_t x = f[u], y = f[v], lo = gd.row_ptr[x], hi = gd.row_ptr[x + 1];
                    while (lo < hi) {
                        int32_t mid = lo + (hi - lo) / 2;
                        if (gd.col[mid] == y) { c += ec[mid]; break; }
                        if (gd.col[mid] < y) lo = mid + 1; else hi = mid;
                    }
                }
            cost[r] = c;
            ord[r] = r;
        }
        if (rc == OR_OK) adj_free(&gp);
    }
    if (rc == OR_OK) {
        g_sort_k = np;
        g_rows_k_base = rows;
        g_costs_base = cost;
        if (nr > 1) qsort(ord, (size_t)nr, sizeof(int64_t), cmp_scored);
        int64_t keep = (top_k >= 0 && top_k < nr) ? top_k : nr;
        int32_t *ro = (int32_t *)malloc(sizeof(int32_t) * (size_t)(keep * np + 1));
        uint64_t *co = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(keep + 1));
        if (!ro || !co) {
            free(ro);
            free(co);
            rc = OR_NOMEM;
        } else {
            for (int64_t i = 0; i < keep; i++) {
                memcpy(ro + i * np, rows + ord[i] * np, sizeof(int32_t) * (size_t)np);
                co[i] = cost[ord[i]];
            }
            *rows_out = ro;
            *costs_out = co;
            *n_rows = keep;
            *total = tot;
        }
    }
    free(rows);
    free(cost);
    free(ord);
    free(ec);
    free(seen);
    adj_free(&gd);
    return rc;
}

/* Hash of one row given in pattern-vertex order (for table-side summaries). */
uint64_t oracle_row_hash(const int32_t *row, int32_t k) { return row_hash(row, k); }

void oracle_free(void *p) { free(p); }

int oracle_mutant_id(void) { return ORACLE_MUTANT; }

/* The SplitMix64 output step on its own (so tests can check it against the
 * generator's published outputs). */
uint64_t oracle_mix64(uint64_t x) { return mix64(x); }
