/*
 * Plain serial Brandes betweenness centrality -- the ORACLE.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file: only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code with the GPU library.
 *
 * What it computes (Kintali, "Betweenness Centrality: Algorithms and Lower
 * Bounds", Sec. 1.1):
 *   - d(s,v), the distance, with d(s,s) = 0;
 *   - lambda_sv, the number of shortest s-v paths, with lambda_ss = 1
 *     (called sigma here, as in Brandes);
 *   - the dependency delta_s*(v) by Theorem 1.1,
 *       delta_s*(v) = sum over w with v in P_s(w) of
 *                     (lambda_sv / lambda_sw) * (1 + delta_s*(w)),
 *     where P_s(w) = { u : (u,w) in E, d(s,w) = d(s,u) + w(u,w) };
 *   - BC(v) = sum over sources s != v of delta_s*(v): the running score of
 *     Brandes's algorithm, over ordered pairs, with no halving;
 *   - optionally the edge betweenness of every edge {v,x}: the sum over
 *     ordered pairs (s,t) of the fraction of shortest s-t paths that use the
 *     edge.  For a source s each shortest-path DAG arc v -> x (v in P_s(x))
 *     carries (lambda_sv / lambda_sx) * (1 + delta_s*(x)) of them -- the same
 *     per-arc term whose sum over x is delta_s*(v) in Theorem 1.1.
 *
 * Unit weights use a FIFO breadth-first search; positive integer weights use
 * Dijkstra's algorithm with a binary heap, then visit the reached vertices in
 * nondecreasing (distance, id) order, which is a topological order of the
 * shortest-path DAG because every weight is at least 1.
 *
 * Path counts are exact: they are held as unsigned 128-bit integers with
 * checked additions.  A count above 2^128 - 1 makes the call fail with
 * ORACLE_ERR_OVERFLOW.  Dependencies and BC are IEEE double.  The ratio
 * lambda_sv / lambda_sw is the correctly rounded quotient of the two counts
 * converted to double, and the dependency sum is taken term by term in the
 * per-arc form of Theorem 1.1.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

enum { ORACLE_OK = 0, ORACLE_ERR_OVERFLOW = 1, ORACLE_ERR_ARG = 2, ORACLE_ERR_NOMEM = 3 };

typedef struct {
    int32_t n;
    const int32_t *row_ptr;
    const int32_t *col;
    const uint32_t *weight; /* NULL: every edge weighs 1 */
} graph_t;

typedef struct {
    int64_t *dist;   /* -1 = unreachable */
    u128 *sigma;
    double *delta;
    int32_t *order;  /* reached vertices, nondecreasing distance */
    int64_t *heap_d; /* Dijkstra heap: keys */
    int32_t *heap_v; /* Dijkstra heap: vertices */
    int32_t reached;
    int sigma_above_u64; /* some count exceeded 2^64 - 1 */
} work_t;

static int work_alloc(work_t *w, int32_t n, int64_t nnz) {
    memset(w, 0, sizeof(*w));
    size_t nn = n > 0 ? (size_t)n : 1;
    size_t hh = (size_t)nnz + nn + 1;
    w->dist = malloc(nn * sizeof(int64_t));
    w->sigma = malloc(nn * sizeof(u128));
    w->delta = malloc(nn * sizeof(double));
    w->order = malloc(nn * sizeof(int32_t));
    w->heap_d = malloc(hh * sizeof(int64_t));
    w->heap_v = malloc(hh * sizeof(int32_t));
    return (w->dist && w->sigma && w->delta && w->order && w->heap_d && w->heap_v) ? 0 : -1;
}

static void work_free(work_t *w) {
    free(w->dist); free(w->sigma); free(w->delta);
    free(w->order); free(w->heap_d); free(w->heap_v);
}

static int add_count(u128 *acc, u128 x, work_t *w) {
    u128 r;
    if (__builtin_add_overflow(*acc, x, &r)) return -1;
    *acc = r;
    if (r > (u128)UINT64_MAX) w->sigma_above_u64 = 1;
    return 0;
}

/* ---- forward sweep, unit weights: breadth-first search, counting paths ---- */
static int forward_bfs(const graph_t *g, int32_t s, work_t *w) {
    for (int32_t v = 0; v < g->n; ++v) { w->dist[v] = -1; w->sigma[v] = 0; }
    w->dist[s] = 0;
    w->sigma[s] = 1;
    int32_t head = 0, tail = 0;
    w->order[tail++] = s;
    while (head < tail) {
        int32_t v = w->order[head++];
        for (int32_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
            int32_t x = g->col[e];
            if (w->dist[x] < 0) {
                w->dist[x] = w->dist[v] + 1;
                w->order[tail++] = x;
            }
            if (w->dist[x] == w->dist[v] + 1) {
                if (add_count(&w->sigma[x], w->sigma[v], w)) return ORACLE_ERR_OVERFLOW;
            }
        }
    }
    w->reached = tail;
    return ORACLE_OK;
}

/* ---- forward sweep, integer weights: Dijkstra, then counts in order ---- */
static void heap_push(work_t *w, int32_t *size, int64_t d, int32_t v) {
    int32_t i = (*size)++;
    while (i > 0) {
        int32_t p = (i - 1) / 2;
        if (w->heap_d[p] <= d) break;
        w->heap_d[i] = w->heap_d[p]; w->heap_v[i] = w->heap_v[p];
        i = p;
    }
    w->heap_d[i] = d; w->heap_v[i] = v;
}

static void heap_pop(work_t *w, int32_t *size, int64_t *d, int32_t *v) {
    *d = w->heap_d[0]; *v = w->heap_v[0];
    int32_t n = --(*size);
    int64_t kd = w->heap_d[n]; int32_t kv = w->heap_v[n];
    int32_t i = 0;
    for (;;) {
        int32_t c = 2 * i + 1;
        if (c >= n) break;
        if (c + 1 < n && w->heap_d[c + 1] < w->heap_d[c]) ++c;
        if (w->heap_d[c] >= kd) break;
        w->heap_d[i] = w->heap_d[c]; w->heap_v[i] = w->heap_v[c];
        i = c;
    }
    w->heap_d[i] = kd; w->heap_v[i] = kv;
}

/* sort key of the comparator below, per thread */
static __thread const int64_t *t_sort_dist;

static int by_dist_then_id(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    int64_t dx = t_sort_dist[x], dy = t_sort_dist[y];
    if (dx != dy) return dx < dy ? -1 : 1;
    return (x > y) - (x < y);
}

static int forward_dijkstra(const graph_t *g, int32_t s, work_t *w) {
    for (int32_t v = 0; v < g->n; ++v) { w->dist[v] = -1; w->sigma[v] = 0; }
    int32_t hs = 0, reached = 0;
    w->dist[s] = 0;
    heap_push(w, &hs, 0, s);
    while (hs > 0) {
        int64_t d; int32_t v;
        heap_pop(w, &hs, &d, &v);
        if (d != w->dist[v]) continue;                 /* stale entry */
        for (int32_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
            int32_t x = g->col[e];
            int64_t nd = d + (int64_t)g->weight[e];
            if (w->dist[x] < 0 || nd < w->dist[x]) {
                w->dist[x] = nd;
                heap_push(w, &hs, nd, x);
            }
        }
    }
    for (int32_t v = 0; v < g->n; ++v)
        if (w->dist[v] >= 0) w->order[reached++] = v;
    t_sort_dist = w->dist;
    qsort(w->order, (size_t)reached, sizeof(int32_t), by_dist_then_id);
    /* counts: sigma(x) = sum of sigma(v) over predecessors v of x */
    w->sigma[s] = 1;
    for (int32_t i = 1; i < reached; ++i) {
        int32_t x = w->order[i];
        for (int32_t e = g->row_ptr[x]; e < g->row_ptr[x + 1]; ++e) {
            int32_t v = g->col[e];
            if (w->dist[v] >= 0 && w->dist[v] + (int64_t)g->weight[e] == w->dist[x])
                if (add_count(&w->sigma[x], w->sigma[v], w)) return ORACLE_ERR_OVERFLOW;
        }
    }
    w->reached = reached;
    return ORACLE_OK;
}

/* ---- backward sweep: Theorem 1.1, farthest vertices first ---- */
/* eb (may be NULL): per-arc edge betweenness, each DAG arc's term added to it */
static void backward(const graph_t *g, work_t *w, double *eb) {
    for (int32_t v = 0; v < g->n; ++v) w->delta[v] = 0.0;
    for (int32_t i = w->reached - 1; i >= 0; --i) {
        int32_t v = w->order[i];
        double acc = 0.0;
        for (int32_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
            int32_t x = g->col[e];
            int64_t wt = g->weight ? (int64_t)g->weight[e] : 1;
            if (w->dist[x] >= 0 && w->dist[x] == w->dist[v] + wt) { /* v in P_s(x) */
                double ratio = (double)w->sigma[v] / (double)w->sigma[x];
                double term = ratio * (1.0 + w->delta[x]);
                acc += term;
                if (eb) eb[e] += term;
            }
        }
        w->delta[v] = acc;
    }
}

static int single_source(const graph_t *g, int32_t s, work_t *w, double *eb) {
    int rc = g->weight ? forward_dijkstra(g, s, w) : forward_bfs(g, s, w);
    if (rc) return rc;
    backward(g, w, eb);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */

typedef struct {
    const graph_t *g;
    const int32_t *sources;
    int64_t begin, end;
    double *bc;  /* this thread's partial sum, n entries */
    double *eb;  /* this thread's per-arc partial sum, nnz entries, or NULL */
    int rc;
    int above_u64;
} job_t;

static void *run_job(void *arg) {
    job_t *j = (job_t *)arg;
    work_t w;
    if (work_alloc(&w, j->g->n, j->g->row_ptr[j->g->n])) { work_free(&w); j->rc = ORACLE_ERR_NOMEM; return NULL; }
    for (int64_t i = j->begin; i < j->end && !j->rc; ++i) {
        int32_t s = j->sources[i];
        j->rc = single_source(j->g, s, &w, j->eb);
        if (j->rc) break;
        for (int32_t v = 0; v < j->g->n; ++v)
            if (v != s) j->bc[v] += w.delta[v];
    }
    j->above_u64 = w.sigma_above_u64;
    work_free(&w);
    return NULL;
}

static int check_graph(int32_t n, const int32_t *row_ptr, const int32_t *col) {
    if (n < 0 || !row_ptr || (n > 0 && row_ptr[n] > 0 && !col)) return -1;
    if (row_ptr[0] != 0) return -1;
    for (int32_t v = 0; v < n; ++v) {
        if (row_ptr[v + 1] < row_ptr[v]) return -1;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
            if (col[e] < 0 || col[e] >= n) return -1;
    }
    return 0;
}

/*
 * BC over the given sources (a multiset of vertex ids; each entry adds its
 * dependencies).  bc_out: n doubles, overwritten.  eb_out (may be NULL): nnz
 * doubles, overwritten with the edge betweenness of each arc's edge (both
 * arcs of an edge carry the same value: the sum of the terms of its two
 * directions).  Rows must be sorted when eb_out is requested.  Sources are
 * split into nthreads contiguous chunks; per-thread partial sums are added in
 * thread order, so the result is deterministic for a fixed nthreads.
 * above_u64_out (may be NULL): set to 1 when some path count exceeded 2^64-1.
 */
int oracle_edge_bc(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint32_t *weight,
                   const int32_t *sources, int64_t nsources, int32_t nthreads,
                   double *bc_out, double *eb_out, int32_t *above_u64_out) {
    if (check_graph(n, row_ptr, col) || !bc_out || nsources < 0 || (nsources > 0 && !sources))
        return ORACLE_ERR_ARG;
    for (int64_t i = 0; i < nsources; ++i)
        if (sources[i] < 0 || sources[i] >= n) return ORACLE_ERR_ARG;
    if (weight)
        for (int32_t e = 0; e < row_ptr[n]; ++e)
            if (weight[e] == 0) return ORACLE_ERR_ARG;
    const int64_t nnz = row_ptr[n];
    graph_t g = { n, row_ptr, col, weight };
    if (nthreads < 1) nthreads = 1;
    if (nthreads > nsources && nsources > 0) nthreads = (int32_t)nsources;
    if (nsources == 0) nthreads = 1;
    job_t *jobs = calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *th = calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return ORACLE_ERR_NOMEM; }
    int rc = ORACLE_OK;
    for (int32_t t = 0; t < nthreads; ++t) {
        jobs[t].g = &g;
        jobs[t].sources = sources;
        jobs[t].begin = nsources * t / nthreads;
        jobs[t].end = nsources * (t + 1) / nthreads;
        jobs[t].bc = calloc(n > 0 ? (size_t)n : 1, sizeof(double));
        if (!jobs[t].bc) rc = ORACLE_ERR_NOMEM;
        if (eb_out) {
            jobs[t].eb = calloc(nnz > 0 ? (size_t)nnz : 1, sizeof(double));
            if (!jobs[t].eb) rc = ORACLE_ERR_NOMEM;
        }
    }
    if (rc == ORACLE_OK) {
        if (nthreads == 1) {
            run_job(&jobs[0]);
        } else {
            for (int32_t t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, run_job, &jobs[t]);
            for (int32_t t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
        }
        for (int32_t v = 0; v < n; ++v) bc_out[v] = 0.0;
        int above = 0;
        for (int32_t t = 0; t < nthreads; ++t) {
            if (jobs[t].rc && !rc) rc = jobs[t].rc;
            above |= jobs[t].above_u64;
            for (int32_t v = 0; v < n; ++v) bc_out[v] += jobs[t].bc[v];
        }
        if (eb_out) {
            double *arc = calloc(nnz > 0 ? (size_t)nnz : 1, sizeof(double));
            if (!arc) rc = rc ? rc : ORACLE_ERR_NOMEM;
            else {
                for (int32_t t = 0; t < nthreads; ++t)
                    for (int64_t e = 0; e < nnz; ++e) arc[e] += jobs[t].eb[e];
                /* an edge's value: the terms of both of its arcs */
                for (int32_t v = 0; v < n; ++v)
                    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                        int32_t x = col[e], lo = row_ptr[x], hi = row_ptr[x + 1];
                        while (lo < hi) { /* the reverse arc x -> v in x's sorted row */
                            int32_t mid = lo + (hi - lo) / 2;
                            if (col[mid] < v) lo = mid + 1;
                            else hi = mid;
                        }
                        eb_out[e] = arc[e] + (lo < row_ptr[x + 1] && col[lo] == v ? arc[lo] : 0.0);
                    }
                free(arc);
            }
        }
        if (above_u64_out) *above_u64_out = above;
    }
    for (int32_t t = 0; t < nthreads; ++t) { free(jobs[t].bc); free(jobs[t].eb); }
    free(jobs); free(th);
    return rc;
}

/* BC only: oracle_edge_bc without the edge output. */
int oracle_bc(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint32_t *weight,
              const int32_t *sources, int64_t nsources, int32_t nthreads,
              double *bc_out, int32_t *above_u64_out) {
    return oracle_edge_bc(n, row_ptr, col, weight, sources, nsources, nthreads, bc_out, NULL, above_u64_out);
}

/*
 * One source's forward and backward sweeps.  Outputs (each n entries, any may
 * be NULL): dist (-1 = unreachable), the path count split into its low and
 * high 64-bit halves, and the dependency delta_s*(v) (delta_s*(s) included:
 * the recurrence gives it the number of other reachable vertices).
 */
int oracle_sssp(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint32_t *weight,
                int32_t s, int64_t *dist, uint64_t *sigma_lo, uint64_t *sigma_hi, double *delta) {
    if (check_graph(n, row_ptr, col) || s < 0 || s >= n) return ORACLE_ERR_ARG;
    graph_t g = { n, row_ptr, col, weight };
    work_t w;
    if (work_alloc(&w, n, row_ptr[n])) { work_free(&w); return ORACLE_ERR_NOMEM; }
    int rc = single_source(&g, s, &w, NULL);
    if (rc == ORACLE_OK) {
        for (int32_t v = 0; v < n; ++v) {
            if (dist) dist[v] = w.dist[v];
            if (sigma_lo) sigma_lo[v] = (uint64_t)w.sigma[v];
            if (sigma_hi) sigma_hi[v] = (uint64_t)(w.sigma[v] >> 64);
            if (delta) delta[v] = w.delta[v];
        }
    }
    work_free(&w);
    return rc;
}
