/*
 * bc.h -- exact betweenness centrality on AMD Instinct MI355X (gfx950).
 *
 * The library computes, for an undirected graph with positive integer edge
 * weights, the betweenness centrality of every vertex (Kintali, "Betweenness
 * Centrality: Algorithms and Lower Bounds", Sec. 1.1):
 *
 *   BC(v) = sum over ordered pairs (s,t), s != v != t, of
 *           lambda_st(v) / lambda_st
 *         = sum over sources s != v of delta_s*(v),
 *
 * where lambda_st counts shortest s-t paths and delta_s*(v) is the dependency
 * of s on v.  Each source is processed as a forward sweep (distances and path
 * counts over the shortest-path DAG) followed by a backward sweep that applies
 * Brandes's recurrence (Theorem 1.1) farthest vertices first, and the
 * dependencies are added into a running score (Brandes's algorithm, Sec. 1.1).
 * Pairs are ORDERED and nothing is halved: the unordered-pair value is BC/2.
 * Unreachable targets contribute nothing.
 *
 * Every entry point returns a bc_status; no exception crosses this boundary.
 * All pointers are plain host or device pointers as stated per argument.
 * A context owns every device buffer it allocates until bc_destroy.  A context
 * is bound to one HIP stream and one device and is not thread-safe.
 */
#ifndef BC_H
#define BC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bc_ctx bc_ctx; /* opaque */

typedef enum {
    BC_OK = 0,
    BC_ERR_INVALID_ARG = 1,   /* NULL where a pointer is required, bad size, bad option */
    BC_ERR_INVALID_GRAPH = 2, /* CSR violates the graph model (see bc_graph) */
    BC_ERR_NOMEM = 3,         /* a device or host allocation failed */
    BC_ERR_DEVICE = 4,        /* a HIP runtime call failed; the context is poisoned */
    BC_ERR_OVERFLOW = 5,      /* a shortest-path count exceeded 2^64 - 1 */
    BC_ERR_STATE = 6,         /* call not allowed in the context's current state: the context
                                 was poisoned by a device error, or its stream is being
                                 captured into a HIP graph (no call may be recorded) */
    BC_ERR_UNSUPPORTED = 7    /* valid request this form cannot serve */
} bc_status;

typedef enum { BC_MEM_HOST = 0, BC_MEM_DEVICE = 1 } bc_mem;

/*
 * How the sweeps are computed.  Every form returns the same BC up to
 * floating-point rounding, and the same distances and path counts exactly.
 *
 *  BC_FORM_PLAIN_FP64  one source per workgroup, per-source state, dependencies
 *                      in FP64.  Unit weights by the level sweep of Sec. 4;
 *                      integer weights by bucketed shortest paths with one
 *                      bucket per distance value.
 *  BC_FORM_SPARSE      sources in batches (64, 128, 256 or 512; 0 = tuned);
 *                      per-level frontier bitmaps, one bit per (vertex, source);
 *                      CSR gathers pulled per vertex; path counts uint64,
 *                      dependency state stored as FP32 with FP64 accumulation.
 *                      Unit weights.
 *  BC_FORM_ALGEBRAIC   the algebraic method of Sec. 3.1 on a batch of sources:
 *                      frontier-matrix x adjacency products on MFMA, path
 *                      counts carried exactly in 7-bit limbs by int8 products
 *                      with int32 sums (forward), dependencies by BF16
 *                      products with FP32 sums (backward).  Unit
 *                      weights, or integer weights up to
 *                      BC_ALGEBRAIC_MAX_WEIGHT (Sec. 3.2): one 0/1 matrix per
 *                      weight c, levels are distances, and level L is the
 *                      sum over c of the class-c matrix times level L - c.
 *  BC_FORM_HYBRID      the sparse form's batches, where each level l >= 1 goes
 *                      either by CSR pulls or by the algebraic form's products,
 *                      chosen per batch from the level's union-frontier density
 *                      (the fraction of vertices at level l for at least one
 *                      source of the batch) against two thresholds (forward,
 *                      backward) fixed at create time by timed calibration
 *                      batches or a tuning cache.  Unit weights.  Graphs of
 *                      more than 92672 vertices (padded to a multiple of 256),
 *                      or with a degree above 65792, run every level by pulls.
 *  BC_FORM_AUTO        chosen by the library from the graph's shape.
 */
/* Largest integer weight the algebraic form takes (one product class each). */
#define BC_ALGEBRAIC_MAX_WEIGHT 8
/* Largest vertex degree the algebraic form takes: an output of a forward
 * product sums at most deg 7-bit limb terms in int32 and is copied to FP32
 * for the epilogue, exact while 127 * deg < 2^24 (this limit leaves a factor
 * of two).  bc_create refuses a larger degree with BC_ERR_UNSUPPORTED for the
 * algebraic form; the hybrid form then runs every level by pulls. */
#define BC_ALGEBRAIC_MAX_DEGREE 65792

typedef enum {
    BC_FORM_AUTO = 0,
    BC_FORM_PLAIN_FP64 = 1,
    BC_FORM_SPARSE = 2,
    BC_FORM_ALGEBRAIC = 3,
    BC_FORM_HYBRID = 4,
    BC_FORM_MANY = 5 /* reported by bc_get_info for bc_create_many contexts */
} bc_form;

/*
 * An undirected simple graph as a symmetric CSR (Sec. 1.1: vertices 0..n-1,
 * positive integer edge weights, unweighted meaning w = 1).
 *   n        number of vertices, 0 <= n < 2^31
 *   nnz      number of arcs = 2m (each undirected edge appears as both arcs)
 *   row_ptr  n+1 int32, row_ptr[0] = 0, nondecreasing, row_ptr[n] = nnz
 *   col      nnz int32; row v lists the neighbours of v in strictly
 *            increasing order (so no duplicate arcs); no self-loops; the arc
 *            (u,v) is present iff (v,u) is
 *   weight   nnz uint32 or NULL for unit weights; every weight >= 1; the two
 *            arcs of an edge carry the same weight; max weight * (n-1) < 2^31
 *   mem      whether row_ptr/col/weight are host or device pointers
 * Violations give BC_ERR_INVALID_GRAPH.  The arrays are copied; the caller
 * may free them as soon as the call returns.
 */
typedef struct {
    int32_t n;
    int32_t nnz;
    const int32_t *row_ptr;
    const int32_t *col;
    const uint32_t *weight;
    bc_mem mem;
} bc_graph;

/*
 * Device-memory provider.  alloc returns `bytes` of device memory usable on
 * `stream` (NULL on failure); free releases a pointer alloc returned.  When
 * both are NULL the library uses hipMalloc / hipFree.
 */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *user);
    void (*free)(void *ptr, void *stream, void *user);
    void *user;
} bc_allocator;

typedef struct {
    uint32_t struct_size; /* sizeof(bc_options); set by bc_options_init */
    bc_form form;         /* default BC_FORM_AUTO */
    int32_t batch;        /* sources per batch for batched forms.  0 = tuned for
                             the sparse and hybrid forms (timed calibration
                             batches choose among 128, 256, 512, or 256 and 512
                             when products are possible; graphs under 2048
                             vertices take 256), 256 for the algebraic form */
    int32_t device;       /* HIP device ordinal; -1 = the current device */
    void *stream;         /* hipStream_t to run on; NULL = the null stream */
    bc_allocator allocator;
    int32_t timing;       /* 0: off; k >= 1: HIP events on the launches of one source batch in k */
    int32_t split_degree; /* batched forms: rows longer than this are split into
                             segments of this many arcs; 0 = default (128) */
    int32_t vertex_order; /* internal vertex numbering (a device layout choice that
                             results never show): BC_ORDER_DEGREE (default) or
                             BC_ORDER_INPUT */
    int32_t arena_log2;   /* weighted graphs: each workgroup files relaxed vertices in
                             a ring of 2^arena_log2 entries (0 = default, max(4n, 2^16)
                             rounded up); a source that outgrows it is re-run with a
                             ring of nnz entries, so results never depend on it */
    const char *tune_cache; /* sparse, hybrid and algebraic forms and
                             bc_create_many: path of a text file of tuning
                             results keyed by the graph's shape (n, m, degree
                             histogram; for many graphs, the histograms of their
                             sizes), the form, the requested batch and the
                             device; a hit skips calibration, a miss appends the
                             result (measured, or measured earlier in this
                             process).  NULL = this process only. */
    int32_t grid;         /* plain form (unit and integer weights): persistent
                             workgroups, each running one source at a time;
                             0 = default (the most that fit a workspace budget,
                             at most 2048 unweighted, 1024 weighted; the budget
                             is 16 GB unweighted, 96 GB weighted, 192 GB weighted
                             with an explicit grid) */
    int32_t edges;        /* nonzero: also accumulate edge betweenness (read with
                             bc_read_edges).  Plain, sparse and hybrid forms
                             (the hybrid form then takes every backward level
                             by pulls); BC_ERR_UNSUPPORTED for the algebraic
                             form and bc_create_many. */
    int32_t host_driven;  /* batched forms, unit weights.  0 (default): bc_run
                             records one source batch's launches (every level of
                             the forward and backward sweeps, up to the deepest
                             level seen so far plus one) into a HIP graph once
                             and replays it for every batch, with no host
                             synchronisation between batches; a batch that
                             goes deeper, or whose counts need 64 bits, is
                             handed back and re-run when the context is next
                             used.  Nonzero: every batch is driven level by
                             level from the host, one synchronisation per
                             batch.  Results are the same. */
} bc_options;

/* Where the batch width and hybrid thresholds of a context came from. */
enum { BC_TUNE_DEFAULT = 0, BC_TUNE_MEASURED = 1, BC_TUNE_CACHED = 2 };

/* Internal vertex numbering.  BC_ORDER_DEGREE renumbers vertices by
 * nonincreasing degree so that the rows of high-degree vertices, which most
 * arcs point to, share a small region of memory; every input and output of the
 * interface stays in the caller's numbering. */
enum { BC_ORDER_DEGREE = 0, BC_ORDER_INPUT = 1 };

/* Fills *opt with the defaults above.  Never fails for a non-NULL opt. */
void bc_options_init(bc_options *opt);

/*
 * Validates the graph on the host (before any device work), then copies it to
 * device memory obtained from the allocator and prepares the chosen form.
 * On success *out receives a new context; on failure *out is set to NULL and
 * nothing stays allocated.  Errors: BC_ERR_INVALID_ARG, BC_ERR_INVALID_GRAPH,
 * BC_ERR_UNSUPPORTED (form cannot take this graph, e.g. weights with the
 * algebraic form), BC_ERR_NOMEM, BC_ERR_DEVICE.
 */
bc_status bc_create(const bc_graph *g, const bc_options *opt, bc_ctx **out);

/*
 * Many small graphs in one context, for all-source BC of every graph.
 *   gs[0..count)  unweighted graphs in host memory (mem = BC_MEM_HOST), each
 *                 satisfying the bc_graph model with at most 4096 vertices
 * The graphs are concatenated: vertex v of graph g has id
 * (n_0 + ... + n_{g-1}) + v, and bc_read returns BC in that numbering
 * (sum of n_g doubles).  opt->batch, when nonzero, is the number of sources
 * one work unit takes; 0 = tuned (timed launches over a sample of the graphs
 * choose among 16, 32, 64, 128 and 256; 64 when the graphs hold under 2048
 * vertices in all).  bc_run accepts only "every vertex"
 * (NULL, -1): it runs one persistent launch over a work queue of
 * (graph, source range) units, largest graphs first, recorded once into a HIP
 * graph and replayed.  bc_read_sssp takes ids in the concatenated numbering.
 * Errors: as bc_create; BC_ERR_UNSUPPORTED for weights or a graph above 4096
 * vertices.
 */
bc_status bc_create_many(const bc_graph *gs, int32_t count, const bc_options *opt, bc_ctx **out);

/*
 * Adds, for every entry s of `sources`, the dependencies delta_s*(v) of
 * s on every v != s into the context's running BC (Sec. 1.1, Brandes's
 * running centrality score).  `sources` is a multiset of vertex ids in
 * [0, n): an id listed twice adds twice.  sources = NULL with count = -1 means
 * every vertex once.  `mem` tells where `sources` lives.  The call is
 * asynchronous on the context's stream except where a form must read a
 * frontier size back; results are visible to bc_read.
 * Errors: BC_ERR_INVALID_ARG (id out of range, bad count), BC_ERR_STATE
 * (poisoned context), BC_ERR_OVERFLOW (a path count of an earlier call
 * exceeded 2^64 - 1), BC_ERR_NOMEM, BC_ERR_DEVICE.
 */
bc_status bc_run(bc_ctx *ctx, const int32_t *sources, int64_t count, bc_mem mem);

/*
 * Synchronises the context's stream, then copies BC (n doubles, vertex order)
 * to `bc_out` (host or device per `mem`).  Returns BC_ERR_OVERFLOW, leaving
 * bc_out unwritten, if any path count so far exceeded 2^64 - 1.
 */
bc_status bc_read(bc_ctx *ctx, double *bc_out, bc_mem mem);

/*
 * Edge betweenness (contexts created with edges != 0): for every arc e of the
 * caller's CSR, the betweenness of its undirected edge {u, col[e]} -- the sum,
 * over the sources run and every target t, of the fraction of shortest s-t
 * paths that use the edge (ordered pairs, no halving, as BC; both arcs of an
 * edge carry the same value).  For a source s each shortest-path DAG arc
 * v -> w contributes lambda_sv * (1 + delta_s*(w)) / lambda_sw, the per-arc
 * term of Theorem 1.1.  eb_out: nnz doubles (host or device per mem);
 * synchronises.  Errors: BC_ERR_UNSUPPORTED (context without edges),
 * BC_ERR_OVERFLOW as bc_read.
 */
bc_status bc_read_edges(bc_ctx *ctx, double *eb_out, bc_mem mem);

/* Zeroes the running BC (and edge betweenness) and clears a recorded overflow. */
bc_status bc_reset(bc_ctx *ctx);

/*
 * Runs `count` sources (1 <= count <= bc_info.batch) through exactly the
 * kernels and launch configuration bc_run uses, WITHOUT adding to BC, and
 * copies each source's per-vertex results to host arrays laid out
 * [count][n] (source-major; any pointer may be NULL):
 *   dist   d(s,v) (Sec. 1.1), -1 where v is unreachable from s
 *   sigma  lambda_sv, the number of shortest s-v paths (0 where unreachable)
 *   delta  delta_s*(v); delta_s*(s) is the recurrence's own value, the number
 *          of other vertices reachable from s
 * Errors as bc_run, plus BC_ERR_OVERFLOW when a count of these sources
 * exceeded 2^64 - 1 (the outputs are then unspecified).
 */
bc_status bc_read_sssp(bc_ctx *ctx, const int32_t *sources, int32_t count,
                       int32_t *dist, uint64_t *sigma, double *delta);

/*
 * Betweenness over every ordered pair by Algorithm 2 (Sec. 4.2.1).  Fills the
 * all-pairs distance matrix D and path-count matrix Lambda with the context's
 * own forward kernels (every vertex a source), then sums on the device, for
 * each vertex v, lambda_sv * lambda_vt / lambda_st over the ordered pairs
 * (s, t) with s != v != t and d(s,t) = d(s,v) + d(v,t): no dependencies and no
 * backward pass.  The result equals all-source BC (bc_run over every vertex)
 * and serves as an independent check of it and of the forward outputs.
 * Writes n doubles in the caller's vertex order to bc_out (host or device per
 * mem), computed in FP64; the running BC is left untouched.  Holds 12 n^2
 * bytes of device memory during the call (n <= BC_ALL_PAIRS_MAX_N: 12.9 GB).
 * Synchronises.
 * Errors: BC_ERR_UNSUPPORTED (context of many graphs, n above the limit),
 * BC_ERR_OVERFLOW (a path count exceeded 2^64 - 1; the running BC's own
 * overflow state is unchanged), BC_ERR_NOMEM, BC_ERR_DEVICE, BC_ERR_STATE.
 */
#define BC_ALL_PAIRS_MAX_N 32768
bc_status bc_all_pairs(bc_ctx *ctx, double *bc_out, bc_mem mem);

/*
 * Distances by Algorithm 1 (Sec. 4.1.1), the sampled forward for unweighted
 * graphs.  The distinguished set S is `sources` (each once) followed by
 * `sample` (the caller's random sample; ids already in S are skipped).  From
 * every x in S a `limit`-limited breadth-first search gives d'(x, v)
 * (limit 0 = ceil(sqrt(n))); the weighted graph H on S takes the edge weights
 * d'(x, y); all-pairs distances D_H of H follow; and for each source,
 * dist_out[i][v] = min over x in S of D_H(s_i, x) + d'(x, v).  Every value is
 * the length of a real walk, so it is never below d(s_i, v); it equals it when
 * each shortest path meets S at least once in every `limit` consecutive hops,
 * which a uniform sample of about sqrt(n) ln n vertices does with high
 * probability at limit sqrt(n).  -1 where no walk was found.  The number of
 * shortest paths (the paper's last step, a count of minimising vertices) is
 * not a path count and is not computed.
 *   sources, sample   host arrays of vertex ids in [0, n) (caller numbering)
 *   dist_out          count * n int32, row i for sources[i], in host or device
 *                     memory as `mem` says (device: written on the context's
 *                     stream, ordered before the call returns)
 * Synchronises.  Errors: BC_ERR_INVALID_ARG (bad id, count, limit above 65534),
 * BC_ERR_UNSUPPORTED (weighted graph, context of many graphs, |S| above
 * BC_SAMPLED_MAX_S), BC_ERR_NOMEM, BC_ERR_DEVICE, BC_ERR_STATE.
 */
#define BC_SAMPLED_MAX_S 4096
bc_status bc_sampled_distances(bc_ctx *ctx, const int32_t *sources, int32_t count, const int32_t *sample,
                               int32_t nsample, int32_t limit, int32_t *dist_out, bc_mem mem);

/*
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid allocation): bc_read_sssp, every output in DEVICE
 * memory, allocating nothing.
 *   sources             host array of count vertex ids, 1 <= count <= the
 *                       limit of bc_read_sssp
 *   dist, sigma, delta  device arrays of count * n elements (any may be NULL),
 *                       written exactly as bc_read_sssp writes its host arrays
 * The call stages the internal source ids and count * n cells of distance,
 * count and dependency -- about 20 * count * n bytes, plus 12 * count for a
 * context of many graphs -- in one fixed device array of
 * BC_NOALLOC_SCRATCH_BYTES, which the library holds on every GPU it runs on
 * until the process ends; a larger request gives BC_ERR_UNSUPPORTED.  Any
 * other allocation the context would need on the way (frontier levels for a
 * graph deeper than any batch run so far, a weighted source's larger arena,
 * the handed-back batches of an earlier replayed run) gives BC_ERR_NOMEM
 * instead; an ordinary call with the same sources first makes that room.
 * Every call on one GPU uses the same array, which keeps the last call's
 * contents: calls that overlap on one GPU (from several threads, or
 * contexts on other streams) race.  Synchronises.
 * Errors: as bc_read_sssp, BC_ERR_UNSUPPORTED, BC_ERR_NOMEM.
 */
#define BC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
bc_status bc_read_sssp_noalloc(bc_ctx *ctx, const int32_t *sources, int32_t count,
                               int32_t *dist, uint64_t *sigma, double *delta);

typedef struct {
    int32_t n;           /* vertices */
    int64_t m;           /* undirected edges = nnz / 2 */
    int32_t max_degree;
    int32_t weighted;    /* 1 when the graph carries weights */
    bc_form form;        /* the form in use (never BC_FORM_AUTO) */
    int32_t batch;       /* sources per batch (1 for the plain form; sources
                            per work unit for bc_create_many) */
    int32_t max_levels;  /* deepest level (or distinct distance count) seen + 1 */
    int64_t sources_run; /* sources accumulated since create / reset */
    int64_t device_bytes;/* device memory the context holds */
    double mfma_density_fwd; /* hybrid form: forward level l -> l+1 by products when
                                density(l) >= this (above 1: never); 0 for both
                                directions in the every-level mode (every level
                                by products and the algebraic form's end of
                                search), which the tuner keeps when whole
                                batches with it are faster */
    double mfma_density_bwd; /* hybrid form: backward level l by products when
                                density(l) >= this (above 1: never) */
    int32_t tune_source;     /* BC_TUNE_* for the tuned choices: batch width and
                                thresholds (sparse, hybrid), forward block rows
                                (algebraic, hybrid), sources per work unit
                                (bc_create_many) */
    int64_t mfma_planes;     /* products with the adjacency issued since create /
                                reset: one per 7-bit limb of a forward level, three
                                per backward level; each is batch * npad * K
                                multiply-adds, 2 * batch * npad * K flops (npad = n
                                rounded up to 256; K = npad, or M * npad with
                                weights 1..M) */
    int64_t mfma_ktiles_run;   /* k-tiles multiplied by those products; a k-tile is
                                  one plane's 32 adjacency columns (k) by 128
                                  adjacency rows by 128 sources, 2^20 flops, so
                                  executed flops = 2^20 * mfma_ktiles_run */
    int64_t mfma_ktiles_dense; /* k-tiles the issued products cover (2^20 *
                                  mfma_ktiles_dense = mfma_planes * 2 * batch *
                                  npad * K); the difference was skipped, every
                                  plane's k-tile zero */
    int64_t mfma_ktiles_run_fwd;   /* the forward products' share of mfma_ktiles_run */
    int64_t mfma_ktiles_dense_fwd; /* the forward products' share of mfma_ktiles_dense */
    int32_t mfma_fwd_rows;   /* algebraic and hybrid forms: adjacency rows per
                                workgroup of the forward products (128 or 256;
                                timed at create, see tune_source); 0 when the
                                context has no products */
} bc_info;

/* Fills *out; synchronises the context's stream (mfma_planes and the k-tile
 * counts are read from the device). */
bc_status bc_get_info(const bc_ctx *ctx, bc_info *out);

/*
 * Kernel timing (contexts created with timing = k >= 1).  For the kernel
 * named `kernel` (e.g. "plain_sweep", "fwd_pull", "bwd_pull"), returns the
 * number of its launches since create / reset and their summed duration in
 * milliseconds, measured with HIP events on the context's stream.  With k = 1
 * every launch is timed (the batched forms then drive every batch from the
 * host); with k > 1 the batched forms time every launch of the first source
 * batch and then of every k-th (so every level keeps its share), running
 * those batches host-driven and replaying the others, and scale the timed
 * batches' totals and launch counts to all batches; forms without batches
 * time every launch.  Unknown names give zero.
 * Synchronises the stream.  bc_create refuses a negative k.
 */
bc_status bc_get_timing(bc_ctx *ctx, const char *kernel, double *total_ms, int64_t *launches);

/* Static description of a status code. */
const char *bc_status_string(bc_status s);

/*
 * Message of the last failure on this context, or, with ctx = NULL, of the
 * last failed bc_create on the calling thread.  Valid until the next call on
 * the same context (thread).
 */
const char *bc_last_error(const bc_ctx *ctx);

/* Releases every resource of the context.  NULL is a no-op. */
void bc_destroy(bc_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* BC_H */
