// Internal declarations shared by the host side of the library and the
// kernel launchers.  Not part of the public interface (include/bc.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "bc.h"

// Device status word bits, OR-ed in by kernels and read by bc_read.
enum : uint32_t {
    BC_DEV_SIGMA_OVERFLOW = 1u, // a path count exceeded 2^64 - 1
};

// Timing of one kernel name: HIP event pairs not yet folded into total_ms.
struct KernelTimer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    double total_ms = 0.0; // summed over the timed launches
    int64_t launches = 0;
    int64_t timed = 0;     // launches that carried an event pair
};

// Device control block of a replayed run of source batches (see sparse.hip):
// the batch counter that tells each replay which sources it takes, and what
// the per-batch checks found.
struct BatchCtl {
    int32_t batch;          // index of the batch the next replay runs
    int32_t total;          // sources in the run
    const int32_t *src;     // the run's internal source ids
    int32_t *redo;          // [batches] first source of each batch handed back to the host
    uint32_t redo_count;
    uint32_t max_nlev;      // deepest level count among the batches that completed
    uint32_t need_wide;     // a handed-back batch needs uint64 counts
    uint32_t deep;          // a handed-back batch went past the captured depth
    uint32_t arrived;       // blocks of the current batch check that have finished
};

// State of the batched sparse form (per-level frontier bitmaps).
struct SparseState {
    int32_t batch = 0;        // sources per batch: 64, 128, 256 or 512
    int32_t words = 0;        // batch / 64 bitmap words per vertex
    int32_t level_cap = 0;    // levels the front array can hold
    int32_t split = 256;      // rows longer than this are split into segments
    uint64_t *front = nullptr;   // [level_cap][n][words]
    uint32_t *any = nullptr;     // [level_cap][(n+31)/32] OR over sources, per vertex
    unsigned long long *lvmax = nullptr; // [level_cap] largest count at each level (for limb counts)
    uint64_t *visited = nullptr; // [n][words]
    uint64_t *sigma = nullptr;   // [n][batch] as uint64, or uint32 in its first half
    float *cval = nullptr;       // [n][batch]  c(v) = (1 + delta(v)) / sigma(v)
    int32_t *src = nullptr;      // [batch] sources of the current batch (-1 = empty lane)
    unsigned long long *reach = nullptr; // [0] the batch's sources' component sizes summed,
                                         // [1] (vertex, source) pairs reached so far
    uint32_t *any_host = nullptr; // pinned mirror of any, read once per batch
    int32_t *heavy_id = nullptr; // [n] index among heavy rows or -1
    int32_t *heavy_nseg = nullptr; // [nheavy] segments per heavy row
    uint32_t *arrive = nullptr;  // [nheavy] segment arrival counters (per row)
    uint32_t *arrive_w = nullptr;// [nheavy][words] segment arrival counters (per row and word)
    bool bwd_per_word = true;    // backward: one wave per (row, word) instead of per row
    int32_t bwd_grid = 0;        // per-word backward: blocks per launch (0 = one wave per item)
    int32_t fwd_grid = 0;        // forward pull: blocks per launch (0 = one wave per row or segment)
    int32_t depth_guess = 8;     // forward levels launched before the first check
    int32_t depth_max = 0;       // most levels any batch of this state has had (0: none run yet)
    bool wide = false;           // counts need uint64 storage (else uint32)
    uint32_t *lvflag = nullptr;  // [level_cap] non-zero iff the level holds a vertex for some source
    // replayed batches (unit weights): graphs of one batch's launches, the
    // control block, the handed-back list and what the graphs were made for
    BatchCtl *ctl = nullptr;
    int32_t *redo = nullptr;
    int64_t redo_cap = 0;
    hipStream_t cap_stream = nullptr;  // private stream the batch is captured on
    hipGraphExec_t gexec = nullptr;    // the recorded batch
    int32_t g_levels = 0;              // forward levels the graph holds
    bool g_wide = false;
    const void *g_front = nullptr;     // state pointers the graph was recorded with
    std::vector<uint8_t> g_plan;       // per level: bit 0 forward by products, bit 1 backward
    bool g_pending = false;            // replays whose checks the host has not read
    int32_t *seg_v = nullptr, *seg_beg = nullptr, *seg_end = nullptr; // [nseg]
    int32_t nheavy = 0, nseg = 0;
    double *hacc = nullptr;      // [nheavy][batch] partial sums of split rows (u64 or f64)
};

// State of the algebraic form (products with the adjacency matrix on MFMA).
struct AlgebraicState {
    int32_t npad = 0;                  // n rounded up to 256 (the product's row block)
    int32_t classes = 1;               // M: one 0/1 matrix per integer weight 1..M
    uint32_t *abits = nullptr;         // [M npad / 128][npad][4] 0/1 bits in panels of 128 columns, class c in columns [(c-1) npad, c npad)
    uint32_t *abits8 = nullptr;        // the same bits in the int8 operand order (forward products)
    __bf16 *planes = nullptr;          // up to 8 planes of [M npad/8][batch][8]
    uint64_t *part = nullptr;          // [npad][batch] partial limb sums
    uint32_t *kflags = nullptr;        // [M npad/32][batch/128] non-empty k-tiles
    unsigned long long *planes_issued = nullptr; // products issued (limb or coefficient planes)
    int32_t ksplit = 1;                // forward products: blocks per output tile, each over a share of K
    int32_t fwd_rows = 128;            // forward products: rows per block, 128 or 256 (tuned)
    float *ws = nullptr;               // [8 limbs][tiles][2 halves][64][256] partial sums of split tiles
    uint32_t *arrive = nullptr;        // [8 limbs][tiles] halves arrived
    bool every_level = false;          // the algebraic form: every level l >= 1 by products
};

// Per-level record of batches run while a probe is attached: the GPU time of
// each level's work and the level's union-frontier density.
struct LevelProbe {
    int mode = 0; // 0: follow the thresholds; 1: every level by CSR pulls;
                  // 2: every level >= 1 by products with A
    struct Rec {
        bool forward;
        int32_t level;
        double density;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs; // whoever attached the probe returns the events to the pool
};

// Hybrid form: each level l >= 1 goes by CSR pulls or by products with the
// adjacency matrix, chosen per batch from the union-frontier density of the
// level (the fraction of vertices at level l for at least one source of the
// batch) against thresholds fixed at create time.
struct HybridState {
    bool products = false;   // the adjacency bits exist and levels may use products
    double theta_fwd = 2.0;  // forward l -> l+1 by products when density(l) >= theta_fwd
    double theta_bwd = 2.0;  // backward l by products when density(l) >= theta_bwd
    std::vector<double> prev_density; // level densities of the last batch: the forward
                                      // decides level l from them, so it need not wait
    int32_t tune_source = 0; // BC_TUNE_DEFAULT / BC_TUNE_MEASURED / BC_TUNE_CACHED
    LevelProbe *probe = nullptr;
};

// State of the weighted per-source form (bucketed shortest paths).
struct WeightedBuffers {
    int groups = 0;
    int64_t cap = 0;              // arena ring entries per workgroup (power of two)
    int32_t *dist = nullptr, *order = nullptr, *gstart = nullptr, *gdist = nullptr, *arena = nullptr;
    int32_t *bstart = nullptr, *bcount = nullptr, *pstart = nullptr;
    int32_t *imp_x = nullptr;     // improvement list of the current phase
    uint8_t *imp_c = nullptr;
    int32_t *dag_p = nullptr, *dag_s = nullptr, *dag_a = nullptr, *gdag = nullptr; // DAG arcs by phase
    int64_t icap = 0, dcap = 0;
    uint64_t *sigma = nullptr;
    double *acc = nullptr;
};
struct WeightedState {
    WeightedBuffers main;         // many workgroups, arena of max(4n, 2^16)
    WeightedBuffers big;          // few workgroups, arena of nnz (allocated on first need)
    uint32_t *next = nullptr;
    int32_t *retry = nullptr;     // rows whose live bins outgrew the main arena
    uint32_t *retry_count = nullptr;
    uint32_t *host = nullptr;     // pinned
    int64_t retry_cap = 0;
    int64_t retried = 0;
    int32_t arena_log2 = 0;       // requested main arena size (0 = default)
    int32_t grid = 0;             // requested workgroups (0 = default)
};

// State of a many-graph context (bc_create_many).
constexpr int MG_MAX_N = 4096; // largest graph a many-graph context takes
struct MultiState {
    int32_t ngraphs = 0, nunits = 0, chunk = 64, grid = 0;
    int32_t ncompact = 0;             // units [0, ncompact) go to the compact sweep first
    int32_t *voff = nullptr, *rpoff = nullptr, *rp = nullptr, *units = nullptr;
    int32_t *redo = nullptr;          // compact units handed back to the full sweep
    unsigned int *next = nullptr;     // queue counters: compact, full, redo; [3] = redo count
    std::vector<int32_t> h_voff;
    std::vector<int32_t> h_arcs;      // arcs of each graph
    std::vector<int32_t> h_order;     // graphs by n_g descending (stable)
    hipStream_t stream = nullptr;     // private stream the launch is captured on
    hipEvent_t ev = nullptr;
    hipGraphExec_t exec = nullptr;    // captured reset + persistent sweep
};

// State of the plain per-source form.
struct PlainState {
    int32_t grid = 0;         // requested workgroups (0 = default)
    int32_t groups = 0;       // persistent workgroups
    int32_t *dist = nullptr;  // [groups][n]
    uint64_t *sigma = nullptr;// [groups][n]
    double *acc = nullptr;    // [groups][n]
    int32_t *queue = nullptr; // [groups][n]
    int32_t *lev = nullptr;   // [groups][n + 2] level starts in the queue
    uint32_t *next = nullptr; // work counter
};

struct bc_ctx {
    // graph (host copy of the shape only)
    int32_t n = 0, nnz = 0;
    int32_t max_degree = 0;
    std::vector<int32_t> h_row_ptr; // host copy of the CSR offsets
    uint32_t max_weight = 1;
    bool weighted = false;

    // device, stream, memory
    int device = 0;
    hipStream_t stream = nullptr;
    bc_allocator alloc{};
    std::vector<std::pair<void *, size_t>> owned; // every device allocation
    int64_t device_bytes = 0;

    // internal numbering (null when it equals the caller's)
    int32_t *new_of_old = nullptr; // [n] internal id of caller vertex v
    double *bc_scratch = nullptr;  // [n] BC in the caller's order, for bc_read

    // device copies (internal numbering)
    int32_t *row_ptr = nullptr;
    int32_t *col = nullptr;
    int32_t *comp_size = nullptr;   // [n] vertices in each vertex's connected component
    uint8_t *weight = nullptr;       // weights as bytes (weighted graphs with max weight <= 255)
    double *bc = nullptr;
    double *eb = nullptr;            // [nnz] edge betweenness terms per internal arc (edges on)
    double *eb_scratch = nullptr;    // [nnz] caller-order staging for bc_read_edges
    int32_t *arc_fwd = nullptr;      // [nnz] internal arc of caller arc e = (u, x)
    int32_t *arc_rev = nullptr;      // [nnz] internal arc of (x, u)
    bool edges = false;
    uint32_t *status = nullptr;      // [0]: BC_DEV_* bits; [1]: a batch needs uint64 counts
    uint32_t *status_host = nullptr; // pinned
    int32_t *sources = nullptr;      // staging for bc_run
    int64_t sources_cap = 0;

    // forms
    bc_form form = BC_FORM_PLAIN_FP64;
    SparseState sp;
    AlgebraicState al;
    PlainState pl;
    WeightedState wt;
    MultiState mg;
    HybridState hy;
    bool many = false;

    // bookkeeping
    int64_t sources_run = 0;
    int32_t max_levels = 0;
    bool poisoned = false;
    bool overflow_seen = false;
    std::string err;

    bool host_driven = false;   // batched forms: no replayed batches (bc_options.host_driven)
    bool no_alloc = false;      // inside bc_read_sssp_noalloc: bc_dalloc refuses every request
    bool recording = false;     // launches are being recorded into a graph (no timing events)

    int32_t timing = 0;         // 0 off; k >= 1: events on the launches of one source batch in k
    int64_t timing_batches = 0; // batches begun since create / reset
    int64_t eager_batches = 0;  // of those, batches driven from the host (their launches counted)
    bool timing_sel = true;     // the current batch's launches carry events
    std::map<std::string, KernelTimer> timers;
    std::vector<hipEvent_t> event_pool; // timing events ready for reuse
};

// ---- helpers implemented in bc_api.cpp --------------------------------------
bc_status bc_fail(bc_ctx *ctx, bc_status s, const std::string &msg);
// Entry checks of every call on a context (poisoned, stream under capture),
// then sparse_settle.
bc_status bc_check_usable(bc_ctx *ctx);
// Calls that run sources without adding to BC save the device overflow flag
// and clear it, then read what they raised and put the saved value back.
bc_status bc_status_save(bc_ctx *ctx, uint32_t *before);
bc_status bc_status_restore(bc_ctx *ctx, uint32_t before, uint32_t *now);
bc_status bc_hip(bc_ctx *ctx, hipError_t e, const char *what);
void *bc_dalloc(bc_ctx *ctx, size_t bytes);
void bc_dfree(bc_ctx *ctx, void *p);
// Timing events from the context's pool (created without the system-scope
// fence: they only time work on the stream); nullptr if creation fails.
hipEvent_t bc_event_get(bc_ctx *ctx);
void bc_event_put(bc_ctx *ctx, hipEvent_t e);
// Returns every pending kernel-timer event to the pool and zeroes the timers.
void bc_timers_clear(bc_ctx *ctx);
// Records an event pair around a launch when timing is on and the current
// source batch is timed; every launch is counted.  bc_timing_batch marks the
// start of a batch: with timing = k > 1 every launch of one batch in k carries
// events, so per-launch averages keep every level's share.  Work outside
// batches is timed whenever timing is on.  A replayed batch carries no
// events; a timed batch is run host-driven (bc_timing_eager counts it), and
// bc_get_timing scales the host-driven batches' totals to all batches.
void bc_timing_batch(bc_ctx *ctx);
void bc_timing_eager(bc_ctx *ctx);
struct LaunchTimer {
    bc_ctx *ctx;
    const char *name;
    hipEvent_t a = nullptr, b = nullptr;
    LaunchTimer(bc_ctx *c, const char *nm);
    void done();
};

#define BC_HIP(ctx, expr)                                                         \
    do {                                                                          \
        hipError_t e__ = (expr);                                                  \
        if (e__ != hipSuccess) return bc_hip((ctx), e__, #expr);                  \
    } while (0)

// ---- numbering (common.hip) ------------------------------------------------------
bc_status map_ids_to_internal(bc_ctx *ctx, int32_t *ids, int64_t count);
bc_status fill_all_sources(bc_ctx *ctx, int32_t *ids, int64_t count); // ids[i] = i on the device
bc_status rows_to_caller_order_f64(bc_ctx *ctx, double *out, const double *in, int64_t rows);
bc_status rows_to_caller_order_i32(bc_ctx *ctx, int32_t *out, const int32_t *in, int64_t rows);
bc_status rows_to_caller_order_u64(bc_ctx *ctx, uint64_t *out, const uint64_t *in, int64_t rows);
// out[e] = eb[arc_fwd[e]] + eb[arc_rev[e]] for the caller's arcs
bc_status edges_to_caller_order(bc_ctx *ctx, double *out);

// ---- forms (kernels + launchers) ----------------------------------------------
bc_status plain_prepare(bc_ctx *ctx);
bc_status plain_run(bc_ctx *ctx, const int32_t *d_sources, int64_t count, bool accumulate,
                    double *delta_dump, int32_t *dist_dump, uint64_t *sigma_dump);

bc_status weighted_prepare(bc_ctx *ctx);
bc_status weighted_run(bc_ctx *ctx, const int32_t *d_sources, int64_t count, bool accumulate,
                       double *delta_dump, int32_t *dist_dump, uint64_t *sigma_dump);

bc_status multigraph_prepare(bc_ctx *ctx, const std::vector<int32_t> &voff, const std::vector<int32_t> &rpoff,
                             const std::vector<int32_t> &rp, int32_t chunk);
bc_status multigraph_run(bc_ctx *ctx);
// Rebuilds the work queue over `graphs` (ids in h_order's order; null = every
// graph) at `chunk` sources per unit; the next run records its launches anew.
bc_status multigraph_set_queue(bc_ctx *ctx, const std::vector<int32_t> *graphs, int32_t chunk);
// units: 3 * count int32 of device staging, or nullptr to allocate it
bc_status multigraph_dump(bc_ctx *ctx, const int32_t *h_sources, int32_t count, int32_t *dist_dump,
                          uint64_t *sigma_dump, double *delta_dump, int32_t *units = nullptr);

// ---- allocation-free readout (noalloc.hip) ----------------------------------------
// Looks up, once per device and with that device current, the address of the
// fixed staging array there (called when a context is created).
void noalloc_init_device(int device);
// That address, or nullptr if the lookup failed.
unsigned char *noalloc_scratch(int device);

bc_status sparse_prepare(bc_ctx *ctx, int32_t batch, int32_t split_degree);
bc_status algebraic_prepare(bc_ctx *ctx);
// Forward level l -> l+1 by products (front, counts, any and lvmax of level l+1).
bc_status algebraic_forward_level(bc_ctx *ctx, bool wide, int32_t l);
// Backward level l; `deeper` of the levels l+1 .. l+M exist, fnext = front[l+1].
// With gate = &lvflag[l] (replayed batches), an empty level l exits at once
// and level l+1 counts as existing only if gate[1] is set.
bc_status algebraic_backward_level(bc_ctx *ctx, bool wide, const uint64_t *fcur, const uint64_t *fnext,
                                   int32_t deeper, double *delta_dump, bool accumulate,
                                   const uint32_t *gate = nullptr);
int64_t algebraic_planes_issued(bc_ctx *ctx); // synchronises; -1 on a device error
// k-tiles the products multiplied and those a dense product would have;
// synchronises; false on a device error
bool algebraic_ktiles(bc_ctx *ctx, int64_t *run, int64_t *dense, int64_t *run_fwd, int64_t *dense_fwd);
void algebraic_reset_counters(bc_ctx *ctx);
bc_status sparse_release(bc_ctx *ctx);
bc_status algebraic_release(bc_ctx *ctx);
// One batch of at most sp.batch internal source ids (device memory) through
// the batched forms; accumulate = false leaves BC untouched.
bc_status sparse_batch(bc_ctx *ctx, const int32_t *d_sources, int32_t count, bool accumulate);
bc_status sparse_run(bc_ctx *ctx, const int32_t *d_sources, int64_t count);
// Reads back what replayed batches found and re-runs the batches they handed
// back (on the host-driven path); synchronises.  A no-op when nothing is
// pending.  Every entry point calls it before touching the context's state.
bc_status sparse_settle(bc_ctx *ctx);
// Destroys the recorded batch graphs and their capture stream; synchronises.
void sparse_graphs_release(bc_ctx *ctx);
// delta_dump = nullptr runs the forward only (distances and counts).
bc_status sparse_dump(bc_ctx *ctx, const int32_t *d_sources, int32_t count,
                      int32_t *dist_dump, uint64_t *sigma_dump, double *delta_dump);

// ---- sampled forward (sampled.hip) -------------------------------------------------
// Distances by Algorithm 1; host id arrays, already validated; writes
// count * n caller-order rows to out (host or device memory as out_on_device).
bc_status sampled_distances(bc_ctx *ctx, const int32_t *h_sources, int32_t count, const int32_t *h_sample,
                            int32_t nsample, int32_t limit, int32_t *out, bool out_on_device);

// ---- all pairs (allpairs.hip) ---------------------------------------------------
// BC of every vertex (internal order) by Algorithm 2 from all-pairs D and
// Lambda, which the form's own forward kernels fill; bc_internal: n doubles.
bc_status allpairs_bc(bc_ctx *ctx, double *bc_internal);

// ---- tuning (tune.cpp) ----------------------------------------------------------
// Prepares the sparse, hybrid or algebraic form: batch width, hybrid
// thresholds and forward block rows come from opt, from the tuning cache, or
// from timed calibration batches.
bc_status tune_prepare(bc_ctx *ctx, const bc_options &opt, bc_form form);
// Prepares bc_create_many's work queue; the sources per unit come from opt,
// from the tuning cache, or from timed launches over a sample of the graphs.
bc_status tune_many(bc_ctx *ctx, const bc_options &opt, const std::vector<int32_t> &voff,
                    const std::vector<int32_t> &rpoff, const std::vector<int32_t> &rp);
