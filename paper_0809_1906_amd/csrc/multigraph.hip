// Many small graphs in one persistent launch.
//
// A context built by bc_create_many holds up to millions of small unweighted
// graphs (each with at most MG_MAX_N vertices) concatenated: vertex v of graph
// g has global id voff[g] + v, and BC is returned in that numbering.  bc_run
// computes all-source BC of every graph (Brandes's algorithm, Sec. 1.1, per
// graph).
//
// The work is a device queue of units (graph, [s0, s1) of its sources) sorted
// by n_g^2 descending, largest first (longest-processing-time order).  A grid
// of persistent 512-thread workgroups pulls units with an atomic counter and
// exits when the queue is drained.  For each source the workgroup runs the
// level-synchronous forward sweep (distance, exact uint64 counts) and the
// backward sweep (c(v) = (1 + delta(v)) / lambda(v) in FP32, sums in FP64)
// entirely in LDS; each unit's dependencies are summed in an FP64 LDS vector
// and added to BC once per unit.  The unit's columns are staged in LDS as
// 16-bit local ids when they fit (n <= 4096), so that a level step waits on
// LDS only; larger graphs read them from global memory.
//
// The level steps are latency-bound, so a compact sweep runs first with two
// workgroups per compute unit.  Each takes under half of the LDS:
// - 16-bit distances;
// - 32-bit counts, each overwritten by c(v) in the backward once v's own
//   dependency is known;
// - at most LEVCAP levels;
// - 16-bit row offsets and columns read through the caches.
// It takes the graphs with at most 65535 arcs. A unit whose counts pass 2^32
// - 1 or whose depth passes LEVCAP drops its partial sums and is handed to the
// full sweep. The launches (counter reset, compact sweep, full sweep over the
// remaining graphs, full sweep over the handed-back units) are captured once
// into a HIP graph and replayed.
#include "bc_internal.h"

#include <algorithm>

namespace {

constexpr int MT = 512;          // threads per workgroup
constexpr int32_t MG_INF = 0x7FFFFFFF;
constexpr int ABURST = 8;        // column reads issued together per vertex
constexpr int32_t COL_CAP = 16320; // 16-bit columns staged in LDS
constexpr int LEVCAP = 1024;       // levels per source in the compact sweep
constexpr uint32_t D16_INF = 0xFFFF;

struct MultiArgs {
    const int32_t *voff;   // [ngraphs+1] first global vertex of each graph
    const int32_t *rpoff;  // [ngraphs] where graph g's row offsets start in rp
    const int32_t *rp;     // concatenated per-graph row offsets (global arc indices)
    const int32_t *col;    // concatenated arcs, local vertex ids
    const int32_t *units;  // [nunits][3] = (graph, s0, s1), local source ids
    int32_t nunits;
    const unsigned int *nunits_dev; // if set, the unit count is read here instead
    unsigned int *next;    // queue counter
    int32_t *redo;         // compact sweep: units handed to the full sweep
    unsigned int *redo_count;
    double *bc;            // [sum n]
    uint32_t *status;
    // per-source readout (bc_read_sssp): unit u covers one source, row u
    int32_t dump_n;        // sum n (row length); 0 = no readout
    int32_t *dist_dump;
    uint64_t *sigma_dump;
    double *delta_dump;
};

__global__ void k_mg_reset(unsigned int *next) {
    if (threadIdx.x < 4) next[threadIdx.x] = 0;
}

struct MgShared {
    int32_t dist[MG_MAX_N];
    unsigned long long sig[MG_MAX_N];
    float c[MG_MAX_N];
    uint16_t queue[MG_MAX_N];
    uint16_t lev[MG_MAX_N + 2];
    double bc[MG_MAX_N];
    int32_t rp[MG_MAX_N + 1]; // the unit's graph: row offsets relative to its first arc
    uint16_t col[COL_CAP];    // the unit's columns, when they fit
    int32_t unit, cnt[3];
    uint32_t ovf;
};

// The sources [s0, s1) of unit u; columns from LDS (LC) or global memory.
template <bool LC>
__device__ __forceinline__ void mg_unit(const MultiArgs &a, MgShared &sh, int32_t u, int32_t n, int32_t vo,
                                        const int32_t *gcol, int32_t s0, int32_t s1) {
    int32_t *s_dist = sh.dist;
    unsigned long long *s_sig = sh.sig;
    float *s_c = sh.c;
    uint16_t *s_queue = sh.queue, *s_lev = sh.lev;
    double *s_bc = sh.bc;
    const int32_t *s_rp = sh.rp;
    int32_t *s_cnt = sh.cnt;
    const int tid = threadIdx.x;
    auto col = [&](int32_t e) -> int32_t { return LC ? (int32_t)sh.col[e] : gcol[e]; };
        for (int32_t s = s0; s < s1; ++s) {
            for (int32_t v = tid; v < n; v += MT) {
                s_dist[v] = v == s ? 0 : MG_INF;
                s_sig[v] = v == s ? 1ull : 0ull;
            }
            if (tid == 0) {
                s_queue[0] = (uint16_t)s;
                s_lev[0] = 0;
                s_lev[1] = 1;
                s_cnt[0] = 0;
                s_cnt[1] = 0;
                s_cnt[2] = 0;
            }
            __syncthreads();
            // forward: level L spans queue[qb, qe); appends of level L go to
            // queue[qe + s_cnt[L % 3]].  Three counters let one barrier per
            // level suffice: while level L appends to s_cnt[L % 3], thread 0
            // clears s_cnt[(L + 1) % 3], last read before the previous barrier.
            int32_t qb = 0, qe = 1, L = 0;
            while (qb < qe) {
                const int cur = L % 3;
                if (tid == 0) s_cnt[(L + 1) % 3] = 0;
                for (int32_t i = qb + tid; i < qe; i += MT) {
                    const int32_t v = s_queue[i];
                    const unsigned long long sv = s_sig[v];
                    const int32_t rb = s_rp[v], re = s_rp[v + 1];
                    for (int32_t e0 = rb; e0 < re; e0 += ABURST) {
                        int32_t ws[ABURST]; // one burst of column reads in flight
#pragma unroll
                        for (int j = 0; j < ABURST; ++j) ws[j] = e0 + j < re ? col(e0 + j) : -1;
#pragma unroll
                        for (int j = 0; j < ABURST; ++j) {
                            const int32_t w = ws[j];
                            if (w < 0) continue;
                            int32_t dw = s_dist[w];
                            if (dw == MG_INF) {
                                const int32_t old = atomicCAS(&s_dist[w], MG_INF, L + 1);
                                if (old == MG_INF) {
                                    s_queue[qe + atomicAdd(&s_cnt[cur], 1)] = (uint16_t)w;
                                    dw = L + 1;
                                } else {
                                    dw = old;
                                }
                            }
                            if (dw == L + 1) { // v in P_s(w)
                                const unsigned long long old = atomicAdd(&s_sig[w], sv);
                                if (old + sv < old) sh.ovf = 1;
                            }
                        }
                    }
                }
                __syncthreads();
                qb = qe;
                qe += s_cnt[cur];
                ++L;
                if (tid == 0) s_lev[L + 1] = (uint16_t)qe;
            }
            __syncthreads();
            const int32_t nlev = L;
            // backward: deepest level first; one thread per vertex, no atomics
            const int32_t lowest = a.dump_n ? 0 : 1;
            for (int32_t l = nlev - 1; l >= lowest; --l) {
                for (int32_t i = s_lev[l] + tid; i < s_lev[l + 1]; i += MT) {
                    const int32_t v = s_queue[i];
                    double acc = 0.0;
                    if (l + 1 < nlev) {
                        const int32_t rb = s_rp[v], re = s_rp[v + 1];
                        for (int32_t e0 = rb; e0 < re; e0 += ABURST) {
                            int32_t ws[ABURST];
#pragma unroll
                            for (int j = 0; j < ABURST; ++j) ws[j] = e0 + j < re ? col(e0 + j) : -1;
#pragma unroll
                            for (int j = 0; j < ABURST; ++j)
                                if (ws[j] >= 0 && s_dist[ws[j]] == l + 1) acc += (double)s_c[ws[j]];
                        }
                    }
                    const double sv = (double)s_sig[v];
                    const double dl = sv * acc;
                    s_c[v] = (float)((1.0 + dl) / sv);
                    if (v != s) s_bc[v] += dl;
                    if (a.dump_n) a.delta_dump[(size_t)u * a.dump_n + vo + v] = dl;
                }
                __syncthreads();
            }
            if (a.dump_n) {
                for (int32_t v = tid; v < n; v += MT) {
                    const int32_t d = s_dist[v];
                    a.dist_dump[(size_t)u * a.dump_n + vo + v] = d == MG_INF ? -1 : d;
                    a.sigma_dump[(size_t)u * a.dump_n + vo + v] = d == MG_INF ? 0 : s_sig[v];
                    if (d == MG_INF) a.delta_dump[(size_t)u * a.dump_n + vo + v] = 0.0;
                }
            }
            __syncthreads();
        }
}

__global__ __launch_bounds__(MT) void k_mg_sweep(MultiArgs a) {
    __shared__ MgShared sh;
    const int tid = threadIdx.x;
    const int32_t nunits = a.nunits_dev ? (int32_t)*a.nunits_dev : a.nunits;
    for (;;) {
        if (tid == 0) sh.unit = (int32_t)atomicAdd(a.next, 1u);
        __syncthreads();
        const int32_t u = sh.unit;
        if (u >= nunits) break;
        const int32_t g = a.units[3 * u], s0 = a.units[3 * u + 1], s1 = a.units[3 * u + 2];
        const int32_t vo = a.voff[g], n = a.voff[g + 1] - vo;
        const int32_t *grp = a.rp + a.rpoff[g];
        const int32_t *col = a.col + grp[0];
        const int32_t arcs = grp[n] - grp[0];
        const bool lds_col = arcs <= COL_CAP;
        for (int32_t v = tid; v <= n; v += MT) sh.rp[v] = grp[v] - grp[0];
        for (int32_t v = tid; v < n; v += MT) sh.bc[v] = 0.0;
        if (lds_col)
            for (int32_t e = tid; e < arcs; e += MT) sh.col[e] = (uint16_t)col[e];
        if (tid == 0) sh.ovf = 0;
        __syncthreads();
        if (lds_col) mg_unit<true>(a, sh, u, n, vo, col, s0, s1);
        else mg_unit<false>(a, sh, u, n, vo, col, s0, s1);
        if (!a.dump_n)
            for (int32_t v = tid; v < n; v += MT)
                if (sh.bc[v] != 0.0) unsafeAtomicAdd(&a.bc[vo + v], sh.bc[v]);
        if (tid == 0 && sh.ovf) atomicOr(a.status, (uint32_t)BC_DEV_SIGMA_OVERFLOW);
        __syncthreads();
    }
}

// ---- the compact sweep ------------------------------------------------------------

struct MgCompact {
    uint32_t dist2[MG_MAX_N / 2]; // two 16-bit distances per word, D16_INF = unreached
    uint32_t sc[MG_MAX_N];        // the count (uint32) in the forward; c(v) (float bits) after v's backward step
    uint16_t queue[MG_MAX_N];
    uint16_t lev[LEVCAP + 2];
    double bc[MG_MAX_N];
    uint16_t rp[MG_MAX_N + 1];    // row offsets relative to the graph's first arc
    int32_t unit, cnt[3];
    uint32_t fail;                // counts or depth out of range: the full sweep redoes the unit
};

__device__ __forceinline__ uint32_t d16_get(const uint32_t *d2, int32_t v) {
    return (d2[v >> 1] >> (16 * (v & 1))) & 0xFFFFu;
}

// Level of w, claiming it for level nl when it is unreached (*claimed says so).
__device__ __forceinline__ uint32_t d16_claim(uint32_t *d2, int32_t w, uint32_t nl, bool &claimed) {
    const int sh = 16 * (w & 1);
    uint32_t word = d2[w >> 1];
    for (;;) {
        const uint32_t cur = (word >> sh) & 0xFFFFu;
        if (cur != D16_INF) {
            claimed = false;
            return cur;
        }
        const uint32_t want = (word & ~(0xFFFFu << sh)) | (nl << sh);
        const uint32_t old = atomicCAS(&d2[w >> 1], word, want);
        if (old == word) {
            claimed = true;
            return nl;
        }
        word = old; // the other half changed, or another thread claimed w
    }
}

// The sources [s0, s1) of the unit in sh (graph of n vertices, columns col).
__device__ void mg_unit_compact(MgCompact &sh, int32_t n, const int32_t *__restrict__ col, int32_t s0, int32_t s1) {
    const int tid = threadIdx.x;
    for (int32_t s = s0; s < s1 && !sh.fail; ++s) {
        for (int32_t v = tid; v < (n + 1) / 2; v += MT) sh.dist2[v] = 0xFFFFFFFFu;
        for (int32_t v = tid; v < n; v += MT) sh.sc[v] = 0;
        __syncthreads();
        if (tid == 0) {
            sh.dist2[s >> 1] &= ~(0xFFFFu << (16 * (s & 1))); // level 0
            sh.sc[s] = 1;
            sh.queue[0] = (uint16_t)s;
            sh.lev[0] = 0;
            sh.lev[1] = 1;
            sh.cnt[0] = sh.cnt[1] = sh.cnt[2] = 0;
        }
        __syncthreads();
        // forward: as in the full sweep (three counters, one barrier per level)
        int32_t qb = 0, qe = 1, L = 0;
        while (qb < qe) {
            const int cur = L % 3;
            if (tid == 0) sh.cnt[(L + 1) % 3] = 0;
            for (int32_t i = qb + tid; i < qe; i += MT) {
                const int32_t v = sh.queue[i];
                const uint32_t sv = sh.sc[v];
                const int32_t rb = sh.rp[v], re = sh.rp[v + 1];
                for (int32_t e0 = rb; e0 < re; e0 += ABURST) {
                    int32_t ws[ABURST];
#pragma unroll
                    for (int j = 0; j < ABURST; ++j) ws[j] = e0 + j < re ? col[e0 + j] : -1;
#pragma unroll
                    for (int j = 0; j < ABURST; ++j) {
                        const int32_t w = ws[j];
                        if (w < 0) continue;
                        bool claimed = false;
                        const uint32_t dw = d16_claim(sh.dist2, w, (uint32_t)(L + 1), claimed);
                        if (claimed) sh.queue[qe + atomicAdd(&sh.cnt[cur], 1)] = (uint16_t)w;
                        if (dw == (uint32_t)(L + 1)) { // v in P_s(w)
                            const uint32_t old = atomicAdd(&sh.sc[w], sv);
                            if (old + sv < old) sh.fail = 1;
                        }
                    }
                }
            }
            __syncthreads();
            qb = qe;
            qe += sh.cnt[cur];
            ++L;
            if (L + 1 > LEVCAP) {
                if (tid == 0) sh.fail = 1;
                break;
            }
            if (tid == 0) sh.lev[L + 1] = (uint16_t)qe;
        }
        __syncthreads();
        if (sh.fail) break;
        const int32_t nlev = L;
        // backward: deepest level first; one thread per vertex; c(v) replaces
        // the count of v (read only by v's own thread, just before)
        for (int32_t l = nlev - 1; l >= 1; --l) {
            for (int32_t i = sh.lev[l] + tid; i < sh.lev[l + 1]; i += MT) {
                const int32_t v = sh.queue[i];
                double acc = 0.0;
                if (l + 1 < nlev) {
                    const int32_t rb = sh.rp[v], re = sh.rp[v + 1];
                    for (int32_t e0 = rb; e0 < re; e0 += ABURST) {
                        int32_t ws[ABURST];
#pragma unroll
                        for (int j = 0; j < ABURST; ++j) ws[j] = e0 + j < re ? col[e0 + j] : -1;
#pragma unroll
                        for (int j = 0; j < ABURST; ++j)
                            if (ws[j] >= 0 && d16_get(sh.dist2, ws[j]) == (uint32_t)(l + 1))
                                acc += (double)__uint_as_float(sh.sc[ws[j]]);
                    }
                }
                const double sv = (double)sh.sc[v];
                const double dl = sv * acc;
                sh.sc[v] = __float_as_uint((float)((1.0 + dl) / sv));
                if (v != s) sh.bc[v] += dl;
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(MT, 2) void k_mg_sweep_compact(MultiArgs a) {
    __shared__ MgCompact sh;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) sh.unit = (int32_t)atomicAdd(a.next, 1u);
        __syncthreads();
        const int32_t u = sh.unit;
        if (u >= a.nunits) break;
        const int32_t g = a.units[3 * u], s0 = a.units[3 * u + 1], s1 = a.units[3 * u + 2];
        const int32_t vo = a.voff[g], n = a.voff[g + 1] - vo;
        const int32_t *grp = a.rp + a.rpoff[g];
        for (int32_t v = tid; v <= n; v += MT) sh.rp[v] = (uint16_t)(grp[v] - grp[0]);
        for (int32_t v = tid; v < n; v += MT) sh.bc[v] = 0.0;
        if (tid == 0) sh.fail = 0;
        __syncthreads();
        mg_unit_compact(sh, n, a.col + grp[0], s0, s1);
        __syncthreads();
        if (!sh.fail) {
            for (int32_t v = tid; v < n; v += MT)
                if (sh.bc[v] != 0.0) unsafeAtomicAdd(&a.bc[vo + v], sh.bc[v]);
        } else if (tid == 0) {
            const unsigned int k = atomicAdd(a.redo_count, 1u);
            a.redo[3 * k] = g;
            a.redo[3 * k + 1] = s0;
            a.redo[3 * k + 2] = s1;
        }
        __syncthreads();
    }
}

// Fill for the per-source readout rows: vertices of other graphs are
// unreachable (-1, 0, 0).
__global__ __launch_bounds__(256) void k_mg_fill(int64_t cells, int32_t *dist, uint64_t *sigma, double *delta) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= cells) return;
    dist[i] = -1;
    sigma[i] = 0;
    delta[i] = 0.0;
}

MultiArgs args_of(bc_ctx *ctx, const int32_t *units, int32_t nunits) {
    MultiState &m = ctx->mg;
    MultiArgs a{};
    a.voff = m.voff;
    a.rpoff = m.rpoff;
    a.rp = m.rp;
    a.col = ctx->col;
    a.units = units;
    a.nunits = nunits;
    a.next = m.next;
    a.bc = ctx->bc;
    a.status = ctx->status;
    return a;
}

} // namespace

// Host side of bc_create_many: concatenated arrays and the LPT-ordered queue.
bc_status multigraph_prepare(bc_ctx *ctx, const std::vector<int32_t> &voff, const std::vector<int32_t> &rpoff,
                             const std::vector<int32_t> &rp, int32_t chunk) {
    MultiState &m = ctx->mg;
    const int32_t ng = (int32_t)voff.size() - 1;
    m.ngraphs = ng;
    m.h_voff = voff;
    m.h_arcs.assign((size_t)ng, 0);
    for (int32_t g = 0; g < ng; ++g) {
        const int32_t n = voff[g + 1] - voff[g];
        m.h_arcs[(size_t)g] = rp[(size_t)rpoff[(size_t)g] + n] - rp[(size_t)rpoff[(size_t)g]];
    }
    // graphs by n_g descending (stable: ties keep graph order)
    m.h_order.resize((size_t)ng);
    for (int32_t g = 0; g < ng; ++g) m.h_order[(size_t)g] = g;
    std::stable_sort(m.h_order.begin(), m.h_order.end(), [&](int32_t x, int32_t y) {
        return voff[x + 1] - voff[x] > voff[y + 1] - voff[y];
    });
    m.voff = (int32_t *)bc_dalloc(ctx, voff.size() * sizeof(int32_t));
    m.rpoff = (int32_t *)bc_dalloc(ctx, std::max<size_t>(rpoff.size(), 1) * sizeof(int32_t));
    m.rp = (int32_t *)bc_dalloc(ctx, std::max<size_t>(rp.size(), 1) * sizeof(int32_t));
    m.next = (unsigned int *)bc_dalloc(ctx, 256);
    if (!m.voff || !m.rpoff || !m.rp || !m.next) return bc_fail(ctx, BC_ERR_NOMEM, "many graphs: allocation failed");
    BC_HIP(ctx, hipMemcpy(m.voff, voff.data(), voff.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    if (!rpoff.empty())
        BC_HIP(ctx, hipMemcpy(m.rpoff, rpoff.data(), rpoff.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    if (!rp.empty()) BC_HIP(ctx, hipMemcpy(m.rp, rp.data(), rp.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    return multigraph_set_queue(ctx, nullptr, chunk > 0 ? chunk : 64);
}

// Units (graph, s0, s1) of `chunk` sources: the compact sweep's graphs (at
// most 65535 arcs) first, then the others, each group largest first.
bc_status multigraph_set_queue(bc_ctx *ctx, const std::vector<int32_t> *graphs, int32_t chunk) {
    MultiState &m = ctx->mg;
    const std::vector<int32_t> &order = graphs ? *graphs : m.h_order;
    std::vector<int32_t> units;
    int32_t ncompact = 0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int32_t g : order) {
            const int32_t n = m.h_voff[(size_t)g + 1] - m.h_voff[(size_t)g];
            if ((m.h_arcs[(size_t)g] <= 65535) != (pass == 0)) continue;
            for (int32_t s0 = 0; s0 < n; s0 += chunk) {
                units.push_back(g);
                units.push_back(s0);
                units.push_back(std::min(n, s0 + chunk));
            }
        }
        if (pass == 0) ncompact = (int32_t)(units.size() / 3);
    }
    if (m.exec) { // recorded with the old queue's addresses and sizes
        BC_HIP(ctx, hipStreamSynchronize(m.stream));
        BC_HIP(ctx, hipGraphExecDestroy(m.exec));
        m.exec = nullptr;
    }
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream)); // no launch still reads the old queue
    if (m.units) bc_dfree(ctx, m.units);
    if (m.redo) bc_dfree(ctx, m.redo);
    m.units = (int32_t *)bc_dalloc(ctx, std::max<size_t>(units.size(), 3) * sizeof(int32_t));
    m.redo = (int32_t *)bc_dalloc(ctx, (size_t)std::max(ncompact, 1) * 3 * sizeof(int32_t));
    if (!m.units || !m.redo) return bc_fail(ctx, BC_ERR_NOMEM, "many graphs: allocation failed");
    if (!units.empty())
        BC_HIP(ctx, hipMemcpy(m.units, units.data(), units.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    m.chunk = chunk;
    m.ncompact = ncompact;
    m.nunits = (int32_t)(units.size() / 3);
    int cus = 0;
    BC_HIP(ctx, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    m.grid = std::max(1, std::min(m.nunits, cus > 0 ? cus : 256));
    return BC_OK;
}

// All sources of every graph.  The first call records the launch into a HIP
// graph on the context's stream; later calls replay it.
bc_status multigraph_run(bc_ctx *ctx) {
    MultiState &m = ctx->mg;
    if (m.nunits == 0) return BC_OK;
    if (!m.exec) {
        // compact sweep, full sweep over the other graphs, full sweep over the
        // units the compact sweep handed back (its count read on the device)
        MultiArgs ac = args_of(ctx, m.units, m.ncompact);
        ac.next = m.next;
        ac.redo = m.redo;
        ac.redo_count = m.next + 3;
        MultiArgs af = args_of(ctx, m.units + (size_t)3 * m.ncompact, m.nunits - m.ncompact);
        af.next = m.next + 1;
        MultiArgs ar = args_of(ctx, m.redo, 0);
        ar.nunits_dev = m.next + 3;
        ar.next = m.next + 2;
        hipGraph_t graph = nullptr;
        BC_HIP(ctx, hipStreamBeginCapture(m.stream, hipStreamCaptureModeThreadLocal));
        hipLaunchKernelGGL(k_mg_reset, dim3(1), dim3(64), 0, m.stream, m.next);
        if (m.ncompact > 0)
            hipLaunchKernelGGL(k_mg_sweep_compact, dim3(std::min(m.ncompact, 2 * m.grid)), dim3(MT), 0, m.stream, ac);
        if (m.nunits > m.ncompact)
            hipLaunchKernelGGL(k_mg_sweep, dim3(std::min(m.nunits - m.ncompact, m.grid)), dim3(MT), 0, m.stream, af);
        if (m.ncompact > 0) hipLaunchKernelGGL(k_mg_sweep, dim3(m.grid), dim3(MT), 0, m.stream, ar);
        BC_HIP(ctx, hipStreamEndCapture(m.stream, &graph));
        const hipError_t e = hipGraphInstantiate(&m.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return bc_hip(ctx, e, "hipGraphInstantiate");
    }
    // order the private capture stream after prior work on the context stream
    BC_HIP(ctx, hipEventRecord(m.ev, ctx->stream));
    BC_HIP(ctx, hipStreamWaitEvent(m.stream, m.ev, 0));
    LaunchTimer t(ctx, "multigraph_sweep");
    BC_HIP(ctx, hipGraphLaunch(m.exec, m.stream));
    BC_HIP(ctx, hipEventRecord(m.ev, m.stream));
    BC_HIP(ctx, hipStreamWaitEvent(ctx->stream, m.ev, 0));
    t.done();
    return BC_OK;
}

// Per-source readout: global vertex ids of the concatenated numbering.
bc_status multigraph_dump(bc_ctx *ctx, const int32_t *h_sources, int32_t count, int32_t *dist_dump,
                          uint64_t *sigma_dump, double *delta_dump, int32_t *units_buf) {
    MultiState &m = ctx->mg;
    std::vector<int32_t> units((size_t)3 * count);
    for (int32_t i = 0; i < count; ++i) {
        const int32_t s = h_sources[i];
        const int32_t g = (int32_t)(std::upper_bound(m.h_voff.begin(), m.h_voff.end(), s) - m.h_voff.begin()) - 1;
        units[(size_t)3 * i] = g;
        units[(size_t)3 * i + 1] = s - m.h_voff[(size_t)g];
        units[(size_t)3 * i + 2] = s - m.h_voff[(size_t)g] + 1;
    }
    int32_t *du = units_buf ? units_buf : (int32_t *)bc_dalloc(ctx, units.size() * sizeof(int32_t));
    if (!du) return bc_fail(ctx, BC_ERR_NOMEM, "many graphs: readout allocation failed");
    BC_HIP(ctx, hipMemcpy(du, units.data(), units.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    const int64_t cells = (int64_t)count * ctx->n;
    hipLaunchKernelGGL(k_mg_fill, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, ctx->stream, cells, dist_dump,
                       sigma_dump, delta_dump);
    MultiArgs a = args_of(ctx, du, count);
    a.dump_n = ctx->n;
    a.dist_dump = dist_dump;
    a.sigma_dump = sigma_dump;
    a.delta_dump = delta_dump;
    hipLaunchKernelGGL(k_mg_reset, dim3(1), dim3(64), 0, ctx->stream, m.next);
    hipLaunchKernelGGL(k_mg_sweep, dim3(std::min(count, m.grid)), dim3(MT), 0, ctx->stream, a);
    BC_HIP(ctx, hipGetLastError());
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (!units_buf) bc_dfree(ctx, du);
    return BC_OK;
}
