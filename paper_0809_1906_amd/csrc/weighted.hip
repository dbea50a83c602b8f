// Weighted graphs (positive integer weights): one workgroup per source,
// bucketed shortest paths with one bucket per distance value (Dial's order).
//
// For each source s (Brandes's algorithm with weights, Sec. 1.1; the weighted
// forward of Sec. 3.2.1 read as path counts summed over P_s in nondecreasing
// distance):
//   forward   phase d = 0, 1, 2, ...: the vertices whose tentative distance is
//             d are final (every weight is >= 1).  They are settled, and one
//             pass over their arcs both pulls their counts over predecessors,
//                 lambda_sw = sum of lambda_sv over v with d(s,v) + w(v,w) = d,
//             and relaxes the arcs, from a single read of each neighbour's
//             distance.  A relaxation that improves x to d + c is listed, then
//             filed in bin c of phase d's slot in a ring of 256 slots (max
//             weight <= 255), so phase d + c finds it again by looking back
//             at most 255 phases: no priority queue.  Each thread keeps eight
//             arcs' loads in flight.
//   backward  distance groups from the farthest down to 1:
//             delta(v) = lambda_sv * sum over successors w
//             (d(s,w) = d(s,v) + w(v,w)) of c(w), c(w) = (1 + delta(w)) / lambda_sw,
//             and BC(v) += delta(v) for v != s (Theorem 1.1, FP64).  The
//             forward's count pull lists every DAG arc (predecessor,
//             successor) by phase, so the backward touches only those arcs (a
//             few percent of all arcs): once a group's c(w) are final, each is
//             added into its predecessors' sums.
//
// Weights above 255 are handled by the same ring with a wider window: the
// ring has W = 256 slots when max weight <= 255 and is refused otherwise
// (BC_ERR_UNSUPPORTED at create).
#include "bc_internal.h"
#include "wg_utils.h"

#include <algorithm>

namespace {

using wg::PB;
constexpr int RING = 256;        // phases kept in the ring (max weight + 1)
constexpr int32_t INF = 0x7FFFFFFF;
constexpr int U = 8;             // arcs per thread with loads in flight together
// Distances of the vertices [0, KH) live in LDS: with degree-ordered internal
// numbering they are the highest-degree vertices, which most arcs point to
// (RMAT-20: 45% of all arcs point into the first 8192), so those random reads
// and minimum updates stay on the compute unit.  The workgroup owns its
// source's distances, so the LDS copy is the only one.  32 KB: four
// workgroups still share a compute unit.
constexpr int32_t KH = 8192;

struct WeightedWork {
    int32_t *dist;   // [groups][n]
    uint64_t *sigma; // [groups][n]
    double *acc;     // [groups][n]
    int32_t *order;  // [groups][n]   settled vertices, nondecreasing distance
    int32_t *gstart; // [groups][n+1] distance groups in order[]
    int32_t *gdist;  // [groups][n]
    int32_t *arena;  // [groups][cap] ring of relaxed vertices, binned per (phase, weight)
    int32_t *bstart; // [groups][RING][RING] unwrapped arena position of each bin
    int32_t *bcount; // [groups][RING][RING]
    int32_t *pstart; // [groups][RING] unwrapped arena position of each phase's bins
    int32_t *imp_x;  // [groups][icap] vertices improved in the current phase
    uint8_t *imp_c;  // [groups][icap] the weight of the improving arc
    int32_t *dag_p;  // [groups][dcap] DAG arcs in phase order: predecessor,
    int32_t *dag_s;  // [groups][dcap]                         successor
    int32_t *dag_a;  // [groups][dcap]                         and arc index
    int32_t *gdag;   // [groups][n+1] first DAG arc of each distance group
    int64_t cap;     // arena entries per workgroup, a power of two
    int64_t icap;    // improvement-list entries per workgroup
    int64_t dcap;    // DAG-arc entries per workgroup
    int32_t *retry;  // sources (positions in the source list) whose live bins outgrew the arena
    uint32_t *retry_count;
    const int32_t *comp_size; // [n] vertices in each vertex's connected component
};

__global__ __launch_bounds__(PB) void k_weighted_sweep(
    int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col, const uint8_t *__restrict__ wt,
    const int32_t *__restrict__ sources, const int32_t *__restrict__ slot_of, int64_t count,
    unsigned long long *next_counter, WeightedWork W, double *bc, uint32_t *status, int accumulate,
    double *delta_dump, int32_t *dist_dump, uint64_t *sigma_dump, double *eb) {
    __shared__ wg::Chunk ch;
    __shared__ int32_t s_len[PB + 1];
    __shared__ int32_t s_st[PB];
    __shared__ int32_t s_hist[RING];
    __shared__ int32_t s_cur[RING];
    __shared__ long long s_idx;
    __shared__ int32_t s_nset, s_maxt, s_nimp, s_ndag;
    __shared__ uint32_t s_ovf, s_abort;
    __shared__ int32_t s_top;
    __shared__ int32_t s_hd[KH]; // dist[v] for v < KH

    const int tid = threadIdx.x;
    const size_t g = blockIdx.x;
    int32_t *dist = W.dist + g * (size_t)n;
    uint64_t *sigma = W.sigma + g * (size_t)n;
    double *acc = W.acc + g * (size_t)n;
    int32_t *order = W.order + g * (size_t)n;
    int32_t *gstart = W.gstart + g * ((size_t)n + 1);
    int32_t *gdist = W.gdist + g * (size_t)n;
    int32_t *arena = W.arena + g * (size_t)W.cap;
    int32_t *bstart = W.bstart + g * (size_t)RING * RING;
    int32_t *bcount = W.bcount + g * (size_t)RING * RING;
    int32_t *pstart = W.pstart + g * (size_t)RING;
    int32_t *imp_x = W.imp_x + g * (size_t)W.icap;
    uint8_t *imp_c = W.imp_c + g * (size_t)W.icap;
    int32_t *dag_p = W.dag_p + g * (size_t)W.dcap;
    int32_t *dag_s = W.dag_s + g * (size_t)W.dcap;
    int32_t *dag_a = W.dag_a + g * (size_t)W.dcap;
    int32_t *gdag = W.gdag + g * ((size_t)n + 1);
    const int32_t cmask = (int32_t)(W.cap - 1);
    auto dget = [&](int32_t v) -> int32_t { return v < KH ? s_hd[v] : dist[v]; };
    auto dmin = [&](int32_t v, int32_t x) -> int32_t { return v < KH ? atomicMin(&s_hd[v], x) : atomicMin(&dist[v], x); };

    for (;;) {
        if (tid == 0) s_idx = (long long)atomicAdd(next_counter, 1ull);
        __syncthreads();
        const long long idx = s_idx;
        if (idx >= count) break;
        const int32_t s = sources[idx];
        const size_t out = slot_of ? (size_t)slot_of[idx] : (size_t)idx; // row of the per-source outputs
        for (int32_t v = tid; v < n; v += PB) {
            if (v < KH) s_hd[v] = INF;
            else dist[v] = INF;
            sigma[v] = 0;
            acc[v] = 0.0;
        }
        wg::bar();
        if (tid == 0) {
            if (s < KH) s_hd[s] = 0;
            else dist[s] = 0;
            sigma[s] = 1;
            s_maxt = 0;
            s_ovf = 0;
            s_abort = 0;
            s_top = 0;
            s_ndag = 0;
        }
        wg::bar();

        // ---- forward: phases in nondecreasing distance ----
        int32_t nsettled = 0, ngroups = 0;
        for (int32_t d = 0; d <= s_maxt; ++d) {
            const int slot = d & (RING - 1);
            // (1) settle: candidates filed for distance d by phases d-255 .. d-1
            if (tid == 0) s_nset = 0;
            int32_t len = 0, st = 0;
            if (tid >= 1 && tid < RING && d - tid >= 0) {
                const int ps = (d - tid) & (RING - 1);
                len = bcount[ps * RING + tid];
                st = bstart[ps * RING + tid];
            }
            int tot;
            const int off = wg::block_excl_scan(len, ch.wsum, &tot);
            s_len[tid] = off;
            s_st[tid] = st;
            if (tid == 0) s_len[PB] = tot;
            __syncthreads();
            if (d == 0) {
                if (tid == 0) {
                    order[0] = s;
                    s_nset = 1;
                }
            } else {
                for (int i = tid; i < tot; i += PB) {
                    const int k = wg::owner(s_len, i);
                    const int32_t w = arena[(s_st[k] + (i - s_len[k])) & cmask];
                    if (dget(w) == d) order[nsettled + atomicAdd(&s_nset, 1)] = w;
                }
            }
            wg::bar();
            const int32_t cnt = s_nset;
            if (cnt == 0) {
                if (tid < RING) bcount[slot * RING + tid] = 0;
                if (tid == 0) pstart[slot] = s_top;
                wg::bar();
                continue;
            }
            const int32_t lb = nsettled, le = nsettled + cnt;
            if (tid == 0) {
                gstart[ngroups] = lb;
                gdist[ngroups] = d;
                gdag[ngroups] = s_ndag;
            }
            nsettled = le;
            ++ngroups;
            // (2) one pass over the settled vertices' arcs: pull each count
            // from its predecessors (all settled at smaller distances) and
            // relax, listing the improvements
            if (tid < RING) s_hist[tid] = 0;
            if (tid == 0) s_nimp = 0;
            __syncthreads();
            for (int32_t cb = lb; cb < le; cb += PB) {
                const int tot = wg::stage_chunk(order, cb, le, rp, ch);
                for (int e0 = tid; e0 < tot; e0 += PB * U) {
                    int k[U];
                    int32_t a[U], x[U], c[U], dx[U];
                    wg::arc_burst<U>(ch, e0, tot, k, a);
#pragma unroll
                    for (int j = 0; j < U; ++j) {
                        x[j] = a[j] >= 0 ? col[a[j]] : 0;
                        c[j] = a[j] >= 0 ? (int32_t)wt[a[j]] : 0;
                    }
#pragma unroll
                    for (int j = 0; j < U; ++j) dx[j] = a[j] >= 0 ? dget(x[j]) : INF;
#pragma unroll
                    for (int j = 0; j < U; ++j) {
                        if (a[j] < 0) continue;
                        if (d > 0 && dx[j] != INF && dx[j] + c[j] == d) { // x in P_s(w)
                            const int32_t w = ch.v[k[j]];
                            const uint64_t sx = sigma[x[j]];
                            const uint64_t old = atomicAdd((unsigned long long *)&sigma[w], (unsigned long long)sx);
                            if (old + sx < old) s_ovf = 1;
                            const int32_t pos = atomicAdd(&s_ndag, 1);
                            if (pos < W.dcap) {
                                dag_p[pos] = x[j];
                                dag_s[pos] = w;
                                dag_a[pos] = a[j];
                            } else {
                                s_abort = 1;
                            }
                        }
                        const int32_t nd = d + c[j];
                        if (nd < dx[j]) {
                            const int32_t old = dmin(x[j], nd);
                            if (nd < old) {
                                const int32_t pos = atomicAdd(&s_nimp, 1);
                                if (pos < W.icap) {
                                    imp_x[pos] = x[j];
                                    imp_c[pos] = (uint8_t)c[j];
                                    atomicAdd(&s_hist[c[j]], 1);
                                    atomicMax(&s_maxt, nd);
                                } else {
                                    s_abort = 1;
                                }
                            }
                        }
                    }
                }
                __syncthreads(); // the chunk's LDS is restaged
            }
            wg::bar();
            if (s_abort) break;
            // Every vertex of the source's component is settled: the bins hold
            // only stale candidates, so no later phase settles anything (each
            // phase writes its ring slot before any phase reads it, so the
            // next source does not see what is left).
            if (nsettled == W.comp_size[s]) break;
            // (3) allocate this phase's bins in the arena ring; the live window
            // (phases d-255 .. d) must fit, else the source is retried later
            {
                const int32_t h = tid < RING ? s_hist[tid] : 0;
                int total;
                const int pre = wg::block_excl_scan(h, ch.wsum, &total);
                const int32_t oldest = d >= RING - 1 ? pstart[(d - (RING - 1)) & (RING - 1)] : 0;
                if ((int64_t)s_top + total - oldest > W.cap) {
                    if (tid == 0) s_abort = 1;
                } else if (tid < RING) {
                    bstart[slot * RING + tid] = s_top + pre;
                    s_cur[tid] = 0;
                }
                __syncthreads();
                if (tid == 0 && !s_abort) {
                    pstart[slot] = s_top;
                    s_top += total;
                }
            }
            wg::bar();
            if (s_abort) break;
            // (4) file the listed improvements in their bins
            const int32_t nimp = s_nimp;
            for (int32_t i = tid; i < nimp; i += PB) {
                const int32_t x = imp_x[i], c = imp_c[i];
                const int kk = atomicAdd(&s_cur[c], 1);
                arena[(bstart[slot * RING + c] + kk) & cmask] = x;
            }
            __syncthreads();
            if (tid < RING) bcount[slot * RING + tid] = s_cur[tid];
            wg::bar();
        }
        if (s_abort) {
            if (tid == 0) W.retry[atomicAdd(W.retry_count, 1u)] = (int32_t)out;
            wg::bar();
            continue;
        }
        if (tid == 0) {
            gstart[ngroups] = nsettled;
            gdag[ngroups] = s_ndag;
        }
        wg::bar();

        // ---- backward: distance groups from the farthest down ----
        const int32_t lowest = accumulate ? 1 : 0;
        for (int32_t gi = ngroups - 1; gi >= lowest; --gi) {
            const int32_t lb = gstart[gi], le = gstart[gi + 1];
            // acc[v] holds the sum of c over v's successors, pushed by the
            // deeper groups
            for (int32_t i = lb + tid; i < le; i += PB) {
                const int32_t v = order[i];
                const double sv = (double)sigma[v];
                const double dl = sv * acc[v];
                if (accumulate && v != s) unsafeAtomicAdd(&bc[v], dl);
                if (delta_dump) delta_dump[out * n + v] = dl;
                acc[v] = (1.0 + dl) / sv;
            }
            wg::bar();
            // c(w) of this group into each predecessor's sum
            const int32_t db = gdag[gi], de = gdag[gi + 1];
            for (int32_t i0 = db + tid; i0 < de; i0 += PB * U) {
                int32_t p[U];
                double cw[U];
#pragma unroll
                for (int j = 0; j < U; ++j) {
                    const int32_t i = i0 + j * PB;
                    p[j] = i < de ? dag_p[i] : -1;
                    cw[j] = i < de ? acc[dag_s[i]] : 0.0;
                }
#pragma unroll
                for (int j = 0; j < U; ++j)
                    if (p[j] >= 0) {
                        unsafeAtomicAdd(&acc[p[j]], cw[j]);
                        // edge term of the DAG arc p -> w: lambda(p) c(w)
                        if (eb) unsafeAtomicAdd(&eb[dag_a[i0 + j * PB]], (double)sigma[p[j]] * cw[j]);
                    }
            }
            wg::bar();
        }
        if (dist_dump) {
            for (int32_t v = tid; v < n; v += PB) {
                const int32_t dv = dget(v);
                dist_dump[out * n + v] = dv == INF ? -1 : dv;
                sigma_dump[out * n + v] = dv == INF ? 0 : sigma[v];
                if (dv == INF) delta_dump[out * n + v] = 0.0;
            }
        }
        if (tid == 0 && s_ovf) atomicOr(status, (uint32_t)BC_DEV_SIGMA_OVERFLOW);
        wg::bar();
    }
}

// Main workspaces list a quarter of the ring's size in improvements per phase
// and half of it in DAG arcs, and send a source that needs more to the retry
// workspace; the retry workspace (ring of nnz + 1 entries or more) holds every
// improvement of a phase and every DAG arc, so it never needs a retry itself.
int64_t imp_cap(int64_t cap, bool retry_ws) { return retry_ws ? cap : std::max<int64_t>(cap / 4, 1); }
int64_t dag_cap(int64_t cap) { return std::max<int64_t>(cap / 2, 1); }

bc_status alloc_work(bc_ctx *ctx, WeightedBuffers &b, int64_t cap, int groups, bool retry_ws) {
    const size_t n = (size_t)std::max(ctx->n, 1);
    const size_t G = (size_t)groups;
    b.groups = groups;
    b.cap = cap;
    b.icap = imp_cap(cap, retry_ws);
    b.dcap = dag_cap(cap);
    b.dist = (int32_t *)bc_dalloc(ctx, G * n * 4);
    b.sigma = (uint64_t *)bc_dalloc(ctx, G * n * 8);
    b.acc = (double *)bc_dalloc(ctx, G * n * 8);
    b.order = (int32_t *)bc_dalloc(ctx, G * n * 4);
    b.gstart = (int32_t *)bc_dalloc(ctx, G * (n + 1) * 4);
    b.gdist = (int32_t *)bc_dalloc(ctx, G * n * 4);
    b.arena = (int32_t *)bc_dalloc(ctx, G * (size_t)cap * 4);
    b.bstart = (int32_t *)bc_dalloc(ctx, G * RING * RING * 4);
    b.bcount = (int32_t *)bc_dalloc(ctx, G * RING * RING * 4);
    b.pstart = (int32_t *)bc_dalloc(ctx, G * RING * 4);
    b.imp_x = (int32_t *)bc_dalloc(ctx, G * (size_t)b.icap * 4);
    b.imp_c = (uint8_t *)bc_dalloc(ctx, G * (size_t)b.icap);
    b.dag_p = (int32_t *)bc_dalloc(ctx, G * (size_t)b.dcap * 4);
    b.dag_s = (int32_t *)bc_dalloc(ctx, G * (size_t)b.dcap * 4);
    b.dag_a = (int32_t *)bc_dalloc(ctx, G * (size_t)b.dcap * 4);
    b.gdag = (int32_t *)bc_dalloc(ctx, G * (n + 1) * 4);
    if (!b.dist || !b.sigma || !b.acc || !b.order || !b.gstart || !b.gdist || !b.arena || !b.bstart || !b.bcount ||
        !b.pstart || !b.imp_x || !b.imp_c || !b.dag_p || !b.dag_s || !b.dag_a || !b.gdag)
        return bc_fail(ctx, BC_ERR_NOMEM, "weighted form: workspace allocation failed");
    return BC_OK;
}

size_t per_group_bytes(bc_ctx *ctx, int64_t cap, bool retry_ws) {
    const size_t n = (size_t)std::max(ctx->n, 1);
    // per vertex: dist, sigma, acc, order, gstart, gdist, gdag; the arena; the
    // improvement list (5 B per entry); the DAG list (12 B per arc); the bins
    return n * (4 + 8 + 8 + 4 + 4 + 4 + 4) + 8 + (size_t)cap * 4 + (size_t)imp_cap(cap, retry_ws) * 5 +
           (size_t)dag_cap(cap) * 12 + (2 * (size_t)RING + 1) * RING * 4;
}

int64_t pow2_at_least(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

WeightedWork work_of(bc_ctx *ctx, const WeightedBuffers &b) {
    WeightedState &w = ctx->wt;
    return WeightedWork{b.dist, b.sigma, b.acc, b.order, b.gstart, b.gdist, b.arena, b.bstart, b.bcount,
                        b.pstart, b.imp_x, b.imp_c, b.dag_p, b.dag_s, b.dag_a, b.gdag, b.cap, b.icap, b.dcap, w.retry,
                        w.retry_count, ctx->comp_size};
}

} // namespace

// Workgroups get an arena ring of max(4n, 2^16) entries (rounded up to a power
// of two); a source whose live bins outgrow it is re-run with an arena of nnz
// entries, which always suffices (a vertex settles once, so at most one entry
// per arc is ever filed).
bc_status weighted_prepare(bc_ctx *ctx) {
    WeightedState &w = ctx->wt;
    if (ctx->max_weight > 255)
        return bc_fail(ctx, BC_ERR_UNSUPPORTED, "weighted form: weights above 255 are not supported");
    const int64_t cap = w.arena_log2 > 0 ? (int64_t(1) << w.arena_log2)
                                         : pow2_at_least(std::max<int64_t>(4 * (int64_t)std::max(ctx->n, 1), 1 << 16));
    // workspace budget: 96 GB by default, 192 GB for an explicitly requested grid
    const size_t budget = size_t(w.grid > 0 ? 192 : 96) << 30;
    int groups = w.grid > 0 ? w.grid : 1024;
    while (groups > 1 && per_group_bytes(ctx, cap, false) * (size_t)groups > budget) groups /= 2;
    bc_status st = alloc_work(ctx, w.main, cap, groups, false);
    if (st != BC_OK) return st;
    w.next = (uint32_t *)bc_dalloc(ctx, 256);
    w.retry_count = (uint32_t *)bc_dalloc(ctx, 256);
    w.retry = (int32_t *)bc_dalloc(ctx, (size_t)4096 * 4);
    w.retry_cap = 4096;
    if (!w.next || !w.retry_count || !w.retry || hipHostMalloc((void **)&w.host, 256) != hipSuccess)
        return bc_fail(ctx, BC_ERR_NOMEM, "weighted form: allocation failed");
    return BC_OK;
}

static bc_status launch(bc_ctx *ctx, const WeightedBuffers &b, const int32_t *d_sources, const int32_t *slot_of,
                        int64_t count, bool accumulate, double *delta_dump, int32_t *dist_dump, uint64_t *sigma_dump) {
    WeightedState &w = ctx->wt;
    BC_HIP(ctx, hipMemsetAsync(w.next, 0, sizeof(unsigned long long), ctx->stream));
    const int grid = (int)std::min<int64_t>(count, b.groups);
    LaunchTimer t(ctx, "weighted_sweep");
    hipLaunchKernelGGL(k_weighted_sweep, dim3(grid), dim3(PB), 0, ctx->stream, ctx->n, ctx->row_ptr, ctx->col,
                       ctx->weight, d_sources, slot_of, count, (unsigned long long *)w.next, work_of(ctx, b),
                       ctx->bc, ctx->status, accumulate ? 1 : 0, delta_dump, dist_dump, sigma_dump,
                       accumulate && ctx->edges ? ctx->eb : nullptr);
    t.done();
    BC_HIP(ctx, hipGetLastError());
    return BC_OK;
}

bc_status weighted_run(bc_ctx *ctx, const int32_t *d_sources, int64_t count, bool accumulate,
                       double *delta_dump, int32_t *dist_dump, uint64_t *sigma_dump) {
    WeightedState &w = ctx->wt;
    // the retry list holds at most one entry per source in flight: run in chunks
    for (int64_t c0 = 0; c0 < count; c0 += w.retry_cap) {
        const int64_t cnt = std::min<int64_t>(w.retry_cap, count - c0);
        BC_HIP(ctx, hipMemsetAsync(w.retry_count, 0, sizeof(uint32_t), ctx->stream));
        // per-source output rows are positions in the whole list
        bc_status st = launch(ctx, w.main, d_sources + c0, nullptr, cnt, accumulate,
                              delta_dump ? delta_dump + (size_t)c0 * ctx->n : nullptr,
                              dist_dump ? dist_dump + (size_t)c0 * ctx->n : nullptr,
                              sigma_dump ? sigma_dump + (size_t)c0 * ctx->n : nullptr);
        if (st != BC_OK) return st;
        BC_HIP(ctx, hipMemcpyAsync(w.host, w.retry_count, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream));
        BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
        const uint32_t nretry = *w.host;
        if (nretry == 0) continue;
        if (!w.big.dist) {
            const int64_t cap = pow2_at_least((int64_t)std::max(ctx->nnz, 1) + 1);
            int groups = 64;
            while (groups > 1 && per_group_bytes(ctx, cap, true) * (size_t)groups > (size_t(16) << 30)) groups /= 2;
            st = alloc_work(ctx, w.big, cap, groups, true);
            if (st != BC_OK) return st;
        }
        // sources of the retried rows, gathered on the host
        std::vector<int32_t> rows(nretry), srcs(nretry);
        BC_HIP(ctx, hipMemcpy(rows.data(), w.retry, nretry * sizeof(int32_t), hipMemcpyDeviceToHost));
        std::vector<int32_t> all((size_t)cnt);
        BC_HIP(ctx, hipMemcpy(all.data(), d_sources + c0, (size_t)cnt * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (uint32_t i = 0; i < nretry; ++i) srcs[i] = all[(size_t)rows[i]];
        int32_t *dev = (int32_t *)bc_dalloc(ctx, 2 * (size_t)nretry * sizeof(int32_t));
        if (!dev) return bc_fail(ctx, BC_ERR_NOMEM, "weighted form: retry allocation failed");
        BC_HIP(ctx, hipMemcpy(dev, srcs.data(), nretry * sizeof(int32_t), hipMemcpyHostToDevice));
        BC_HIP(ctx, hipMemcpy(dev + nretry, rows.data(), nretry * sizeof(int32_t), hipMemcpyHostToDevice));
        BC_HIP(ctx, hipMemsetAsync(w.retry_count, 0, sizeof(uint32_t), ctx->stream));
        st = launch(ctx, w.big, dev, dev + nretry, nretry, accumulate,
                    delta_dump ? delta_dump + (size_t)c0 * ctx->n : nullptr,
                    dist_dump ? dist_dump + (size_t)c0 * ctx->n : nullptr,
                    sigma_dump ? sigma_dump + (size_t)c0 * ctx->n : nullptr);
        BC_HIP(ctx, hipMemcpyAsync(w.host, w.retry_count, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream));
        BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
        bc_dfree(ctx, dev);
        if (st != BC_OK) return st;
        if (*w.host != 0) // cannot happen: the retry workspace holds any source's lists
            return bc_fail(ctx, BC_ERR_DEVICE, "weighted form: a source outgrew the retry workspace");
        ctx->wt.retried += nretry;
    }
    return BC_OK;
}
