// Weighted graphs (positive integer weights): one workgroup per source,
// bucketed shortest paths with one bucket per distance value (Dial's order).
//
// For each source s (Brandes's algorithm with weights, Sec. 1.1; the weighted
// forward of Sec. 3.2.1 read as path counts summed over P_s in nondecreasing
// distance):
//   forward   phase d = 0, 1, 2, ...: the vertices whose tentative distance is
//             d are final (every weight is >= 1).  They are settled, their
//             count is pulled over predecessors,
//                 lambda_sw = sum of lambda_sv over v with d(s,v) + w(v,w) = d,
//             and their arcs are relaxed.  A relaxation that improves x to
//             d + c is filed in bin c of phase d's slot in a ring of 256
//             slots (max weight <= 255), so phase d + c finds it again by
//             looking back at most 255 phases: no priority queue.
//   backward  distance groups from the farthest down to 1:
//             delta(v) = lambda_sv * sum over successors w
//             (d(s,w) = d(s,v) + w(v,w)) of c(w), c(w) = (1 + delta(w)) / lambda_sw,
//             and BC(v) += delta(v) for v != s (Theorem 1.1, FP64).
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
    int64_t cap;     // arena entries per workgroup, a power of two
    int32_t *retry;  // sources (positions in the source list) whose live bins outgrew the arena
    uint32_t *retry_count;
};

__global__ __launch_bounds__(PB) void k_weighted_sweep(
    int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col, const uint32_t *__restrict__ wt,
    const int32_t *__restrict__ sources, const int32_t *__restrict__ slot_of, int64_t count,
    unsigned long long *next_counter, WeightedWork W, double *bc, uint32_t *status, int accumulate,
    double *delta_dump, int32_t *dist_dump, uint64_t *sigma_dump) {
    __shared__ wg::Chunk ch;
    __shared__ int32_t s_len[PB + 1];
    __shared__ int32_t s_st[PB];
    __shared__ int32_t s_hist[RING];
    __shared__ int32_t s_cur[RING];
    __shared__ long long s_idx;
    __shared__ int32_t s_nset, s_maxt;
    __shared__ uint32_t s_ovf, s_abort;
    __shared__ int32_t s_top;

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
    const int32_t cmask = (int32_t)(W.cap - 1);
    auto none = [](int, int32_t) {};

    for (;;) {
        if (tid == 0) s_idx = (long long)atomicAdd(next_counter, 1ull);
        __syncthreads();
        const long long idx = s_idx;
        if (idx >= count) break;
        const int32_t s = sources[idx];
        const size_t out = slot_of ? (size_t)slot_of[idx] : (size_t)idx; // row of the per-source outputs
        for (int32_t v = tid; v < n; v += PB) {
            dist[v] = INF;
            sigma[v] = 0;
            acc[v] = 0.0;
        }
        wg::bar();
        if (tid == 0) {
            dist[s] = 0;
            sigma[s] = 1;
            s_maxt = 0;
            s_ovf = 0;
            s_abort = 0;
            s_top = 0;
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
                    if (dist[w] == d) order[nsettled + atomicAdd(&s_nset, 1)] = w;
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
            }
            nsettled = le;
            ++ngroups;
            // (2) one pass over the settled vertices' arcs: pull counts from
            // predecessors (all settled at smaller distances) and count, per
            // weight, the relaxations that would improve a neighbour
            if (tid < RING) s_hist[tid] = 0;
            wg::bar();
            wg::for_arcs(order, lb, le, rp, ch, none, [&](int, int32_t w, int32_t a) {
                const int32_t v = col[a];
                const int32_t c = (int32_t)wt[a];
                const int32_t dv = dist[v];
                if (d > 0 && dv != INF && dv + c == d) {
                    const uint64_t x = sigma[v];
                    const uint64_t old = atomicAdd((unsigned long long *)&sigma[w], (unsigned long long)x);
                    if (old + x < old) s_ovf = 1;
                }
                if (d + c < dv) atomicAdd(&s_hist[c], 1);
            });
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
            wg::for_arcs(order, lb, le, rp, ch, none, [&](int, int32_t, int32_t a) {
                const int32_t x = col[a];
                const int32_t c = (int32_t)wt[a];
                const int32_t nd = d + c;
                if (nd < dist[x]) {
                    const int32_t old = atomicMin(&dist[x], nd);
                    if (nd < old) {
                        const int k = atomicAdd(&s_cur[c], 1);
                        arena[(bstart[slot * RING + c] + k) & cmask] = x;
                        atomicMax(&s_maxt, nd);
                    }
                }
            });
            if (tid < RING) bcount[slot * RING + tid] = s_cur[tid];
            wg::bar();
        }
        if (s_abort) {
            if (tid == 0) W.retry[atomicAdd(W.retry_count, 1u)] = (int32_t)out;
            wg::bar();
            continue;
        }
        if (tid == 0) gstart[ngroups] = nsettled;
        wg::bar();

        // ---- backward: distance groups from the farthest down ----
        const int32_t lowest = accumulate ? 1 : 0;
        for (int32_t gi = ngroups - 1; gi >= lowest; --gi) {
            const int32_t lb = gstart[gi], le = gstart[gi + 1], d = gdist[gi];
            if (gi < ngroups - 1) {
                wg::for_arcs(order, lb, le, rp, ch, none, [&](int, int32_t v, int32_t a) {
                    const int32_t w = col[a];
                    if (dist[w] != INF && dist[w] == d + (int32_t)wt[a]) unsafeAtomicAdd(&acc[v], acc[w]);
                });
            }
            for (int32_t i = lb + tid; i < le; i += PB) {
                const int32_t v = order[i];
                const double sv = (double)sigma[v];
                const double dl = sv * acc[v];
                if (accumulate && v != s) unsafeAtomicAdd(&bc[v], dl);
                if (delta_dump) delta_dump[out * n + v] = dl;
                acc[v] = (1.0 + dl) / sv;
            }
            wg::bar();
        }
        if (dist_dump) {
            for (int32_t v = tid; v < n; v += PB) {
                const int32_t dv = dist[v];
                dist_dump[out * n + v] = dv == INF ? -1 : dv;
                sigma_dump[out * n + v] = dv == INF ? 0 : sigma[v];
                if (dv == INF) delta_dump[out * n + v] = 0.0;
            }
        }
        if (tid == 0 && s_ovf) atomicOr(status, (uint32_t)BC_DEV_SIGMA_OVERFLOW);
        wg::bar();
    }
}

bc_status alloc_work(bc_ctx *ctx, WeightedBuffers &b, int64_t cap, int groups) {
    const size_t n = (size_t)std::max(ctx->n, 1);
    const size_t G = (size_t)groups;
    b.groups = groups;
    b.cap = cap;
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
    if (!b.dist || !b.sigma || !b.acc || !b.order || !b.gstart || !b.gdist || !b.arena || !b.bstart || !b.bcount ||
        !b.pstart)
        return bc_fail(ctx, BC_ERR_NOMEM, "weighted form: workspace allocation failed");
    return BC_OK;
}

size_t per_group_bytes(bc_ctx *ctx, int64_t cap) {
    const size_t n = (size_t)std::max(ctx->n, 1);
    return n * (4 + 8 + 8 + 4 + 4 + 4) + 4 + (size_t)cap * 4 + (2 * (size_t)RING + 1) * RING * 4;
}

int64_t pow2_at_least(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

WeightedWork work_of(bc_ctx *ctx, const WeightedBuffers &b) {
    WeightedState &w = ctx->wt;
    return WeightedWork{b.dist, b.sigma, b.acc, b.order, b.gstart, b.gdist, b.arena, b.bstart, b.bcount,
                        b.pstart, b.cap, w.retry, w.retry_count};
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
    const size_t budget = size_t(48) << 30;
    int groups = 1024;
    while (groups > 1 && per_group_bytes(ctx, cap) * (size_t)groups > budget) groups /= 2;
    bc_status st = alloc_work(ctx, w.main, cap, groups);
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
                       ctx->bc, ctx->status, accumulate ? 1 : 0, delta_dump, dist_dump, sigma_dump);
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
            while (groups > 1 && per_group_bytes(ctx, cap) * (size_t)groups > (size_t(16) << 30)) groups /= 2;
            st = alloc_work(ctx, w.big, cap, groups);
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
        BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
        bc_dfree(ctx, dev);
        if (st != BC_OK) return st;
        ctx->wt.retried += nretry;
    }
    return BC_OK;
}
