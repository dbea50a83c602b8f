// Plain FP64 form: one workgroup per source, per-source state in HBM.
//
// For each source s (Brandes's algorithm, Sec. 1.1):
//   forward   level-synchronous breadth-first search from s (the parallel BFS
//             of Sec. 4): a vertex w first reached from level l gets
//             d(s,w) = l+1, and every arc (v,w) with d(s,v) = l, d(s,w) = l+1
//             (v in P_s(w)) adds lambda_sv into lambda_sw;
//   backward  levels from the deepest down to 1: for v at level l,
//             delta_s*(v) = lambda_sv * sum over successors w of c(w), with
//             c(w) = (1 + delta_s*(w)) / lambda_sw -- Theorem 1.1 with the
//             factor lambda_sv taken out of the sum (the per-edge term of
//             ParallelCompute, Sec. 4.2.2);
//   score     BC(v) += delta_s*(v) for v != s.
//
// Each level's frontier is expanded in chunks of 256 vertices whose degree
// prefix sums are staged in LDS, so a thread takes arcs, not vertices: hub
// vertices are spread over the whole workgroup.  Each thread keeps eight
// arcs' loads in flight.
#include "bc_internal.h"
#include "wg_utils.h"

namespace {

using wg::PB;
constexpr int U = 8; // arcs per thread with loads in flight together

__global__ __launch_bounds__(PB) void k_plain_sweep(
    int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const int32_t *__restrict__ sources, int64_t count, unsigned long long *next_counter,
    int32_t *dist_all, uint64_t *sigma_all, double *acc_all, int32_t *queue_all, int32_t *lev_all,
    double *bc, uint32_t *status, int accumulate,
    double *delta_dump, int32_t *dist_dump, uint64_t *sigma_dump, double *eb) {
    __shared__ wg::Chunk ch;
    __shared__ int32_t s_tail;
    __shared__ long long s_idx;
    __shared__ uint32_t s_ovf;

    const int tid = threadIdx.x;
    const size_t g = blockIdx.x;
    int32_t *dist = dist_all + g * (size_t)n;
    uint64_t *sigma = sigma_all + g * (size_t)n;
    double *acc = acc_all + g * (size_t)n;
    int32_t *queue = queue_all + g * (size_t)n;
    int32_t *lev = lev_all + g * ((size_t)n + 2);

    for (;;) {
        if (tid == 0) s_idx = (long long)atomicAdd(next_counter, 1ull);
        __syncthreads();
        const long long idx = s_idx;
        if (idx >= count) break;
        const int32_t s = sources[idx];

        for (int32_t v = tid; v < n; v += PB) {
            dist[v] = -1;
            sigma[v] = 0;
            acc[v] = 0.0;
        }
        wg::bar();
        if (tid == 0) {
            dist[s] = 0;
            sigma[s] = 1;
            queue[0] = s;
            lev[0] = 0;
            lev[1] = 1;
            s_tail = 1;
            s_ovf = 0;
        }
        wg::bar();

        // ---- forward: level L spans queue[qb, qe) ----
        int32_t qb = 0, qe = 1, L = 0;
        while (qb < qe) {
            for (int32_t cb = qb; cb < qe; cb += PB) {
                const int tot = wg::stage_chunk(queue, cb, qe, rp, ch);
                for (int e0 = tid; e0 < tot; e0 += PB * U) {
                    int k[U];
                    int32_t a[U], w[U], dw[U];
                    wg::arc_burst<U>(ch, e0, tot, k, a);
#pragma unroll
                    for (int j = 0; j < U; ++j) w[j] = a[j] >= 0 ? col[a[j]] : 0;
#pragma unroll
                    for (int j = 0; j < U; ++j) dw[j] = a[j] >= 0 ? dist[w[j]] : 0;
#pragma unroll
                    for (int j = 0; j < U; ++j) {
                        if (a[j] < 0) continue;
                        int32_t d = dw[j];
                        if (d < 0) {
                            const int32_t old = atomicCAS(&dist[w[j]], -1, L + 1);
                            if (old == -1) {
                                queue[atomicAdd(&s_tail, 1)] = w[j];
                                d = L + 1;
                            } else {
                                d = old;
                            }
                        }
                        if (d == L + 1) { // v in P_s(w)
                            const uint64_t x = sigma[ch.v[k[j]]];
                            const uint64_t old = atomicAdd((unsigned long long *)&sigma[w[j]], (unsigned long long)x);
                            if (old + x < old) s_ovf = 1;
                        }
                    }
                }
                __syncthreads(); // the chunk's LDS is restaged
            }
            wg::bar();
            qb = qe;
            qe = s_tail;
            ++L;
            if (tid == 0) lev[L + 1] = qe;
            wg::bar();
        }
        const int32_t nlev = L; // non-empty levels 0..nlev-1

        // ---- backward: deepest level first ----
        // (level 0 adds nothing to BC, but its arcs carry edge terms)
        const int32_t lowest = accumulate && !eb ? 1 : 0;
        for (int32_t l = nlev - 1; l >= lowest; --l) {
            const int32_t lb = lev[l], le = lev[l + 1];
            if (l < nlev - 1) {
                // acc[v] = sum of c(w) = acc[w] over successors w (level l + 1)
                for (int32_t cb = lb; cb < le; cb += PB) {
                    const int tot = wg::stage_chunk(queue, cb, le, rp, ch);
                    for (int e0 = tid; e0 < tot; e0 += PB * U) {
                        int k[U];
                        int32_t a[U], w[U], dw[U];
                        wg::arc_burst<U>(ch, e0, tot, k, a);
#pragma unroll
                        for (int j = 0; j < U; ++j) w[j] = a[j] >= 0 ? col[a[j]] : 0;
#pragma unroll
                        for (int j = 0; j < U; ++j) dw[j] = a[j] >= 0 ? dist[w[j]] : -1;
#pragma unroll
                        for (int j = 0; j < U; ++j)
                            if (a[j] >= 0 && dw[j] == l + 1) {
                                const int32_t v = ch.v[k[j]];
                                const double cw = acc[w[j]];
                                unsafeAtomicAdd(&acc[v], cw);
                                // edge term of arc v -> w: lambda(v) c(w)
                                if (eb) unsafeAtomicAdd(&eb[a[j]], (double)sigma[v] * cw);
                            }
                    }
                    __syncthreads();
                }
                wg::bar();
            }
            for (int32_t i = lb + tid; i < le; i += PB) {
                const int32_t v = queue[i];
                const double sv = (double)sigma[v];
                const double dl = sv * acc[v];
                if (accumulate && v != s) unsafeAtomicAdd(&bc[v], dl);
                if (delta_dump) delta_dump[(size_t)idx * n + v] = dl;
                acc[v] = (1.0 + dl) / sv;
            }
            wg::bar();
        }
        if (dist_dump) {
            for (int32_t v = tid; v < n; v += PB) {
                const int32_t d = dist[v];
                dist_dump[(size_t)idx * n + v] = d;
                sigma_dump[(size_t)idx * n + v] = d >= 0 ? sigma[v] : 0;
                if (d < 0) delta_dump[(size_t)idx * n + v] = 0.0;
            }
        }
        if (tid == 0 && s_ovf) atomicOr(status, (uint32_t)BC_DEV_SIGMA_OVERFLOW);
        wg::bar();
    }
}

} // namespace

bc_status plain_prepare(bc_ctx *ctx) {
    if (ctx->weighted) return weighted_prepare(ctx);
    PlainState &p = ctx->pl;
    const size_t n = (size_t)std::max(ctx->n, 1);
    const size_t per_group = n * (4 + 8 + 8 + 4) + (n + 2) * 4;
    const size_t budget = size_t(16) << 30;
    int groups = p.grid > 0 ? p.grid : 2048;
    while (groups > 1 && per_group * (size_t)groups > budget) groups /= 2;
    p.groups = groups;
    p.dist = (int32_t *)bc_dalloc(ctx, n * groups * sizeof(int32_t));
    p.sigma = (uint64_t *)bc_dalloc(ctx, n * groups * sizeof(uint64_t));
    p.acc = (double *)bc_dalloc(ctx, n * groups * sizeof(double));
    p.queue = (int32_t *)bc_dalloc(ctx, n * groups * sizeof(int32_t));
    p.lev = (int32_t *)bc_dalloc(ctx, (n + 2) * groups * sizeof(int32_t));
    p.next = (uint32_t *)bc_dalloc(ctx, 256);
    if (!p.dist || !p.sigma || !p.acc || !p.queue || !p.lev || !p.next)
        return bc_fail(ctx, BC_ERR_NOMEM, "plain form: workspace allocation failed");
    return BC_OK;
}

bc_status plain_run(bc_ctx *ctx, const int32_t *d_sources, int64_t count, bool accumulate,
                    double *delta_dump, int32_t *dist_dump, uint64_t *sigma_dump) {
    if (ctx->weighted) return weighted_run(ctx, d_sources, count, accumulate, delta_dump, dist_dump, sigma_dump);
    PlainState &p = ctx->pl;
    BC_HIP(ctx, hipMemsetAsync(p.next, 0, sizeof(unsigned long long), ctx->stream));
    const int grid = (int)std::min<int64_t>(count, p.groups);
    LaunchTimer t(ctx, "plain_sweep");
    hipLaunchKernelGGL(k_plain_sweep, dim3(grid), dim3(PB), 0, ctx->stream, ctx->n, ctx->row_ptr, ctx->col,
                       d_sources, count, (unsigned long long *)p.next, p.dist, p.sigma, p.acc, p.queue, p.lev,
                       ctx->bc, ctx->status, accumulate ? 1 : 0, delta_dump, dist_dump, sigma_dump,
                       accumulate && ctx->edges ? ctx->eb : nullptr);
    t.done();
    BC_HIP(ctx, hipGetLastError());
    return BC_OK;
}
