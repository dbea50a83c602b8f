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
// prefix sums are staged in LDS, so a thread takes one arc, not one vertex:
// hub vertices are spread over the whole workgroup.
#include "bc_internal.h"

namespace {

constexpr int PB = 256; // threads per workgroup

// Workgroup barrier with device-scope ordering: the per-source arrays are
// updated by device atomics (performed in L2), so every phase change must
// make them visible across the workgroup's waves.
__device__ __forceinline__ void bar() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ __forceinline__ int wave_incl_scan(int x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive prefix sum over the workgroup; *total receives the sum.
__device__ __forceinline__ int block_excl_scan(int x, int *wsum, int *total) {
    const int incl = wave_incl_scan(x);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < PB / 64; ++i) {
        int s = wsum[i];
        if (i < wid) off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + incl - x;
}

// Largest k in [0, PB) with off[k] <= e, given off[0] = 0 <= e < off[PB].
__device__ __forceinline__ int owner(const int *off, int e) {
    int lo = 0, hi = PB;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= e) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(PB) void k_plain_sweep(
    int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const int32_t *__restrict__ sources, int64_t count, unsigned long long *next_counter,
    int32_t *dist_all, uint64_t *sigma_all, double *acc_all, int32_t *queue_all, int32_t *lev_all,
    double *bc, uint32_t *status, int accumulate,
    double *delta_dump, int32_t *dist_dump, uint64_t *sigma_dump) {
    __shared__ int32_t s_v[PB];
    __shared__ int32_t s_rp[PB];
    __shared__ int32_t s_off[PB + 1];
    __shared__ uint64_t s_sig[PB];
    __shared__ int32_t s_wsum[PB / 64];
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
        bar();
        if (tid == 0) {
            dist[s] = 0;
            sigma[s] = 1;
            queue[0] = s;
            lev[0] = 0;
            lev[1] = 1;
            s_tail = 1;
            s_ovf = 0;
        }
        bar();

        // ---- forward: level L spans queue[qb, qe) ----
        int32_t qb = 0, qe = 1, L = 0;
        while (qb < qe) {
            for (int32_t cb = qb; cb < qe; cb += PB) {
                const int32_t i = cb + tid;
                int32_t v = -1, r = 0, d = 0;
                uint64_t sg = 0;
                if (i < qe) {
                    v = queue[i];
                    r = rp[v];
                    d = rp[v + 1] - r;
                    sg = sigma[v];
                }
                int tot;
                const int off = block_excl_scan(d, s_wsum, &tot);
                s_v[tid] = v;
                s_rp[tid] = r;
                s_off[tid] = off;
                s_sig[tid] = sg;
                if (tid == 0) s_off[PB] = tot;
                __syncthreads();
                for (int e = tid; e < tot; e += PB) {
                    const int k = owner(s_off, e);
                    const int32_t w = col[s_rp[k] + (e - s_off[k])];
                    int32_t dw = dist[w];
                    if (dw < 0) {
                        const int32_t old = atomicCAS(&dist[w], -1, L + 1);
                        if (old == -1) {
                            const int pos = atomicAdd(&s_tail, 1);
                            queue[pos] = w;
                            dw = L + 1;
                        } else {
                            dw = old;
                        }
                    }
                    if (dw == L + 1) { // v in P_s(w)
                        const uint64_t x = s_sig[k];
                        const uint64_t old = atomicAdd((unsigned long long *)&sigma[w], (unsigned long long)x);
                        if (old + x < old) s_ovf = 1;
                    }
                }
                bar();
            }
            qb = qe;
            qe = s_tail;
            ++L;
            if (tid == 0) lev[L + 1] = qe;
            bar();
        }
        const int32_t nlev = L; // non-empty levels 0..nlev-1

        // ---- backward: deepest level first ----
        const int32_t lowest = accumulate ? 1 : 0;
        for (int32_t l = nlev - 1; l >= lowest; --l) {
            const int32_t lb = lev[l], le = lev[l + 1];
            if (l < nlev - 1) {
                for (int32_t cb = lb; cb < le; cb += PB) {
                    const int32_t i = cb + tid;
                    int32_t v = -1, r = 0, d = 0;
                    if (i < le) {
                        v = queue[i];
                        r = rp[v];
                        d = rp[v + 1] - r;
                    }
                    int tot;
                    const int off = block_excl_scan(d, s_wsum, &tot);
                    s_v[tid] = v;
                    s_rp[tid] = r;
                    s_off[tid] = off;
                    if (tid == 0) s_off[PB] = tot;
                    __syncthreads();
                    for (int e = tid; e < tot; e += PB) {
                        const int k = owner(s_off, e);
                        const int32_t w = col[s_rp[k] + (e - s_off[k])];
                        if (dist[w] == l + 1) unsafeAtomicAdd(&acc[s_v[k]], acc[w]); // acc[w] holds c(w)
                    }
                    bar();
                }
            }
            for (int32_t i = lb + tid; i < le; i += PB) {
                const int32_t v = queue[i];
                const double sv = (double)sigma[v];
                const double dl = sv * acc[v];
                if (accumulate && v != s) unsafeAtomicAdd(&bc[v], dl);
                if (delta_dump) delta_dump[(size_t)idx * n + v] = dl;
                acc[v] = (1.0 + dl) / sv;
            }
            bar();
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
        bar();
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
                       ctx->bc, ctx->status, accumulate ? 1 : 0, delta_dump, dist_dump, sigma_dump);
    t.done();
    BC_HIP(ctx, hipGetLastError());
    return BC_OK;
}
