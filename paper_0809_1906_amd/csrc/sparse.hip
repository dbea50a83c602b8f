// Batched sparse form: B sources at once (B a multiple of 64), unit weights.
//
// State is batch-minor.  For level l the frontier is a bitmap
// front[l][v][q] (uint64): bit b of word q is set iff d(s_{64q+b}, v) = l.
// Path counts sigma[v][64q+b] are uint64 and c(v) = (1 + delta(v)) / sigma(v)
// is stored as FP32 in cval[v][64q+b]; all sums are formed in FP64 registers.
//
// One wave handles one (vertex, word) pair; lane b is source 64q+b, so every
// gather of a neighbour's sigma or c row is one coalesced 512 B (256 B) read.
// The wave first loads 64 neighbour ids and their frontier words at once,
// keeps only the neighbours whose word intersects its own mask (ballot), and
// then gathers rows for those neighbours only.
//
//   forward level l -> l+1 (pull):  for w with unvisited sources U,
//       sigma(w,b) = sum over neighbours v with bit b of front[l][v] & U of
//       sigma(v,b);  front[l+1][w] = bits where that sum is non-zero.
//       This is the level-synchronous search of Sec. 4 with the counting rule
//       lambda_sw = sum of lambda_sv over v in P_s(w) (Sec. 1.1).
//   backward level l (pull):  for v with bits F = front[l][v],
//       delta(v,b) = sigma(v,b) * sum over neighbours w with bit b of
//       front[l+1][w] & F of c(w,b)      (Theorem 1.1; ParallelCompute of
//       Sec. 4.2.2 with the 1/lambda factor kept inside c);
//       BC(v) += sum over b with s_b != v of delta(v,b).
// Level 0 is never accumulated: there v is the source itself.
#include "bc_internal.h"

#include <algorithm>

namespace {

constexpr int SB = 256;      // threads per block = 4 waves
constexpr int CSLOTS = 64;   // frontier counters per level, one per 128 B line
constexpr int CSTRIDE = 32;  // uint32 per counter slot

__device__ __forceinline__ int32_t rl32(int32_t x, int j) { return __builtin_amdgcn_readlane(x, j); }
__device__ __forceinline__ uint64_t rl64(uint64_t x, int j) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, j);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}

__global__ __launch_bounds__(SB) void k_sp_clear(uint64_t *__restrict__ a, uint64_t *__restrict__ b, size_t words) {
    for (size_t i = (size_t)blockIdx.x * SB + threadIdx.x; i < words; i += (size_t)gridDim.x * SB) {
        a[i] = 0;
        b[i] = 0;
    }
}

__global__ __launch_bounds__(SB) void k_sp_seed(const int32_t *__restrict__ src, int32_t count, int32_t B, int32_t NW,
                                                uint64_t *front0, uint64_t *visited, uint64_t *sigma,
                                                int32_t *src_lane) {
    const int32_t b = blockIdx.x * SB + threadIdx.x;
    if (b >= B) return;
    const int32_t s = b < count ? src[b] : -1;
    src_lane[b] = s;
    if (s >= 0) {
        const unsigned long long bit = 1ull << (b & 63);
        atomicOr((unsigned long long *)&front0[(size_t)s * NW + (b >> 6)], bit);
        atomicOr((unsigned long long *)&visited[(size_t)s * NW + (b >> 6)], bit);
        sigma[(size_t)s * B + b] = 1;
    }
}

__global__ __launch_bounds__(SB) void k_fwd_pull(int32_t n, int32_t NW, int32_t B,
                                                 const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                 const uint64_t *__restrict__ fcur, uint64_t *__restrict__ fnext,
                                                 uint64_t *__restrict__ visited, uint64_t *__restrict__ sigma,
                                                 uint32_t *__restrict__ counts, uint32_t *__restrict__ status) {
    __shared__ uint32_t s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * (SB / 64) + (threadIdx.x >> 6);
    if (wid < (int64_t)n * NW) {
        const int32_t w = (int32_t)(wid / NW), q = (int32_t)(wid - (int64_t)w * NW);
        const uint64_t vis = visited[wid];
        const uint64_t U = ~vis;
        uint64_t out = 0;
        if (U != 0) {
            const int32_t beg = rp[w], end = rp[w + 1];
            const uint64_t *sig_q = sigma + (size_t)q * 64 + lane;
            uint64_t acc = 0;
            bool ovf = false;
            for (int32_t base = beg; base < end; base += 64) {
                const int32_t e = base + lane;
                int32_t v = 0;
                uint64_t f = 0;
                if (e < end) {
                    v = col[e];
                    f = fcur[(size_t)v * NW + q] & U;
                }
                uint64_t act = __ballot(f != 0);
                while (act) {
                    const int j = __ffsll((unsigned long long)act) - 1;
                    act &= act - 1;
                    const int32_t vj = rl32(v, j);
                    const uint64_t fj = rl64(f, j);
                    if ((fj >> lane) & 1) {
                        const uint64_t x = sig_q[(size_t)vj * B];
                        const uint64_t t = acc + x;
                        ovf |= t < acc;
                        acc = t;
                    }
                }
            }
            out = __ballot(acc != 0);
            if (acc != 0) sigma[(size_t)w * B + (size_t)q * 64 + lane] = acc;
            if (__any(ovf) && lane == 0) atomicOr(status, (uint32_t)BC_DEV_SIGMA_OVERFLOW);
        }
        if (lane == 0) {
            fnext[wid] = out;
            if (out) {
                visited[wid] = vis | out;
                atomicAdd(&s_cnt, 1u);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt) atomicAdd(&counts[(blockIdx.x % CSLOTS) * CSTRIDE], s_cnt);
}

__global__ __launch_bounds__(SB) void k_bwd_pull(int32_t n, int32_t NW, int32_t B,
                                                 const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                 const uint64_t *__restrict__ fcur, const uint64_t *__restrict__ fnext,
                                                 const uint64_t *__restrict__ sigma, float *__restrict__ cval,
                                                 const int32_t *__restrict__ src_lane, double *__restrict__ bc,
                                                 double *__restrict__ delta_dump, int accumulate) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * (SB / 64) + (threadIdx.x >> 6);
    if (wid >= (int64_t)n * NW) return;
    const uint64_t F = fcur[wid];
    if (F == 0) return;
    const int32_t v = (int32_t)(wid / NW), q = (int32_t)(wid - (int64_t)v * NW);
    double acc = 0.0;
    if (fnext) {
        const int32_t beg = rp[v], end = rp[v + 1];
        const float *c_q = cval + (size_t)q * 64 + lane;
        for (int32_t base = beg; base < end; base += 64) {
            const int32_t e = base + lane;
            int32_t w = 0;
            uint64_t g = 0;
            if (e < end) {
                w = col[e];
                g = fnext[(size_t)w * NW + q] & F;
            }
            uint64_t act = __ballot(g != 0);
            while (act) {
                const int j = __ffsll((unsigned long long)act) - 1;
                act &= act - 1;
                const int32_t wj = rl32(w, j);
                const uint64_t gj = rl64(g, j);
                if ((gj >> lane) & 1) acc += (double)c_q[(size_t)wj * B];
            }
        }
    }
    double contrib = 0.0;
    if ((F >> lane) & 1) {
        const size_t idx = (size_t)v * B + (size_t)q * 64 + lane;
        const double sv = (double)sigma[idx];
        const double dl = sv * acc;
        cval[idx] = (float)((1.0 + dl) / sv);
        if (delta_dump) delta_dump[idx] = dl;
        if (src_lane[q * 64 + lane] != v) contrib = dl;
    }
    if (accumulate) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) contrib += __shfl_xor(contrib, off, 64);
        if (lane == 0 && contrib != 0.0) unsafeAtomicAdd(&bc[v], contrib);
    }
}

// Per-source readout for bc_read_sssp: out[b][v] in source-major layout.
__global__ __launch_bounds__(SB) void k_sp_dump(int32_t n, int32_t NW, int32_t B, int32_t count, int32_t nlev,
                                                const uint64_t *__restrict__ front, const uint64_t *__restrict__ sigma,
                                                const double *__restrict__ dstate, int32_t *__restrict__ dist_out,
                                                uint64_t *__restrict__ sigma_out, double *__restrict__ delta_out) {
    const int64_t i = (int64_t)blockIdx.x * SB + threadIdx.x;
    if (i >= (int64_t)n * count) return;
    const int32_t b = (int32_t)(i / n), v = (int32_t)(i - (int64_t)b * n);
    const int q = b >> 6, bit = b & 63;
    int32_t d = -1;
    for (int32_t l = 0; l < nlev && d < 0; ++l)
        if ((front[((size_t)l * n + v) * NW + q] >> bit) & 1) d = l;
    const size_t idx = (size_t)v * B + b;
    dist_out[i] = d;
    sigma_out[i] = d >= 0 ? sigma[idx] : 0;
    delta_out[i] = d >= 0 ? dstate[idx] : 0.0;
}

bc_status ensure_levels(bc_ctx *ctx, int32_t need) {
    SparseState &s = ctx->sp;
    if (need <= s.level_cap) return BC_OK;
    int32_t cap = std::max(s.level_cap * 2, need);
    const size_t per_level = (size_t)ctx->n * s.words * sizeof(uint64_t);
    const size_t budget = size_t(32) << 30;
    if ((size_t)cap * per_level > budget) {
        cap = need;
        if ((size_t)cap * per_level > budget)
            return bc_fail(ctx, BC_ERR_UNSUPPORTED,
                           "sparse form: the graph is too deep for per-level frontier bitmaps; use the plain form");
    }
    uint64_t *nf = (uint64_t *)bc_dalloc(ctx, (size_t)cap * per_level);
    uint32_t *nc = (uint32_t *)bc_dalloc(ctx, (size_t)cap * CSLOTS * CSTRIDE * sizeof(uint32_t));
    uint32_t *nh = nullptr;
    if (!nf || !nc || hipHostMalloc((void **)&nh, (size_t)cap * CSLOTS * CSTRIDE * sizeof(uint32_t)) != hipSuccess) {
        bc_dfree(ctx, nf);
        bc_dfree(ctx, nc);
        return bc_fail(ctx, BC_ERR_NOMEM, "sparse form: frontier allocation failed");
    }
    if (s.front) {
        BC_HIP(ctx, hipMemcpyAsync(nf, s.front, (size_t)s.level_cap * per_level, hipMemcpyDeviceToDevice, ctx->stream));
        BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
        bc_dfree(ctx, s.front);
        bc_dfree(ctx, s.counts);
        hipHostFree(s.counts_host);
    }
    s.front = nf;
    s.counts = nc;
    s.counts_host = nh;
    s.level_cap = cap;
    return BC_OK;
}

// One batch of up to B sources.  Returns the number of non-empty levels.
bc_status run_batch(bc_ctx *ctx, const int32_t *d_src, int32_t count, bool accumulate, int32_t *nlev_out) {
    SparseState &s = ctx->sp;
    const int32_t n = ctx->n, NW = s.words, B = s.batch;
    const size_t words = (size_t)n * NW;
    const int wave_blocks = (int)(((int64_t)n * NW + (SB / 64) - 1) / (SB / 64));
    {
        LaunchTimer t(ctx, "batch_init");
        const int blocks = (int)std::min<size_t>((words + SB - 1) / SB, 8192);
        hipLaunchKernelGGL(k_sp_clear, dim3(std::max(blocks, 1)), dim3(SB), 0, ctx->stream, s.front, s.visited, words);
        hipLaunchKernelGGL(k_sp_seed, dim3((B + SB - 1) / SB), dim3(SB), 0, ctx->stream, d_src, count, B, NW, s.front,
                           s.visited, s.sigma, s.src);
        t.done();
        BC_HIP(ctx, hipGetLastError());
    }
    int32_t l = 0;
    for (;;) {
        bc_status st = ensure_levels(ctx, l + 2);
        if (st != BC_OK) return st;
        uint32_t *cnt = s.counts + (size_t)(l + 1) * CSLOTS * CSTRIDE;
        BC_HIP(ctx, hipMemsetAsync(cnt, 0, CSLOTS * CSTRIDE * sizeof(uint32_t), ctx->stream));
        LaunchTimer t(ctx, "fwd_pull");
        hipLaunchKernelGGL(k_fwd_pull, dim3(wave_blocks), dim3(SB), 0, ctx->stream, n, NW, B, ctx->row_ptr, ctx->col,
                           s.front + (size_t)l * words, s.front + (size_t)(l + 1) * words, s.visited, s.sigma, cnt,
                           ctx->status);
        t.done();
        BC_HIP(ctx, hipGetLastError());
        uint32_t *hc = s.counts_host + (size_t)(l + 1) * CSLOTS * CSTRIDE;
        BC_HIP(ctx, hipMemcpyAsync(hc, cnt, CSLOTS * CSTRIDE * sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream));
        BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
        uint64_t total = 0;
        for (int i = 0; i < CSLOTS; ++i) total += hc[i * CSTRIDE];
        if (total == 0) break;
        ++l;
    }
    const int32_t nlev = l + 1;
    const int32_t lowest = accumulate ? 1 : 0;
    for (int32_t lv = nlev - 1; lv >= lowest; --lv) {
        LaunchTimer t(ctx, "bwd_pull");
        hipLaunchKernelGGL(k_bwd_pull, dim3(wave_blocks), dim3(SB), 0, ctx->stream, n, NW, B, ctx->row_ptr, ctx->col,
                           s.front + (size_t)lv * words, lv + 1 < nlev ? s.front + (size_t)(lv + 1) * words : nullptr,
                           s.sigma, s.cval, s.src, ctx->bc, accumulate ? nullptr : s.delta_dump, accumulate ? 1 : 0);
        t.done();
        BC_HIP(ctx, hipGetLastError());
    }
    ctx->max_levels = std::max(ctx->max_levels, nlev);
    *nlev_out = nlev;
    return BC_OK;
}

} // namespace

bc_status sparse_prepare(bc_ctx *ctx, int32_t batch) {
    SparseState &s = ctx->sp;
    s.batch = batch;
    s.words = batch / 64;
    const size_t n = (size_t)std::max(ctx->n, 1);
    s.visited = (uint64_t *)bc_dalloc(ctx, n * s.words * sizeof(uint64_t));
    s.sigma = (uint64_t *)bc_dalloc(ctx, n * batch * sizeof(uint64_t));
    s.cval = (float *)bc_dalloc(ctx, n * batch * sizeof(float));
    s.src = (int32_t *)bc_dalloc(ctx, batch * sizeof(int32_t));
    if (!s.visited || !s.sigma || !s.cval || !s.src) return bc_fail(ctx, BC_ERR_NOMEM, "sparse form: state allocation failed");
    return ensure_levels(ctx, 16);
}

bc_status sparse_run(bc_ctx *ctx, const int32_t *d_src, int64_t count) {
    const int32_t B = ctx->sp.batch;
    for (int64_t b0 = 0; b0 < count; b0 += B) {
        int32_t nlev = 0;
        bc_status st = run_batch(ctx, d_src + b0, (int32_t)std::min<int64_t>(B, count - b0), true, &nlev);
        if (st != BC_OK) return st;
    }
    return BC_OK;
}

bc_status sparse_dump(bc_ctx *ctx, const int32_t *d_src, int32_t count,
                      int32_t *dist_dump, uint64_t *sigma_dump, double *delta_dump) {
    SparseState &s = ctx->sp;
    if (!s.delta_dump) {
        s.delta_dump = (double *)bc_dalloc(ctx, (size_t)std::max(ctx->n, 1) * s.batch * sizeof(double));
        if (!s.delta_dump) return bc_fail(ctx, BC_ERR_NOMEM, "sparse form: dump allocation failed");
    }
    int32_t nlev = 0;
    bc_status st = run_batch(ctx, d_src, count, false, &nlev);
    if (st != BC_OK) return st;
    const int64_t cells = (int64_t)ctx->n * count;
    hipLaunchKernelGGL(k_sp_dump, dim3((unsigned)((cells + SB - 1) / SB)), dim3(SB), 0, ctx->stream, ctx->n, s.words,
                       s.batch, count, nlev, s.front, s.sigma, s.delta_dump, dist_dump, sigma_dump, delta_dump);
    BC_HIP(ctx, hipGetLastError());
    return BC_OK;
}
