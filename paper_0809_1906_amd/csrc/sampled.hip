// Algorithm 1 of Sec. 4.1.1, the sampled forward for unweighted graphs,
// distances only.  With a distinguished set S (the requested sources first,
// then the caller's random sample):
//   step 2  a k-limited breadth-first search from every x in S gives d'(x, v):
//           the hop distance when it is at most k, otherwise none;
//   step 3  the weighted graph H on S has edge weights d'(x, y);
//   step 4  all-pairs distances D_H of H (Floyd-Warshall);
//   step 5  d(s, v) = min over x in S of D_H(s, x) + d'(x, v).
// Step 6 (counting minimising vertices) does not count shortest paths and is
// not computed.
//
// Layout: d' is uint16 [Sp][n] (Sp = |S| rounded up to 64; DINF = no path
// within k), H and D_H int32 [Sp][Sp] (HINF = no path; HINF + HINF fits
// int32).  The limited searches run 64 sources at a time as one bitmap word per
// vertex: level L pulls the frontier words of each vertex's neighbours.  The
// final minimum gives each block four sources and 256 vertices; the four rows
// of D_H sit in LDS and each d' row is read coalesced across the block.
#include "bc_internal.h"

#include <algorithm>
#include <cmath>
#include <unordered_map>

namespace {

constexpr int SB = 256;
constexpr uint16_t DINF = 0xFFFF;
constexpr int32_t HINF = 1 << 29;
constexpr int IT = 4; // sources per block of the final minimum

inline unsigned blocks_for(size_t count) { return (unsigned)((count + SB - 1) / SB); }

__global__ __launch_bounds__(SB) void k_fill_u16(uint16_t *__restrict__ x, size_t count, uint16_t value) {
    const size_t i = (size_t)blockIdx.x * SB + threadIdx.x;
    if (i < count) x[i] = value;
}

// Start of a 64-source word: clear the bitmaps (the sources follow).
__global__ __launch_bounds__(SB) void k_lb_clear(int32_t n, uint64_t *__restrict__ front,
                                                 uint64_t *__restrict__ visited) {
    const int32_t v = blockIdx.x * SB + threadIdx.x;
    if (v < n) {
        front[v] = 0;
        visited[v] = 0;
    }
}

// The word's sources at level 0.
__global__ __launch_bounds__(64) void k_lb_sources(int32_t n, const int32_t *__restrict__ S, int32_t base,
                                                   int32_t cnt, uint64_t *__restrict__ front,
                                                   uint64_t *__restrict__ visited, uint16_t *__restrict__ dp) {
    const int b = threadIdx.x;
    if (b >= cnt) return;
    const int32_t x = S[base + b];
    atomicOr((unsigned long long *)&front[x], 1ull << b);
    atomicOr((unsigned long long *)&visited[x], 1ull << b);
    dp[(size_t)(base + b) * n + x] = 0;
}

// Level L of the limited searches of one word: every vertex not yet reached
// by all of the word's sources pulls its neighbours' frontier bits.
__global__ __launch_bounds__(SB) void k_lb_level(int32_t n, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ col, uint64_t full, int32_t base,
                                                 int32_t L, const uint64_t *__restrict__ front,
                                                 uint64_t *__restrict__ next, uint64_t *__restrict__ visited,
                                                 uint16_t *__restrict__ dp, uint32_t *__restrict__ found) {
    const int32_t v = blockIdx.x * SB + threadIdx.x;
    uint64_t nw = 0;
    if (v < n) {
        const uint64_t vis = visited[v];
        if (vis != full) {
            uint64_t acc = 0;
            for (int32_t e = rp[v]; e < rp[v + 1]; ++e) acc |= front[col[e]];
            nw = acc & ~vis & full;
            if (nw) {
                visited[v] = vis | nw;
                for (uint64_t m = nw; m; m &= m - 1) dp[(size_t)(base + __builtin_ctzll(m)) * n + v] = (uint16_t)L;
            }
        }
        next[v] = nw;
    }
    if (__any(nw != 0) && (threadIdx.x & 63) == 0) found[L] = 1;
}

// Step 3: H[i][j] = d'(S_i, S_j), 0 on the diagonal, HINF where no path was
// found and in the padding.
__global__ __launch_bounds__(SB) void k_build_h(int32_t n, int32_t ns, int32_t sp, const int32_t *__restrict__ S,
                                                const uint16_t *__restrict__ dp, int32_t *__restrict__ H) {
    const size_t id = (size_t)blockIdx.x * SB + threadIdx.x;
    if (id >= (size_t)sp * sp) return;
    const int32_t i = (int32_t)(id / sp), j = (int32_t)(id % sp);
    int32_t h = HINF;
    if (i == j) h = 0;
    else if (i < ns && j < ns) {
        const uint16_t d = dp[(size_t)i * n + S[j]];
        h = d == DINF ? HINF : (int32_t)d;
    }
    H[id] = h;
}

// Step 4, pivot k: H[i][j] = min(H[i][j], H[i][k] + H[k][j]).  Row and
// column k do not change in this pass (H[k][k] = 0), so it runs in place.
__global__ __launch_bounds__(SB) void k_fw(int32_t sp, int32_t k, int32_t *__restrict__ H) {
    const size_t id = (size_t)blockIdx.x * SB + threadIdx.x;
    if (id >= (size_t)sp * sp) return;
    const int32_t i = (int32_t)(id / sp), j = (int32_t)(id % sp);
    const int32_t via = H[(size_t)i * sp + k] + H[(size_t)k * sp + j];
    if (via < H[id]) H[id] = via;
}

// Step 5: out[r][v] = min over x of D_H(r, x) + d'(x, v) for the requested
// sources r (rows 0 .. count-1 of S); -1 where no walk was found.
__global__ __launch_bounds__(SB) void k_final(int32_t n, int32_t ns, int32_t sp, int32_t count,
                                              const int32_t *__restrict__ DH, const uint16_t *__restrict__ dp,
                                              int32_t *__restrict__ out) {
    extern __shared__ int32_t s_h[]; // [IT][sp]
    const int32_t r0 = blockIdx.y * IT;
    for (int32_t i = threadIdx.x; i < IT * sp; i += SB) {
        const int32_t t = i / sp, x = i % sp;
        s_h[i] = r0 + t < count ? DH[(size_t)(r0 + t) * sp + x] : HINF;
    }
    __syncthreads();
    const int32_t v = blockIdx.x * SB + threadIdx.x;
    if (v >= n) return;
    int32_t best[IT];
#pragma unroll
    for (int t = 0; t < IT; ++t) best[t] = HINF;
    for (int32_t x = 0; x < ns; ++x) {
        const uint16_t d = dp[(size_t)x * n + v];
        if (d == DINF) continue;
#pragma unroll
        for (int t = 0; t < IT; ++t) best[t] = min(best[t], s_h[t * sp + x] + (int32_t)d);
    }
#pragma unroll
    for (int t = 0; t < IT; ++t)
        if (r0 + t < count) out[(size_t)(r0 + t) * n + v] = best[t] >= HINF ? -1 : best[t];
}

} // namespace

bc_status sampled_distances(bc_ctx *ctx, const int32_t *h_sources, int32_t count, const int32_t *h_sample,
                            int32_t nsample, int32_t limit, int32_t *h_out) {
    const int32_t n = ctx->n;
    // S: the distinct requested sources first (rows 0 .. nreq-1), then the
    // sample; row_of[i] is the row of the i-th requested source
    std::vector<int32_t> S, row_of((size_t)count);
    {
        std::unordered_map<int32_t, int32_t> pos;
        for (int32_t i = 0; i < count; ++i) {
            auto it = pos.emplace(h_sources[i], (int32_t)S.size());
            if (it.second) S.push_back(h_sources[i]);
            row_of[(size_t)i] = it.first->second;
        }
        for (int32_t i = 0; i < nsample; ++i)
            if (pos.emplace(h_sample[i], (int32_t)S.size()).second) S.push_back(h_sample[i]);
    }
    const int32_t ns = (int32_t)S.size();
    int32_t nreq = 0;
    for (int32_t r : row_of) nreq = std::max(nreq, r + 1);
    if (ns > BC_SAMPLED_MAX_S)
        return bc_fail(ctx, BC_ERR_UNSUPPORTED, "sampled forward: more than BC_SAMPLED_MAX_S distinguished vertices");
    const int32_t k = limit > 0 ? limit : std::max(1, (int32_t)std::ceil(std::sqrt((double)n)));
    if (k > 65534) return bc_fail(ctx, BC_ERR_INVALID_ARG, "sampled forward: limit above 65534");
    const int32_t sp = (ns + 63) / 64 * 64;
    int32_t *dS = (int32_t *)bc_dalloc(ctx, sizeof(int32_t) * (size_t)std::max(sp, 1));
    uint16_t *dp = (uint16_t *)bc_dalloc(ctx, sizeof(uint16_t) * (size_t)sp * n);
    int32_t *H = (int32_t *)bc_dalloc(ctx, sizeof(int32_t) * (size_t)sp * sp);
    uint64_t *front = (uint64_t *)bc_dalloc(ctx, sizeof(uint64_t) * (size_t)n);
    uint64_t *next = (uint64_t *)bc_dalloc(ctx, sizeof(uint64_t) * (size_t)n);
    uint64_t *visited = (uint64_t *)bc_dalloc(ctx, sizeof(uint64_t) * (size_t)n);
    uint32_t *found = (uint32_t *)bc_dalloc(ctx, sizeof(uint32_t) * (size_t)(k + 1));
    int32_t *outi = (int32_t *)bc_dalloc(ctx, sizeof(int32_t) * (size_t)std::max(nreq, 1) * n);
    int32_t *outc = (int32_t *)bc_dalloc(ctx, sizeof(int32_t) * (size_t)std::max(nreq, 1) * n);
    std::vector<uint32_t> found_h((size_t)k + 1);
    auto cleanup = [&]() {
        for (void *p : {(void *)dS, (void *)dp, (void *)H, (void *)front, (void *)next, (void *)visited,
                        (void *)found, (void *)outi, (void *)outc})
            bc_dfree(ctx, p);
    };
    if (!dS || !dp || !H || !front || !next || !visited || !found || !outi || !outc) {
        cleanup();
        return bc_fail(ctx, BC_ERR_NOMEM, "sampled forward: allocation failed");
    }
    auto fail_hip = [&](hipError_t e, const char *what) {
        cleanup();
        return bc_hip(ctx, e, what);
    };
    hipError_t e = hipMemcpy(dS, S.data(), sizeof(int32_t) * (size_t)ns, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail_hip(e, "sampled forward: upload");
    bc_status st = map_ids_to_internal(ctx, dS, ns);
    if (st != BC_OK) {
        cleanup();
        return st;
    }
    hipLaunchKernelGGL(k_fill_u16, dim3(blocks_for((size_t)sp * n)), dim3(SB), 0, ctx->stream, dp, (size_t)sp * n,
                       DINF);
    // step 2: limited searches, one word of 64 sources at a time
    {
        LaunchTimer tm(ctx, "limited_bfs");
        for (int32_t base = 0; base < ns; base += 64) {
            const int32_t cnt = std::min(64, ns - base);
            const uint64_t full = cnt == 64 ? ~0ull : ((1ull << cnt) - 1);
            hipLaunchKernelGGL(k_lb_clear, dim3(blocks_for((size_t)n)), dim3(SB), 0, ctx->stream, n, front, visited);
            hipLaunchKernelGGL(k_lb_sources, dim3(1), dim3(64), 0, ctx->stream, n, dS, base, cnt, front, visited, dp);
            e = hipMemsetAsync(found, 0, sizeof(uint32_t) * (size_t)(k + 1), ctx->stream);
            if (e != hipSuccess) return fail_hip(e, "sampled forward: clear");
            uint64_t *f = front, *g = next;
            for (int32_t L = 1; L <= k; ++L) {
                hipLaunchKernelGGL(k_lb_level, dim3(blocks_for((size_t)n)), dim3(SB), 0, ctx->stream, n, ctx->row_ptr,
                                   ctx->col, full, base, L, f, g, visited, dp, found);
                std::swap(f, g);
                // every 8 levels: stop once a level found nothing new
                if (L % 8 == 0 || L == k) {
                    e = hipMemcpyAsync(found_h.data(), found, sizeof(uint32_t) * (size_t)(k + 1),
                                       hipMemcpyDeviceToHost, ctx->stream);
                    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
                    if (e != hipSuccess) return fail_hip(e, "sampled forward: level read-back");
                    if (found_h[(size_t)L] == 0) break;
                }
            }
        }
        tm.done();
    }
    // steps 3 and 4
    hipLaunchKernelGGL(k_build_h, dim3(blocks_for((size_t)sp * sp)), dim3(SB), 0, ctx->stream, n, ns, sp, dS, dp, H);
    {
        LaunchTimer tm(ctx, "floyd_warshall");
        for (int32_t kk = 0; kk < ns; ++kk)
            hipLaunchKernelGGL(k_fw, dim3(blocks_for((size_t)sp * sp)), dim3(SB), 0, ctx->stream, sp, kk, H);
        tm.done();
    }
    // step 5
    if (nreq > 0 && n > 0) {
        LaunchTimer tm(ctx, "sampled_min");
        hipLaunchKernelGGL(k_final, dim3(blocks_for((size_t)n), (nreq + IT - 1) / IT), dim3(SB),
                           sizeof(int32_t) * IT * (size_t)sp, ctx->stream, n, ns, sp, nreq, H, dp, outi);
        tm.done();
    }
    e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "sampled forward");
    if (nreq > 0 && n > 0) {
        st = rows_to_caller_order_i32(ctx, outc, outi, nreq);
        if (st != BC_OK) {
            cleanup();
            return st;
        }
        e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return fail_hip(e, "sampled forward");
        // requested order, repeats included
        std::vector<int32_t> rows((size_t)nreq * n);
        e = hipMemcpy(rows.data(), outc, sizeof(int32_t) * rows.size(), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return fail_hip(e, "sampled forward: copy out");
        for (int32_t i = 0; i < count; ++i)
            std::copy(rows.begin() + (size_t)row_of[i] * n, rows.begin() + (size_t)(row_of[i] + 1) * n,
                      h_out + (size_t)i * n);
    }
    cleanup();
    return BC_OK;
}
