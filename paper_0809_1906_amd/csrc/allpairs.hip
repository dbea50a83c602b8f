// All-pairs betweenness by Algorithm 2 (Sec. 4.2.1, the backward pass from
// all-pairs distances): with the distance matrix D and the path-count matrix
// Lambda of every pair, each vertex v sums, over ordered pairs (s,t) with
// s != v != t and d(s,t) = d(s,v) + d(v,t),
//     BC(v) += lambda_sv * lambda_vt / lambda_st,
// with no dependencies at all.  The context's forward kernels (those bc_run
// uses; the batched forms run their forward only) fill D and Lambda row by
// row, so the triple sum is an independent check of the forward outputs and of
// the Brandes backward.
//
// The context's forward kernels write D (int32, -1 = unreachable) and Lambda
// (uint64) [n][n], row = source, internal numbering.  A preparation pass turns
// them into
//   Dp  uint32 [n][ld], ld = n rounded up to 64: d(s,t) where 0 < d, else FAR
//       (t = s, t unreachable, and the padding columns)
//   R   double [n][n]: 1 / lambda_st where 0 < d(s,t), else 0
// The graph is undirected, so every matrix is symmetric: d(v,t) is row t of Dp
// and lambda_vt is row v of Lambda.
//
// The mask d(s,v) + d(v,t) = d(s,t) holds for a small share of triples (about
// (L - 1) / n of them for mean distance L), so the sum is organised around
// testing it cheaply.  A block takes VT vertices v and SC sources s; each
// thread owns targets t and keeps d(v,t) for its VT vertices in registers; per
// source the VT distances d(s,v) are uniform across the wave and come in by
// scalar loads.  A triple costs one three-operand add, x = d(s,v) + d(v,t) -
// d(s,t) (mod 2^32), and half a three-operand minimum; a group of 8 vertices is
// tested once, by a ballot on its minimum.  Groups with a hit (x = 0) are
// queued and their terms added into the block's LDS accumulators later.  FAR = 2^31 makes
// the one compare exact: real distances are below 2^31, so a sum of two stays
// below 2^32, FAR plus a real distance lies in (2^31, 2^32), FAR + FAR wraps to
// 0, and no Dp entry is 0; x = 0 is the same test.  A sum of two real distances
// equal to 2^31 could meet dst = FAR; R is 0 there, so such a term adds nothing.
#include "bc_internal.h"

#include <type_traits>

namespace {

constexpr int AT = 256;               // threads per block
constexpr int VT = 64;                // vertices v per block
constexpr int SC = 256;               // sources s per block
constexpr uint32_t FAR = 0x80000000u; // t = s, no path, or padding

__global__ __launch_bounds__(256) void k_alg2_prep(int32_t n, int32_t ld, const int32_t *__restrict__ D,
                                                   const uint64_t *__restrict__ Lam, uint32_t *__restrict__ Dp,
                                                   double *__restrict__ R) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (size_t)n * ld) return;
    const int32_t s = (int32_t)(i / ld), c = (int32_t)(i % ld);
    if (c < n) {
        const size_t k = (size_t)s * n + c;
        const int32_t d = D[k];
        Dp[i] = d > 0 ? (uint32_t)d : FAR;
        R[k] = d > 0 ? 1.0 / (double)Lam[k] : 0.0;
    } else {
        Dp[i] = FAR;
    }
}

// Deferred hits: a lane whose group of 8 vertices has a hit appends the code
// (source slot << 3 | group) and -d(s,t) to its own queue in LDS; the queue is
// drained after the source loop, or when some lane of the wave could overflow
// it.  The drain recomputes the 8 tests of each queued group from rows s and t
// (cached) and, for every hit, loads 1/lambda_st, lambda_sv and lambda_vt (a
// count at distance 1 is 1 and is not loaded); its loads are independent
// across lanes and records, so their latency overlaps instead of stalling the
// test loop.
constexpr int QK = 24; // queue entries per thread

__global__ __launch_bounds__(AT) void k_alg2(int32_t n, int32_t ld, const uint32_t *__restrict__ Dp,
                                             const double *__restrict__ R, const uint64_t *__restrict__ Lam,
                                             double *__restrict__ bc) {
    __shared__ double s_acc[VT];
    __shared__ uint16_t s_q[QK][AT];  // source slot << 3 | group
    __shared__ uint32_t s_nd[QK][AT]; // -d(s,t)
    const int tid = threadIdx.x;
    if (tid < VT) s_acc[tid] = 0.0;
    __syncthreads();
    const int32_t v0 = blockIdx.x * VT, sa = blockIdx.y * SC;
    const int32_t ns = min(SC, n - sa);
    // the queued groups of target t: recompute their 8 tests from the record's
    // -d(s,t) and the cached rows s and t, then add the hits.  After the source
    // loop, where d(v,t) no longer occupies registers, several records go per
    // step, so that their loads are in flight together; inside it, one.
    auto drain = [&](int32_t t, int32_t cnt, auto unroll) {
        constexpr int U = decltype(unroll)::value;
        const uint32_t *trow = Dp + (size_t)t * ld + v0;
        const uint64_t *ltrow = Lam + (size_t)t * n + v0;
        for (int32_t i = 0; i < cnt; i += U) {
            int32_t sv[U], gv[U];
            uint32_t ndv[U];
            uint4 p0[U], p1[U], q0[U], q1[U];
            double rv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t e = i + u < cnt ? i + u : i; // a repeat is loaded, not added
                const uint32_t code = s_q[e][tid];
                sv[u] = sa + (int32_t)(code >> 3);
                gv[u] = (int32_t)(code & 7);
                ndv[u] = s_nd[e][tid];
                const uint4 *sp = reinterpret_cast<const uint4 *>(Dp + (size_t)sv[u] * ld + v0 + 8 * gv[u]);
                const uint4 *tp = reinterpret_cast<const uint4 *>(trow + 8 * gv[u]);
                p0[u] = sp[0];
                p1[u] = sp[1];
                q0[u] = tp[0];
                q1[u] = tp[1];
                rv[u] = R[(size_t)sv[u] * n + t];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (i + u >= cnt) break;
                const uint32_t ds[8] = {p0[u].x, p0[u].y, p0[u].z, p0[u].w, p1[u].x, p1[u].y, p1[u].z, p1[u].w};
                const uint32_t dt[8] = {q0[u].x, q0[u].y, q0[u].z, q0[u].w, q1[u].x, q1[u].y, q1[u].z, q1[u].w};
                const uint64_t *lsrow = Lam + (size_t)sv[u] * n + v0;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    if (ds[k] + dt[k] + ndv[u] == 0) {
                        // a hit has d(s,v) < FAR, so v < n; a count at
                        // distance 1 is 1 and is not loaded
                        const int32_t j = 8 * gv[u] + k;
                        const double ls = ds[k] == 1 ? 1.0 : (double)lsrow[j];
                        const double lt = dt[k] == 1 ? 1.0 : (double)ltrow[j];
                        unsafeAtomicAdd(&s_acc[j], ls * lt * rv[u]);
                    }
                }
            }
        }
    };
    for (int32_t t = tid; t < n; t += AT) {
        uint32_t dvt[VT];
        const uint4 *row = reinterpret_cast<const uint4 *>(Dp + (size_t)t * ld + v0);
#pragma unroll
        for (int q = 0; q < VT / 4; ++q) {
            const uint4 x = row[q];
            dvt[4 * q] = x.x;
            dvt[4 * q + 1] = x.y;
            dvt[4 * q + 2] = x.z;
            dvt[4 * q + 3] = x.w;
        }
        int32_t cnt = 0;
        uint32_t dnext = Dp[(size_t)sa * ld + t]; // d(s,t), one source ahead
        for (int32_t sl = 0; sl < ns; ++sl) {
            const int32_t s = sa + sl;
            const uint32_t *srow = Dp + (size_t)s * ld; // uniform
            // -d(s,t), opaque so that x below stays one three-operand add
            uint32_t ndst = 0u - dnext;
            __asm__ volatile("" : "+v"(ndst));
            if (sl + 1 < ns) dnext = srow[(size_t)ld + t];
#pragma unroll
            for (int h = 0; h < VT / 32; ++h) {
                // d(s,v) for 32 vertices: uniform, loaded before any test
                const uint4 *sq = reinterpret_cast<const uint4 *>(srow + v0 + 32 * h);
                uint32_t dsv[32];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const uint4 x = sq[q];
                    dsv[4 * q] = x.x;
                    dsv[4 * q + 1] = x.y;
                    dsv[4 * q + 2] = x.z;
                    dsv[4 * q + 3] = x.w;
                }
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    // x = d(s,v) + d(v,t) - d(s,t) (mod 2^32) for 8 vertices;
                    // the group is tested once, by the minimum
                    uint32_t mn = 0xffffffffu;
#pragma unroll
                    for (int k = 0; k < 8; ++k) mn = min(mn, dsv[8 * g + k] + dvt[32 * h + 8 * g + k] + ndst);
                    // hits are rare: keep the no-hit path a fall-through
                    if (__builtin_expect(__builtin_amdgcn_ballot_w64(mn == 0) != 0, 0)) {
                        if (__builtin_expect(__builtin_amdgcn_ballot_w64(cnt == QK) != 0, 0)) {
                            drain(t, cnt, std::integral_constant<int, 1>());
                            cnt = 0;
                        }
                        if (mn == 0) {
                            s_q[cnt][tid] = (uint16_t)((sl << 3) | (4 * h + g));
                            s_nd[cnt][tid] = ndst;
                            ++cnt;
                        }
                    }
                }
            }
        }
        drain(t, cnt, std::integral_constant<int, 4>());
    }
    __syncthreads();
    if (tid < VT && v0 + tid < n && s_acc[tid] != 0.0) unsafeAtomicAdd(&bc[v0 + tid], s_acc[tid]);
}

__global__ __launch_bounds__(256) void k_iota_from(int32_t *__restrict__ ids, int32_t first, int32_t count) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < count) ids[i] = first + i;
}

__global__ __launch_bounds__(256) void k_zero_f64(double *__restrict__ x, int32_t count) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < count) x[i] = 0.0;
}

} // namespace

bc_status allpairs_bc(bc_ctx *ctx, double *bc_internal) {
    const int32_t n = ctx->n;
    if (n == 0) return BC_OK;
    const int32_t ld = (n + VT - 1) / VT * VT;
    const size_t nn = (size_t)n * n;
    const bool plain = ctx->form == BC_FORM_PLAIN_FP64;
    const int32_t chunk = plain ? std::min(n, 4096) : std::min(n, ctx->sp.batch);
    int32_t *D = (int32_t *)bc_dalloc(ctx, nn * sizeof(int32_t));
    uint64_t *Lam = (uint64_t *)bc_dalloc(ctx, nn * sizeof(uint64_t));
    // the plain sweep dumps dependencies too; the batched forms run the
    // forward only
    double *dtmp = plain ? (double *)bc_dalloc(ctx, (size_t)chunk * n * sizeof(double)) : nullptr;
    int32_t *src = (int32_t *)bc_dalloc(ctx, (size_t)chunk * sizeof(int32_t));
    uint32_t *Dp = nullptr;
    double *R = nullptr;
    auto cleanup = [&]() {
        bc_dfree(ctx, D);
        bc_dfree(ctx, Lam);
        bc_dfree(ctx, dtmp);
        bc_dfree(ctx, src);
        bc_dfree(ctx, Dp);
        bc_dfree(ctx, R);
    };
    if (!D || !Lam || (plain && !dtmp) || !src) {
        cleanup();
        return bc_fail(ctx, BC_ERR_NOMEM, "all pairs: allocation of D and Lambda failed");
    }
    // rows of D and Lambda: every source in internal order, one batch at a time
    for (int32_t s0 = 0; s0 < n; s0 += chunk) {
        const int32_t cnt = std::min(chunk, n - s0);
        hipLaunchKernelGGL(k_iota_from, dim3((cnt + 255) / 256), dim3(256), 0, ctx->stream, src, s0, cnt);
        const size_t row = (size_t)s0 * n;
        bc_status st = plain ? plain_run(ctx, src, cnt, false, dtmp, D + row, Lam + row)
                             : sparse_dump(ctx, src, cnt, D + row, Lam + row, nullptr);
        if (st != BC_OK) {
            cleanup();
            return st;
        }
    }
    bc_dfree(ctx, dtmp);
    dtmp = nullptr;
    Dp = (uint32_t *)bc_dalloc(ctx, (size_t)n * ld * sizeof(uint32_t));
    R = (double *)bc_dalloc(ctx, nn * sizeof(double));
    if (!Dp || !R) {
        cleanup();
        return bc_fail(ctx, BC_ERR_NOMEM, "all pairs: allocation of the prepared matrices failed");
    }
    const size_t cells = (size_t)n * ld;
    hipLaunchKernelGGL(k_alg2_prep, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, ctx->stream, n, ld, D, Lam,
                       Dp, R);
    hipLaunchKernelGGL(k_zero_f64, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, bc_internal, n);
    const dim3 grid(ld / VT, (n + SC - 1) / SC);
    {
        LaunchTimer tm(ctx, "all_pairs");
        hipLaunchKernelGGL(k_alg2, grid, dim3(AT), 0, ctx->stream, n, ld, Dp, R, Lam, bc_internal);
        tm.done();
    }
    const hipError_t e = hipGetLastError();
    const hipError_t sy = hipStreamSynchronize(ctx->stream);
    cleanup();
    if (e != hipSuccess) return bc_hip(ctx, e, "k_alg2");
    if (sy != hipSuccess) return bc_hip(ctx, sy, "all pairs");
    return BC_OK;
}
