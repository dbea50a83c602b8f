// Batched sparse form: B sources at once (B a multiple of 64), unit weights.
//
// State is batch-minor.  For level l the frontier is a bitmap
// front[l][v][q] (uint64): bit b of word q is set iff d(s_{64q+b}, v) = l,
// and any[l] holds one bit per vertex: the OR of its B frontier bits.
// Path counts sigma[v][64q+b] are uint64 and c(v) = (1 + delta(v)) / sigma(v)
// is stored as FP32 in cval[v][64q+b]; all sums are formed in FP64 registers.
//
// One wave handles one (row segment, word) pair; lane b is source 64q+b, so
// every gather of a neighbour's sigma or c row is one coalesced 512 B (256 B)
// read.  The wave loads 64 neighbour ids at once, drops those whose any[] bit
// is clear, gathers the frontier words of the rest, keeps the neighbours whose
// word intersects its own mask (ballot) and gathers rows for those only, four
// at a time.  Rows longer than split_degree arcs (hubs) are cut into segments
// that run on separate waves; their partial sums meet in a small per-hub
// scratch array through atomics, and the last segment wave to finish completes
// the hub.
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
constexpr int WPB = SB / 64; // waves per block
constexpr int CSLOTS = 64;   // frontier counters per level, one per 128 B line
constexpr int CSTRIDE = 32;  // uint32 per counter slot

__device__ __forceinline__ int32_t rl32(int32_t x, int j) { return __builtin_amdgcn_readlane(x, j); }
__device__ __forceinline__ uint64_t rl64(uint64_t x, int j) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, j);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ int pop_lowest(uint64_t &m) {
    const int j = __ffsll((unsigned long long)m) - 1;
    m &= m - 1;
    return j;
}

// Graph-side description shared by the level kernels.
struct Topo {
    int32_t n, NW, B;
    const int32_t *rp, *col;
    const int32_t *heavy_id;                 // [n]: index among heavy rows, -1 for light rows
    const int32_t *seg_v, *seg_beg, *seg_end; // [nseg]: segments of heavy rows
    int32_t nseg;
    const int32_t *heavy_v;                  // [nheavy]
    const int32_t *heavy_nseg;               // [nheavy]: segments per heavy row
    int32_t nheavy;
};

// Sum over arcs [beg, end) of row w of sigma(v, 64q+lane) for neighbours v
// whose frontier word intersects U at this lane.  Returns the sum; ovf is set
// when a uint64 addition wrapped.
__device__ __forceinline__ uint64_t fwd_scan(const Topo &t, int32_t beg, int32_t end, int q, uint64_t U,
                                             const uint32_t *__restrict__ any_cur,
                                             const uint64_t *__restrict__ fcur,
                                             const uint64_t *__restrict__ sigma, int lane, bool &ovf) {
    const uint64_t *sig_q = sigma + (size_t)q * 64 + lane;
    uint64_t acc = 0;
    for (int32_t base = beg; base < end; base += 64) {
        const int32_t e = base + lane;
        int32_t v = 0;
        uint64_t f = 0;
        if (e < end) {
            v = t.col[e];
            if ((any_cur[v >> 5] >> (v & 31)) & 1) f = fcur[(size_t)v * t.NW + q] & U;
        }
        uint64_t act = __ballot(f != 0);
        while (act) {
            const int j0 = pop_lowest(act);
            const int j1 = act ? pop_lowest(act) : -1;
            const int j2 = act ? pop_lowest(act) : -1;
            const int j3 = act ? pop_lowest(act) : -1;
            uint64_t x0 = 0, x1 = 0, x2 = 0, x3 = 0;
            {
                const uint64_t fj = rl64(f, j0);
                if ((fj >> lane) & 1) x0 = sig_q[(size_t)rl32(v, j0) * t.B];
            }
            if (j1 >= 0) {
                const uint64_t fj = rl64(f, j1);
                if ((fj >> lane) & 1) x1 = sig_q[(size_t)rl32(v, j1) * t.B];
            }
            if (j2 >= 0) {
                const uint64_t fj = rl64(f, j2);
                if ((fj >> lane) & 1) x2 = sig_q[(size_t)rl32(v, j2) * t.B];
            }
            if (j3 >= 0) {
                const uint64_t fj = rl64(f, j3);
                if ((fj >> lane) & 1) x3 = sig_q[(size_t)rl32(v, j3) * t.B];
            }
            uint64_t s = acc + x0;
            ovf |= s < acc;
            acc = s;
            s = acc + x1;
            ovf |= s < acc;
            acc = s;
            s = acc + x2;
            ovf |= s < acc;
            acc = s;
            s = acc + x3;
            ovf |= s < acc;
            acc = s;
        }
    }
    return acc;
}

// Sum over arcs [beg, end) of row v of c(w, 64q+lane) for neighbours w whose
// next-level word intersects F at this lane.
__device__ __forceinline__ double bwd_scan(const Topo &t, int32_t beg, int32_t end, int q, uint64_t F,
                                           const uint32_t *__restrict__ any_next,
                                           const uint64_t *__restrict__ fnext,
                                           const float *__restrict__ cval, int lane) {
    const float *c_q = cval + (size_t)q * 64 + lane;
    double acc = 0.0;
    for (int32_t base = beg; base < end; base += 64) {
        const int32_t e = base + lane;
        int32_t w = 0;
        uint64_t g = 0;
        if (e < end) {
            w = t.col[e];
            if ((any_next[w >> 5] >> (w & 31)) & 1) g = fnext[(size_t)w * t.NW + q] & F;
        }
        uint64_t act = __ballot(g != 0);
        while (act) {
            const int j0 = pop_lowest(act);
            const int j1 = act ? pop_lowest(act) : -1;
            const int j2 = act ? pop_lowest(act) : -1;
            const int j3 = act ? pop_lowest(act) : -1;
            float x0 = 0.f, x1 = 0.f, x2 = 0.f, x3 = 0.f;
            {
                const uint64_t gj = rl64(g, j0);
                if ((gj >> lane) & 1) x0 = c_q[(size_t)rl32(w, j0) * t.B];
            }
            if (j1 >= 0) {
                const uint64_t gj = rl64(g, j1);
                if ((gj >> lane) & 1) x1 = c_q[(size_t)rl32(w, j1) * t.B];
            }
            if (j2 >= 0) {
                const uint64_t gj = rl64(g, j2);
                if ((gj >> lane) & 1) x2 = c_q[(size_t)rl32(w, j2) * t.B];
            }
            if (j3 >= 0) {
                const uint64_t gj = rl64(g, j3);
                if ((gj >> lane) & 1) x3 = c_q[(size_t)rl32(w, j3) * t.B];
            }
            acc += (double)x0;
            acc += (double)x1;
            acc += (double)x2;
            acc += (double)x3;
        }
    }
    return acc;
}

// delta(v,b) = sigma(v,b) * acc; c(v,b) = (1 + delta) / sigma; BC(v) += sum of delta
// over this wave's lanes whose source is not v.
__device__ __forceinline__ void bwd_finalize(int32_t v, int q, uint64_t F, double acc, int lane, int B,
                                             const uint64_t *__restrict__ sigma, float *__restrict__ cval,
                                             const int32_t *__restrict__ src_lane, double *__restrict__ bc,
                                             double *__restrict__ delta_dump, int accumulate) {
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

__global__ __launch_bounds__(SB) void k_sp_clear(uint64_t *__restrict__ a, uint64_t *__restrict__ b, size_t words,
                                                 uint32_t *__restrict__ any_all, size_t any_total,
                                                 uint32_t *__restrict__ counts, int32_t count_words) {
    const size_t tid = (size_t)blockIdx.x * SB + threadIdx.x, stride = (size_t)gridDim.x * SB;
    for (size_t i = tid; i < words; i += stride) {
        a[i] = 0;
        b[i] = 0;
    }
    for (size_t i = tid; i < any_total; i += stride) any_all[i] = 0;
    for (size_t i = tid; i < (size_t)count_words; i += stride) counts[i] = 0;
}

__global__ __launch_bounds__(SB) void k_sp_seed(const int32_t *__restrict__ src, int32_t count, int32_t B, int32_t NW,
                                                uint64_t *front0, uint64_t *visited, uint64_t *sigma,
                                                int32_t *src_lane, uint32_t *any0) {
    const int32_t b = blockIdx.x * SB + threadIdx.x;
    if (b >= B) return;
    const int32_t s = b < count ? src[b] : -1;
    src_lane[b] = s;
    if (s >= 0) {
        const unsigned long long bit = 1ull << (b & 63);
        atomicOr((unsigned long long *)&front0[(size_t)s * NW + (b >> 6)], bit);
        atomicOr((unsigned long long *)&visited[(size_t)s * NW + (b >> 6)], bit);
        atomicOr(&any0[s >> 5], 1u << (s & 31));
        sigma[(size_t)s * B + b] = 1;
    }
}

// Whether level l (l >= 1) has any vertex: any of the CSLOTS counters of the
// kernel that produced it is non-zero.  Read by one wave, shared through LDS.
__device__ __forceinline__ bool level_nonempty(const uint32_t *__restrict__ cnt_in, uint32_t *s_flag) {
    if (cnt_in == nullptr) return true;
    if (threadIdx.x < 64) {
        const uint32_t x = threadIdx.x < CSLOTS ? cnt_in[threadIdx.x * CSTRIDE] : 0u;
        const uint64_t nz = __ballot(x != 0);
        if (threadIdx.x == 0) *s_flag = nz != 0;
    }
    __syncthreads();
    return *s_flag != 0;
}

// Last-arriver protocol for split rows: every segment wave of (heavy row h,
// word q) adds its partial sums into hacc with device-scope atomics, waits
// until they have completed, then counts itself in arrive[h][q]; the wave
// that brings the count to the row's segment total resets the counter and
// completes the row, reading hacc with device-scope atomic loads.  hacc and
// arrive are touched only by device-scope atomics, so completion order is all
// the protocol needs: no cache write-back fence.
__device__ __forceinline__ void wait_memory() { __asm__ __volatile__("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ __forceinline__ bool last_arriver(uint32_t *arrive, int32_t total, int lane) {
    wait_memory();
    uint32_t old = 0;
    if (lane == 0) old = atomicAdd(arrive, 1u);
    old = (uint32_t)__builtin_amdgcn_readfirstlane((int)old);
    if (old + 1 != (uint32_t)total) return false;
    if (lane == 0) __hip_atomic_store(arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// Forward level l -> l+1.  Light rows complete in their wave; split rows
// complete in the last segment wave to arrive.  Marks any_next and the level
// counters; exits at once when level l is empty (speculative launch).
__global__ __launch_bounds__(SB) void k_fwd_pull(Topo t, const uint32_t *__restrict__ cnt_in,
                                                 const uint32_t *__restrict__ any_cur,
                                                 const uint64_t *__restrict__ fcur, uint64_t *__restrict__ fnext,
                                                 uint64_t *__restrict__ visited, uint64_t *__restrict__ sigma,
                                                 unsigned long long *__restrict__ hacc, uint32_t *__restrict__ arrive,
                                                 uint32_t *__restrict__ any_next, uint32_t *__restrict__ cnt_out,
                                                 uint32_t *__restrict__ status) {
    __shared__ uint32_t s_flag;
    __shared__ uint32_t s_any[2];
    __shared__ uint32_t s_cnt;
    if (!level_nonempty(cnt_in, &s_flag)) return;
    if (threadIdx.x == 0) {
        s_any[0] = s_any[1] = 0;
        s_cnt = 0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t wid0 = (int64_t)blockIdx.x * WPB;
    const int64_t wid = wid0 + (threadIdx.x >> 6);
    const int64_t nlight = (int64_t)t.n * t.NW;
    const int32_t wbase = (int32_t)(min(wid0, nlight - 1) / t.NW) >> 5; // any word of the block's first vertex
    bool ovf = false;
    if (wid < nlight) {
        const int32_t w = (int32_t)(wid / t.NW), q = (int32_t)(wid - (int64_t)w * t.NW);
        if (t.heavy_id[w] < 0) {
            const uint64_t vis = visited[wid];
            const uint64_t U = ~vis;
            uint64_t out = 0;
            if (U != 0) {
                const uint64_t acc = fwd_scan(t, t.rp[w], t.rp[w + 1], q, U, any_cur, fcur, sigma, lane, ovf);
                out = __ballot(acc != 0);
                if (acc != 0) sigma[(size_t)w * t.B + (size_t)q * 64 + lane] = acc;
            }
            if (lane == 0) {
                fnext[wid] = out;
                if (out) {
                    visited[wid] = vis | out;
                    atomicOr(&s_any[(w >> 5) - wbase], 1u << (w & 31));
                    atomicAdd(&s_cnt, 1u);
                }
            }
        }
    } else if (wid < nlight + (int64_t)t.nseg * t.NW) {
        const int64_t k = (wid - nlight) / t.NW;
        const int32_t q = (int32_t)(wid - nlight - k * t.NW);
        const int32_t w = t.seg_v[k];
        const int32_t h = t.heavy_id[w];
        const size_t vw = (size_t)w * t.NW + q;
        const uint64_t vis = visited[vw];
        const uint64_t U = ~vis;
        if (U == 0) {
            if (lane == 0 && t.seg_beg[k] == t.rp[w]) fnext[vw] = 0;
        } else {
            const size_t hi = (size_t)h * t.B + (size_t)q * 64 + lane;
            const uint64_t acc = fwd_scan(t, t.seg_beg[k], t.seg_end[k], q, U, any_cur, fcur, sigma, lane, ovf);
            if (acc != 0) {
                const unsigned long long old = atomicAdd(&hacc[hi], (unsigned long long)acc);
                ovf |= old + acc < old;
            }
            if (last_arriver(&arrive[(size_t)h * t.NW + q], t.heavy_nseg[h], lane)) {
                const uint64_t x = __hip_atomic_load(&hacc[hi], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (x != 0) {
                    __hip_atomic_store(&hacc[hi], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    sigma[(size_t)w * t.B + (size_t)q * 64 + lane] = x;
                }
                const uint64_t out = __ballot(x != 0);
                if (lane == 0) {
                    fnext[vw] = out;
                    if (out) {
                        visited[vw] = vis | out;
                        atomicOr(&any_next[w >> 5], 1u << (w & 31));
                        atomicAdd(&s_cnt, 1u);
                    }
                }
            }
        }
    }
    if (__any(ovf) && lane == 0) atomicOr(status, (uint32_t)BC_DEV_SIGMA_OVERFLOW);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_any[0]) atomicOr(&any_next[wbase], s_any[0]);
        if (s_any[1]) atomicOr(&any_next[wbase + 1], s_any[1]);
        if (s_cnt) atomicAdd(&cnt_out[(blockIdx.x % CSLOTS) * CSTRIDE], s_cnt);
    }
}

// Backward level l.  Light rows complete in their wave; split rows in the last
// segment wave to arrive.  fnext = nullptr at the deepest level.
__global__ __launch_bounds__(SB) void k_bwd_pull(Topo t, const uint64_t *__restrict__ fcur,
                                                 const uint32_t *__restrict__ any_next,
                                                 const uint64_t *__restrict__ fnext,
                                                 const uint64_t *__restrict__ sigma, float *__restrict__ cval,
                                                 const int32_t *__restrict__ src_lane, double *__restrict__ bc,
                                                 double *__restrict__ hacc, uint32_t *__restrict__ arrive,
                                                 double *__restrict__ delta_dump, int accumulate) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * WPB + (threadIdx.x >> 6);
    const int64_t nlight = (int64_t)t.n * t.NW;
    if (wid < nlight) {
        const uint64_t F = fcur[wid];
        if (F == 0) return;
        const int32_t v = (int32_t)(wid / t.NW), q = (int32_t)(wid - (int64_t)v * t.NW);
        if (t.heavy_id[v] >= 0) return;
        const double acc = fnext ? bwd_scan(t, t.rp[v], t.rp[v + 1], q, F, any_next, fnext, cval, lane) : 0.0;
        bwd_finalize(v, q, F, acc, lane, t.B, sigma, cval, src_lane, bc, delta_dump, accumulate);
    } else if (wid < nlight + (int64_t)t.nseg * t.NW) {
        const int64_t k = (wid - nlight) / t.NW;
        const int32_t q = (int32_t)(wid - nlight - k * t.NW);
        const int32_t v = t.seg_v[k];
        const uint64_t F = fcur[(size_t)v * t.NW + q];
        if (F == 0) return;
        const int32_t h = t.heavy_id[v];
        const size_t hi = (size_t)h * t.B + (size_t)q * 64 + lane;
        const double acc = fnext ? bwd_scan(t, t.seg_beg[k], t.seg_end[k], q, F, any_next, fnext, cval, lane) : 0.0;
        if (acc != 0.0) unsafeAtomicAdd(&hacc[hi], acc);
        if (last_arriver(&arrive[(size_t)h * t.NW + q], t.heavy_nseg[h], lane)) {
            double x = 0.0;
            if ((F >> lane) & 1) {
                x = __hip_atomic_load(&hacc[hi], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (x != 0.0) __hip_atomic_store(&hacc[hi], 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            bwd_finalize(v, q, F, x, lane, t.B, sigma, cval, src_lane, bc, delta_dump, accumulate);
        }
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

Topo topo(bc_ctx *ctx) {
    const SparseState &s = ctx->sp;
    Topo t;
    t.n = ctx->n;
    t.NW = s.words;
    t.B = s.batch;
    t.rp = ctx->row_ptr;
    t.col = ctx->col;
    t.heavy_id = s.heavy_id;
    t.seg_v = s.seg_v;
    t.seg_beg = s.seg_beg;
    t.seg_end = s.seg_end;
    t.nseg = s.nseg;
    t.heavy_v = s.heavy_v;
    t.heavy_nseg = s.heavy_nseg;
    t.nheavy = s.nheavy;
    return t;
}

inline int32_t any_words(const bc_ctx *ctx) { return (ctx->n + 31) >> 5; }

bc_status ensure_levels(bc_ctx *ctx, int32_t need) {
    SparseState &s = ctx->sp;
    if (need <= s.level_cap) return BC_OK;
    int32_t cap = std::max(s.level_cap * 2, need);
    const size_t aw = (size_t)any_words(ctx);
    const size_t cw = (size_t)CSLOTS * CSTRIDE;
    const size_t per_level = (size_t)ctx->n * s.words * sizeof(uint64_t) + aw * sizeof(uint32_t);
    const size_t budget = size_t(32) << 30;
    if ((size_t)cap * per_level > budget) {
        cap = need;
        if ((size_t)cap * per_level > budget)
            return bc_fail(ctx, BC_ERR_UNSUPPORTED,
                           "sparse form: the graph is too deep for per-level frontier bitmaps; use the plain form");
    }
    const size_t lvl_words = (size_t)ctx->n * s.words;
    uint64_t *nf = (uint64_t *)bc_dalloc(ctx, (size_t)cap * lvl_words * sizeof(uint64_t));
    uint32_t *na = (uint32_t *)bc_dalloc(ctx, (size_t)cap * aw * sizeof(uint32_t));
    uint32_t *nc = (uint32_t *)bc_dalloc(ctx, (size_t)cap * cw * sizeof(uint32_t));
    uint32_t *nh = nullptr;
    if (!nf || !na || !nc || hipHostMalloc((void **)&nh, (size_t)cap * cw * sizeof(uint32_t)) != hipSuccess) {
        bc_dfree(ctx, nf);
        bc_dfree(ctx, na);
        bc_dfree(ctx, nc);
        return bc_fail(ctx, BC_ERR_NOMEM, "sparse form: frontier allocation failed");
    }
    const int32_t old = s.level_cap;
    if (s.front) {
        BC_HIP(ctx, hipMemcpyAsync(nf, s.front, (size_t)old * lvl_words * sizeof(uint64_t), hipMemcpyDeviceToDevice,
                                   ctx->stream));
        BC_HIP(ctx, hipMemcpyAsync(na, s.any, (size_t)old * aw * sizeof(uint32_t), hipMemcpyDeviceToDevice, ctx->stream));
        BC_HIP(ctx, hipMemcpyAsync(nc, s.counts, (size_t)old * cw * sizeof(uint32_t), hipMemcpyDeviceToDevice, ctx->stream));
    }
    BC_HIP(ctx, hipMemsetAsync(na + (size_t)old * aw, 0, (size_t)(cap - old) * aw * sizeof(uint32_t), ctx->stream));
    BC_HIP(ctx, hipMemsetAsync(nc + (size_t)old * cw, 0, (size_t)(cap - old) * cw * sizeof(uint32_t), ctx->stream));
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (s.front) {
        bc_dfree(ctx, s.front);
        bc_dfree(ctx, s.any);
        bc_dfree(ctx, s.counts);
        hipHostFree(s.counts_host);
    }
    s.front = nf;
    s.any = na;
    s.counts = nc;
    s.counts_host = nh;
    s.level_cap = cap;
    return BC_OK;
}

// One batch of up to B sources; *nlev_out receives the number of non-empty
// levels.  Forward levels are launched ahead of the host knowing whether they
// are needed (as many as the previous batch used); a kernel whose input level
// is empty exits at once, and the host reads all level counters with one
// synchronisation per batch.
bc_status run_batch(bc_ctx *ctx, const int32_t *d_src, int32_t count, bool accumulate, int32_t *nlev_out) {
    SparseState &s = ctx->sp;
    const int32_t n = ctx->n, NW = s.words, B = s.batch;
    const size_t words = (size_t)n * NW;
    const int32_t aw = any_words(ctx);
    const size_t cw = (size_t)CSLOTS * CSTRIDE;
    const int pull_blocks = (int)(((int64_t)(n + s.nseg) * NW + WPB - 1) / WPB);
    const int32_t guess = std::max(s.depth_guess, 2);
    bc_status st = ensure_levels(ctx, guess + 1);
    if (st != BC_OK) return st;
    const Topo t = topo(ctx);
    {
        LaunchTimer tm(ctx, "batch_init");
        const int blocks = (int)std::min<size_t>((words + SB - 1) / SB, 8192);
        hipLaunchKernelGGL(k_sp_clear, dim3(std::max(blocks, 1)), dim3(SB), 0, ctx->stream, s.front, s.visited, words,
                           s.any, (size_t)s.level_cap * aw, s.counts, (int32_t)((size_t)s.level_cap * cw));
        hipLaunchKernelGGL(k_sp_seed, dim3((B + SB - 1) / SB), dim3(SB), 0, ctx->stream, d_src, count, B, NW, s.front,
                           s.visited, s.sigma, s.src, s.any);
        tm.done();
        BC_HIP(ctx, hipGetLastError());
    }
    int32_t launched = 0, nlev = -1;
    while (nlev < 0) {
        const int32_t target = launched == 0 ? guess : launched + 4;
        st = ensure_levels(ctx, target + 1);
        if (st != BC_OK) return st;
        for (int32_t l = launched; l < target; ++l) {
            LaunchTimer tm(ctx, "fwd_pull");
            hipLaunchKernelGGL(k_fwd_pull, dim3(pull_blocks), dim3(SB), 0, ctx->stream, t,
                               l == 0 ? (const uint32_t *)nullptr : s.counts + (size_t)l * cw, s.any + (size_t)l * aw,
                               s.front + (size_t)l * words, s.front + (size_t)(l + 1) * words, s.visited, s.sigma,
                               (unsigned long long *)s.hacc, s.arrive, s.any + (size_t)(l + 1) * aw,
                               s.counts + (size_t)(l + 1) * cw, ctx->status);
            tm.done();
        }
        BC_HIP(ctx, hipGetLastError());
        BC_HIP(ctx, hipMemcpyAsync(s.counts_host + cw, s.counts + cw, (size_t)target * cw * sizeof(uint32_t),
                                   hipMemcpyDeviceToHost, ctx->stream));
        BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
        for (int32_t l = 1; l <= target && nlev < 0; ++l) {
            uint64_t total = 0;
            for (int i = 0; i < CSLOTS; ++i) total += s.counts_host[(size_t)l * cw + (size_t)i * CSTRIDE];
            if (total == 0) nlev = l;
        }
        launched = target;
    }
    s.depth_guess = nlev;
    const int32_t lowest = accumulate ? 1 : 0;
    double *ddump = accumulate ? nullptr : s.delta_dump;
    for (int32_t lv = nlev - 1; lv >= lowest; --lv) {
        const uint64_t *fcur = s.front + (size_t)lv * words;
        const bool deeper = lv + 1 < nlev;
        const uint64_t *fnext = deeper ? s.front + (size_t)(lv + 1) * words : nullptr;
        const uint32_t *anext = deeper ? s.any + (size_t)(lv + 1) * aw : nullptr;
        LaunchTimer tm(ctx, "bwd_pull");
        hipLaunchKernelGGL(k_bwd_pull, dim3(pull_blocks), dim3(SB), 0, ctx->stream, t, fcur, anext, fnext, s.sigma,
                           s.cval, s.src, ctx->bc, s.hacc, s.arrive, ddump, accumulate ? 1 : 0);
        tm.done();
    }
    BC_HIP(ctx, hipGetLastError());
    ctx->max_levels = std::max(ctx->max_levels, nlev);
    *nlev_out = nlev;
    return BC_OK;
}

} // namespace

bc_status sparse_prepare(bc_ctx *ctx, int32_t batch, int32_t split_degree) {
    SparseState &s = ctx->sp;
    s.batch = batch;
    s.words = batch / 64;
    s.split = split_degree > 0 ? split_degree : 256;
    const int32_t n = ctx->n;
    const size_t nn = (size_t)std::max(n, 1);
    // Heavy rows and their segments, from the host copy of row_ptr.
    const std::vector<int32_t> &rp = ctx->h_row_ptr;
    std::vector<int32_t> heavy_id((size_t)n, -1), heavy_v, heavy_nseg, seg_v, seg_beg, seg_end;
    for (int32_t v = 0; v < n; ++v) {
        const int32_t deg = rp[v + 1] - rp[v];
        if (deg <= s.split) continue;
        heavy_id[v] = (int32_t)heavy_v.size();
        heavy_v.push_back(v);
        heavy_nseg.push_back((deg + s.split - 1) / s.split);
        for (int32_t b = rp[v]; b < rp[v + 1]; b += s.split) {
            seg_v.push_back(v);
            seg_beg.push_back(b);
            seg_end.push_back(std::min(b + s.split, rp[v + 1]));
        }
    }
    s.nheavy = (int32_t)heavy_v.size();
    s.nseg = (int32_t)seg_v.size();
    s.heavy_id = (int32_t *)bc_dalloc(ctx, nn * sizeof(int32_t));
    s.heavy_v = (int32_t *)bc_dalloc(ctx, std::max<size_t>(heavy_v.size(), 1) * sizeof(int32_t));
    s.heavy_nseg = (int32_t *)bc_dalloc(ctx, std::max<size_t>(heavy_v.size(), 1) * sizeof(int32_t));
    s.arrive = (uint32_t *)bc_dalloc(ctx, std::max<size_t>(heavy_v.size(), 1) * s.words * sizeof(uint32_t));
    s.seg_v = (int32_t *)bc_dalloc(ctx, std::max<size_t>(seg_v.size(), 1) * sizeof(int32_t));
    s.seg_beg = (int32_t *)bc_dalloc(ctx, std::max<size_t>(seg_v.size(), 1) * sizeof(int32_t));
    s.seg_end = (int32_t *)bc_dalloc(ctx, std::max<size_t>(seg_v.size(), 1) * sizeof(int32_t));
    s.hacc = (double *)bc_dalloc(ctx, std::max<size_t>(heavy_v.size(), 1) * batch * sizeof(double));
    s.visited = (uint64_t *)bc_dalloc(ctx, nn * s.words * sizeof(uint64_t));
    s.sigma = (uint64_t *)bc_dalloc(ctx, nn * batch * sizeof(uint64_t));
    s.cval = (float *)bc_dalloc(ctx, nn * batch * sizeof(float));
    s.src = (int32_t *)bc_dalloc(ctx, batch * sizeof(int32_t));
    if (!s.heavy_id || !s.heavy_v || !s.heavy_nseg || !s.arrive || !s.seg_v || !s.seg_beg || !s.seg_end || !s.hacc || !s.visited || !s.sigma ||
        !s.cval || !s.src)
        return bc_fail(ctx, BC_ERR_NOMEM, "sparse form: state allocation failed");
    if (n > 0) BC_HIP(ctx, hipMemcpyAsync(s.heavy_id, heavy_id.data(), nn * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
    if (s.nheavy) {
        BC_HIP(ctx, hipMemcpyAsync(s.heavy_v, heavy_v.data(), heavy_v.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
        BC_HIP(ctx, hipMemcpyAsync(s.heavy_nseg, heavy_nseg.data(), heavy_v.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
        BC_HIP(ctx, hipMemcpyAsync(s.seg_v, seg_v.data(), seg_v.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
        BC_HIP(ctx, hipMemcpyAsync(s.seg_beg, seg_beg.data(), seg_v.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
        BC_HIP(ctx, hipMemcpyAsync(s.seg_end, seg_end.data(), seg_v.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
    }
    BC_HIP(ctx, hipMemsetAsync(s.arrive, 0, std::max<size_t>(heavy_v.size(), 1) * s.words * sizeof(uint32_t), ctx->stream));
    BC_HIP(ctx, hipMemsetAsync(s.hacc, 0, std::max<size_t>(heavy_v.size(), 1) * batch * sizeof(double), ctx->stream));
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream)); // host vectors above go out of scope
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
