// Batched sparse form: B sources at once (B = 64 NW, NW in {1, 2, 4, 8}),
// unit weights.
//
// State is batch-minor.  For level l the frontier is a bitmap
// front[l][v][q] (uint64): bit b of word q is set iff d(s_{64q+b}, v) = l,
// and any[l] holds one bit per vertex: the OR of its B frontier bits.
// Path counts sigma[v][64q+b] are exact integers, stored as uint32 while every
// count fits and as uint64 otherwise; c(v) = (1 + delta(v)) / sigma(v) is
// stored as FP32 in cval[v][64q+b]; all sums are formed in 64-bit registers.
//
// One wave handles one row (or one segment of a long row) for all NW words;
// lane b of word q is source 64q+b, so every gather of a neighbour's sigma or
// c row is a coalesced 256 B / 512 B read.  The wave loads 64 neighbour ids at
// once, drops those whose any[] bit is clear, loads the NW frontier words of
// the rest, keeps the neighbours whose words meet its own masks (ballot) and
// gathers rows for those only, several in flight at a time.  Rows longer than
// split_degree arcs (hubs) are cut into segments that run on separate waves;
// their partial sums meet in a small per-hub scratch array through atomics,
// and the last segment wave to finish completes the hub.
//
//   forward level l -> l+1 (pull):  for w with unvisited sources U,
//       sigma(w,b) = sum over neighbours v with bit b of front[l][v] & U of
//       sigma(v,b);  front[l+1][w] = bits where that sum is non-zero.
//       This is the level-synchronous search of Sec. 4 with the counting rule
//       lambda_sw = sum of lambda_sv over v in P_s(w) (Sec. 1.1).  Level 0 -> 1
//       is pushed from the sources instead (lambda = 1 at distance 1).
//   backward level l (pull):  for v with bits F = front[l][v],
//       delta(v,b) = sigma(v,b) * sum over neighbours w with bit b of
//       front[l+1][w] & F of c(w,b)      (Theorem 1.1; ParallelCompute of
//       Sec. 4.2.2 with the 1/lambda factor kept inside c);
//       BC(v) += sum over b with s_b != v of delta(v,b).
// Level 0 is never accumulated: there v is the source itself.
#include "bc_internal.h"

#include <algorithm>
#include <type_traits>

namespace {

constexpr int SB = 256;      // threads per block = 4 waves
constexpr int WPB = SB / 64; // waves per block
constexpr int GDEPTH = 8;    // row gathers issued back to back per wave

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
    int32_t n, B;
    const int32_t *rp, *col;
    const int32_t *heavy_id;                  // [n]: index among heavy rows, -1 for light rows
    const int32_t *seg_v, *seg_beg, *seg_end; // [nseg]: segments of heavy rows
    int32_t nseg;
    const int32_t *heavy_nseg;                // [nheavy]: segments per heavy row
};

// Which row (or row segment) wave `wid` serves.  Returns false when the wave
// has nothing to do (a heavy row in the light range, or past the end).
struct Item {
    int32_t v, beg, end, h;
    bool first; // the segment that starts the row (or a light row)
};
__device__ __forceinline__ bool item_of(const Topo &t, int64_t wid, Item &it) {
    if (wid < t.n) {
        it.v = (int32_t)wid;
        if (t.heavy_id[it.v] >= 0) return false;
        it.beg = t.rp[it.v];
        it.end = t.rp[it.v + 1];
        it.h = -1;
        it.first = true;
        return true;
    }
    const int64_t k = wid - t.n;
    if (k >= t.nseg) return false;
    it.v = t.seg_v[k];
    it.beg = t.seg_beg[k];
    it.end = t.seg_end[k];
    it.h = t.heavy_id[it.v];
    it.first = it.beg == t.rp[it.v];
    return true;
}

// Lane-distributed load of the NW words of a bitmap row, then broadcast.
template <int NW>
__device__ __forceinline__ void load_words(const uint64_t *__restrict__ row, int lane, uint64_t (&w)[NW]) {
    const uint64_t mine = lane < NW ? row[lane] : 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) w[q] = rl64(mine, q);
}

// Path counts are stored as uint32 while they fit (half the gather bytes); a
// count of 2^32 or more raises the need-wide flag and the batch is re-run with
// uint64 storage.
__device__ __forceinline__ void store_count(uint64_t *p, uint64_t x, bool &wide) { *p = x; }
__device__ __forceinline__ void store_count(uint32_t *p, uint64_t x, bool &wide) {
    wide |= x > 0xFFFFFFFFull;
    *p = (uint32_t)x;
}

// Sums of eight per-lane values over the wave by reduce-scatter: lanes trade
// halves of their values with the lanes 32, 16 and 8 apart (4 + 2 + 1
// shuffles), then finish the one value they keep over the lanes 4, 2 and 1
// apart.  Lane l ends with the wave sum of p[(l >> 3) & 7].
__device__ __forceinline__ double wave_sum8(const double (&p)[8], int lane) {
    double a[4], b[2];
    const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double keep = h5 ? p[i + 4] : p[i], send = h5 ? p[i] : p[i + 4];
        a[i] = keep + __shfl_xor(send, 32, 64);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double keep = h4 ? a[i + 2] : a[i], send = h4 ? a[i] : a[i + 2];
        b[i] = keep + __shfl_xor(send, 16, 64);
    }
    double y = (h3 ? b[1] : b[0]) + __shfl_xor(h3 ? b[0] : b[1], 8, 64);
    y += __shfl_xor(y, 4, 64);
    y += __shfl_xor(y, 2, 64);
    y += __shfl_xor(y, 1, 64);
    return y;
}

// Last-arriver protocol for split rows: every segment wave of heavy row h adds
// its partial sums into hacc with device-scope atomics, waits until they have
// completed, then counts itself in arrive[h]; the wave that brings the count to
// the row's segment total resets the counter and completes the row, reading
// hacc with device-scope atomic loads.  hacc and arrive are touched only by
// device-scope atomics, so completion order is all the protocol needs: no
// cache write-back fence.
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

// acc[q] += sum over arcs [beg, end) of sigma(v, 64q+lane) for neighbours v
// whose word q of the level-l frontier meets U[q] at this lane; sigma holds
// the counts as G.  UNIT: every count of level l is 1 (level 1: the source's
// neighbours, one path each in a simple graph), so the sum counts frontier
// bits and gathers no count row.
template <int NW, typename G, bool UNIT>
__device__ __forceinline__ void fwd_scan(const Topo &t, int32_t beg, int32_t end, const uint64_t (&U)[NW],
                                         const uint32_t *__restrict__ any_cur, const uint64_t *__restrict__ fcur,
                                         const G *__restrict__ sigma, int lane, uint64_t (&acc)[NW], bool &ovf) {
    constexpr int ARCS = NW >= GDEPTH ? 1 : GDEPTH / NW; // arcs per round, ARCS * NW gathers in flight
    const G *sig = sigma + lane;
    for (int32_t base = beg; base < end; base += 64) {
        const int32_t e = base + lane;
        int32_t v = 0;
        uint64_t f[NW];
#pragma unroll
        for (int q = 0; q < NW; ++q) f[q] = 0;
        if (e < end) {
            v = t.col[e];
            if ((any_cur[v >> 5] >> (v & 31)) & 1) {
#pragma unroll
                for (int q = 0; q < NW; ++q) f[q] = fcur[(size_t)v * NW + q] & U[q];
            }
        }
        uint64_t nz = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) nz |= f[q];
        uint64_t act = __ballot(nz != 0);
        if constexpr (UNIT) {
            while (act) {
                const int j = pop_lowest(act);
#pragma unroll
                for (int q = 0; q < NW; ++q) acc[q] += (rl64(f[q], j) >> lane) & 1;
            }
            continue;
        }
        // Straight-line loads, the lane's bit selecting after all are issued:
        // a load under a per-lane branch was compiled with a wait for its own
        // result, so the gathers of a round ran one after another.  An arc
        // slot past the last active arc, or a word with no source of this
        // lane's mask, reads row 0 instead: a valid, cached address whose
        // value is then dropped.
        using X = typename std::conditional<sizeof(G) == 8, uint64_t, uint32_t>::type;
        while (act) {
            X x[ARCS][NW];
            uint64_t m[ARCS][NW];
#pragma unroll
            for (int a = 0; a < ARCS; ++a) {
                const bool live = act != 0;
                const int j = live ? pop_lowest(act) : 0;
                const size_t row = live ? (size_t)rl32(v, j) * t.B : 0;
#pragma unroll
                for (int q = 0; q < NW; ++q) {
                    m[a][q] = live ? rl64(f[q], j) : 0;
                    x[a][q] = sig[m[a][q] != 0 ? row + (size_t)q * 64 : 0];
                }
            }
#pragma unroll
            for (int a = 0; a < ARCS; ++a) {
#pragma unroll
                for (int q = 0; q < NW; ++q) {
                    if ((m[a][q] >> lane) & 1) {
                        const uint64_t s = acc[q] + (uint64_t)x[a][q];
                        ovf |= s < acc[q];
                        acc[q] = s;
                    }
                }
            }
        }
    }
}

// acc[q] += sum over arcs [beg, end) of c(w, 64q+lane) for neighbours w whose
// word q of the level-(l+1) frontier meets F[q] at this lane.
template <int NW>
__device__ __forceinline__ void bwd_scan(const Topo &t, int32_t beg, int32_t end, const uint64_t (&F)[NW],
                                         const uint32_t *__restrict__ any_next, const uint64_t *__restrict__ fnext,
                                         const float *__restrict__ cval, int lane, double (&acc)[NW]) {
    constexpr int ARCS = NW >= GDEPTH ? 1 : GDEPTH / NW;
    const float *c = cval + lane;
    for (int32_t base = beg; base < end; base += 64) {
        const int32_t e = base + lane;
        int32_t w = 0;
        uint64_t g[NW];
#pragma unroll
        for (int q = 0; q < NW; ++q) g[q] = 0;
        if (e < end) {
            w = t.col[e];
            if ((any_next[w >> 5] >> (w & 31)) & 1) {
#pragma unroll
                for (int q = 0; q < NW; ++q) g[q] = fnext[(size_t)w * NW + q] & F[q];
            }
        }
        uint64_t nz = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) nz |= g[q];
        uint64_t act = __ballot(nz != 0);
        while (act) {
            float x[ARCS][NW];
#pragma unroll
            for (int a = 0; a < ARCS; ++a) {
#pragma unroll
                for (int q = 0; q < NW; ++q) x[a][q] = 0.f;
                if (act) {
                    const int j = pop_lowest(act);
                    const size_t row = (size_t)rl32(w, j) * t.B;
#pragma unroll
                    for (int q = 0; q < NW; ++q) {
                        const uint64_t gj = rl64(g[q], j);
                        if (gj != 0 && ((gj >> lane) & 1)) x[a][q] = c[row + (size_t)q * 64];
                    }
                }
            }
#pragma unroll
            for (int a = 0; a < ARCS; ++a) {
#pragma unroll
                for (int q = 0; q < NW; ++q) acc[q] += (double)x[a][q];
            }
        }
    }
}

// For every word with sources at this level: delta(v,b) = sigma(v,b) * acc,
// c(v,b) = (1 + delta) / sigma; BC(v) += sum of delta over lanes whose source
// is not v (one atomic per vertex).  A dump of the dependencies is
// source-major, delta_dump[b][v] (n per row), the layout bc_read_sssp returns.
template <int NW, typename S>
__device__ __forceinline__ void bwd_finalize(int32_t v, const uint64_t (&F)[NW], const double (&acc)[NW], int lane,
                                             int B, int32_t n, const S *__restrict__ sigma, float *__restrict__ cval,
                                             const int32_t *__restrict__ src_lane, double *__restrict__ bc,
                                             double *__restrict__ delta_dump, int accumulate) {
    double contrib = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        if ((F[q] >> lane) & 1) {
            const size_t idx = (size_t)v * B + (size_t)q * 64 + lane;
            const double sv = (double)sigma[idx];
            const double dl = sv * acc[q];
            cval[idx] = (float)((1.0 + dl) / sv);
            if (delta_dump) delta_dump[(size_t)(q * 64 + lane) * n + v] = dl;
            if (src_lane[q * 64 + lane] != v) contrib += dl;
        }
    }
    if (accumulate) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) contrib += __shfl_xor(contrib, off, 64);
        if (lane == 0 && contrib != 0.0) unsafeAtomicAdd(&bc[v], contrib);
    }
}

// Clears front levels 0 and 1 (a: 2 * words entries), visited (b), every
// level's vertex filter and every level's flag.
__global__ __launch_bounds__(SB) void k_sp_clear(uint64_t *__restrict__ a, uint64_t *__restrict__ b, size_t words,
                                                 uint32_t *__restrict__ any_all, size_t any_total,
                                                 unsigned long long *__restrict__ lvmax, uint32_t *__restrict__ lvflag,
                                                 int32_t levels, unsigned long long *__restrict__ reach) {
    const size_t tid = (size_t)blockIdx.x * SB + threadIdx.x, stride = (size_t)gridDim.x * SB;
    if (tid < 2) reach[tid] = 0;
    for (size_t i = tid; i < words; i += stride) {
        a[i] = 0;
        a[words + i] = 0;
        b[i] = 0;
    }
    for (size_t i = tid; i < any_total; i += stride) any_all[i] = 0;
    // every count of level 1 is 1 (the pushed first level)
    for (size_t i = tid; i < (size_t)levels; i += stride) {
        lvmax[i] = i <= 1 ? 1ull : 0ull;
        lvflag[i] = 0;
    }
}

// Start of a replayed run: the control block's batch counter, sources and
// handed-back list.
__global__ void k_run_init(BatchCtl *ctl, const int32_t *src, int32_t total, int32_t *redo) {
    if (threadIdx.x != 0) return;
    ctl->batch = 0;
    ctl->total = total;
    ctl->src = src;
    ctl->redo = redo;
    ctl->redo_count = 0;
    ctl->max_nlev = 0;
    ctl->need_wide = 0;
    ctl->deep = 0;
    ctl->arrived = 0;
}

// Seeds the batch: lane b takes source src[b] (b < count).  In a replayed
// batch (ctl non-null) the sources are the run's batch ctl->batch instead.
// The end-of-search counts get, one atomic per wave, the pairs the sources
// can reach (their components' sizes) and those of level 0, and with rp
// non-null (unit weights: level 1 is pushed, all of it) those of level 1,
// each source's neighbours (distinct in a simple graph).  With weights a
// neighbour's level is its arc's weight, and the products count level 1.
template <typename S>
__global__ __launch_bounds__(SB) void k_sp_seed(const int32_t *__restrict__ src, int32_t count, int32_t B, int32_t NW,
                                                uint64_t *front0, uint64_t *visited, S *sigma, int32_t *src_lane,
                                                uint32_t *any0, const BatchCtl *__restrict__ ctl,
                                                const int32_t *__restrict__ comp_size, const int32_t *__restrict__ rp,
                                                unsigned long long *reach) {
    const int32_t b = blockIdx.x * SB + threadIdx.x;
    if (b >= B) return; // B is a multiple of 64: whole waves return here (the shuffles below)
    if (ctl) {
        const int64_t b0 = (int64_t)ctl->batch * B;
        src = ctl->src + b0;
        count = (int32_t)min((int64_t)B, (int64_t)ctl->total - b0);
    }
    const int32_t s = b < count ? src[b] : -1;
    src_lane[b] = s;
    unsigned long long comp = 0, lanes = 0;
    if (s >= 0) {
        const unsigned long long bit = 1ull << (b & 63);
        atomicOr((unsigned long long *)&front0[(size_t)s * NW + (b >> 6)], bit);
        atomicOr((unsigned long long *)&visited[(size_t)s * NW + (b >> 6)], bit);
        atomicOr(&any0[s >> 5], 1u << (s & 31));
        sigma[(size_t)s * B + b] = 1;
        comp = (unsigned long long)comp_size[s];
        // s, and with rp its neighbours (level 1 of an unweighted batch)
        lanes = 1 + (rp ? (unsigned long long)(rp[s + 1] - rp[s]) : 0ull);
    }
    // the pair counts of the end-of-search test: one atomic per wave
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        comp += __shfl_xor(comp, off, 64);
        lanes += __shfl_xor(lanes, off, 64);
    }
    if ((threadIdx.x & 63) == 0 && lanes) {
        atomicAdd(&reach[0], comp);
        atomicAdd(&reach[1], lanes);
    }
}

// Forward level 0 -> 1, pushed from the sources: every neighbour w of s_b
// is at distance 1 with exactly one shortest path (lambda = 1).  One block per
// batch lane; the block's threads take the source's arcs.  The level's pairs
// were counted by the seed kernel, and its vertex filter is written by
// k_any_from_front after this kernel: the filter words are shared by the
// sources adjacent to any of their 32 vertices, so an atomic per arc on them
// serialised (ER n = 16384, 512 sources: about 256 atomics per word; 55 ->
// 16 us per launch with the separate pass).
template <typename S>
__global__ __launch_bounds__(SB) void k_fwd_push0(Topo t, int32_t NW, const int32_t *__restrict__ src_lane,
                                                  uint64_t *__restrict__ fnext, uint64_t *__restrict__ visited,
                                                  S *__restrict__ sigma) {
    const int32_t b = blockIdx.x;
    const int32_t s = src_lane[b];
    if (s < 0) return;
    const unsigned long long bit = 1ull << (b & 63);
    const int q = b >> 6;
    for (int32_t e = t.rp[s] + threadIdx.x; e < t.rp[s + 1]; e += SB) {
        const int32_t w = t.col[e];
        atomicOr((unsigned long long *)&fnext[(size_t)w * NW + q], bit);
        atomicOr((unsigned long long *)&visited[(size_t)w * NW + q], bit);
        sigma[(size_t)w * t.B + b] = 1;
    }
}

// Level 1's vertex filter from its frontier words, after the push: thread v
// tests vertex v's NW words, and each wave's ballot is two whole filter
// words (aw = ceil(n / 32) words; plain stores, one writer per word).
__global__ __launch_bounds__(SB) void k_any_from_front(int32_t n, int32_t NW, size_t aw,
                                                       const uint64_t *__restrict__ front,
                                                       uint32_t *__restrict__ any) {
    const int32_t v = blockIdx.x * SB + threadIdx.x;
    bool nz = false;
    if (v < n)
        for (int q = 0; q < NW; ++q) nz |= front[(size_t)v * NW + q] != 0;
    const uint64_t m = __ballot(nz);
    const size_t w0 = (size_t)(v >> 6) * 2; // v - lane is a multiple of 64
    if ((threadIdx.x & 63) == 0) {
        if (w0 < aw) any[w0] = (uint32_t)m;
        if (w0 + 1 < aw) any[w0 + 1] = (uint32_t)(m >> 32);
    }
}

// Largest x over the wave into *dst (every lane of the wave calls).  The
// maximum settles after a few waves; later waves read it and skip the atomic.
__device__ __forceinline__ void wave_max_to(unsigned long long *dst, uint64_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(x, off, 64);
        x = o > x ? o : x;
    }
    if ((threadIdx.x & 63) == 0 && x > __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(dst, (unsigned long long)x);
}

// Writes the level-(l+1) words of vertex w (lanes 0..NW-1) and marks any_next.
template <int NW>
__device__ __forceinline__ void fwd_commit(int32_t w, const uint64_t (&vis)[NW], const uint64_t (&out)[NW], int lane,
                                           uint64_t *__restrict__ fnext, uint64_t *__restrict__ visited,
                                           uint32_t *__restrict__ any_next) {
    uint64_t mine_out = 0, mine_vis = 0, all = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        if (lane == q) {
            mine_out = out[q];
            mine_vis = vis[q] | out[q];
        }
        all |= out[q];
    }
    if (lane < NW) {
        fnext[(size_t)w * NW + lane] = mine_out;
        if (mine_out) visited[(size_t)w * NW + lane] = mine_vis;
    }
    if (lane == 0 && all) atomicOr(&any_next[w >> 5], 1u << (w & 31));
}

// Forward level l -> l+1 for l >= 1.  Light rows complete in their wave; split
// rows complete in the last segment wave to arrive.  After the last real level
// every vertex is visited for every source it can reach, so speculative
// launches past the depth exit after one load per wave.
// Variants of the forward pull (uniform over a launch):
// - FWD_GENERAL gathers level l's counts from sigma;
// - FWD_UNIT (level 1 -> 2) sums frontier bits, every level-1 count being 1,
//   and when sig16 is set also stores the level-2 counts there as 16 bits
//   (each is at most the vertex's degree, below 2^16: the host checks);
// - FWD_HALF (level 2 -> 3, after FWD_UNIT) gathers the level-2 counts from
//   sig16: half the bytes of a uint32 row.
enum { FWD_GENERAL = 0, FWD_UNIT = 1, FWD_HALF = 2 };
template <int NW, typename S, int MODE>
__device__ __forceinline__ void fwd_item(const Topo &t, int64_t wid, const uint32_t *__restrict__ any_cur,
                                         const uint64_t *__restrict__ fcur, uint64_t *__restrict__ fnext,
                                         uint64_t *__restrict__ visited, S *__restrict__ sigma,
                                         uint16_t *__restrict__ sig16, unsigned long long *__restrict__ hacc,
                                         uint32_t *__restrict__ arrive, uint32_t *__restrict__ any_next,
                                         uint32_t *__restrict__ status, unsigned long long *__restrict__ lvmax_next,
                                         int lane) {
    Item it;
    if (!item_of(t, wid, it)) return;
    const int32_t w = it.v;
    uint64_t vis[NW], U[NW];
    load_words<NW>(visited + (size_t)w * NW, lane, vis);
    uint64_t anyU = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        U[q] = ~vis[q];
        anyU |= U[q];
    }
    if (anyU == 0) {
        if (it.first && lane < NW) fnext[(size_t)w * NW + lane] = 0;
        return;
    }
    uint64_t acc[NW];
#pragma unroll
    for (int q = 0; q < NW; ++q) acc[q] = 0;
    bool ovf = false, wide = false;
    if constexpr (MODE == FWD_HALF)
        fwd_scan<NW, uint16_t, false>(t, it.beg, it.end, U, any_cur, fcur, sig16, lane, acc, ovf);
    else
        fwd_scan<NW, S, MODE == FWD_UNIT>(t, it.beg, it.end, U, any_cur, fcur, sigma, lane, acc, ovf);
    uint64_t out[NW];
    if (it.h < 0) {
        uint64_t mx = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            out[q] = __ballot(acc[q] != 0);
            if (acc[q] != 0) {
                const size_t idx = (size_t)w * t.B + (size_t)q * 64 + lane;
                store_count(&sigma[idx], acc[q], wide);
                if (MODE == FWD_UNIT && sig16) sig16[idx] = (uint16_t)acc[q];
            }
            mx = acc[q] > mx ? acc[q] : mx;
        }
        fwd_commit<NW>(w, vis, out, lane, fnext, visited, any_next);
        if (lvmax_next) wave_max_to(lvmax_next, mx);
    } else {
        unsigned long long *hrow = hacc + (size_t)it.h * t.B + lane;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            if (acc[q] != 0) {
                const unsigned long long old = atomicAdd(&hrow[q * 64], (unsigned long long)acc[q]);
                ovf |= old + acc[q] < old;
            }
        }
        if (last_arriver(&arrive[it.h], t.heavy_nseg[it.h], lane)) {
            uint64_t mx = 0;
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                const uint64_t x = __hip_atomic_load(&hrow[q * 64], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (x != 0) {
                    __hip_atomic_store(&hrow[q * 64], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const size_t idx = (size_t)w * t.B + (size_t)q * 64 + lane;
                    store_count(&sigma[idx], x, wide);
                    if (MODE == FWD_UNIT && sig16) sig16[idx] = (uint16_t)x;
                }
                out[q] = __ballot(x != 0);
                mx = x > mx ? x : mx;
            }
            fwd_commit<NW>(w, vis, out, lane, fnext, visited, any_next);
            if (lvmax_next) wave_max_to(lvmax_next, mx);
        }
    }
    if (__any(ovf) && lane == 0) atomicOr(&status[0], (uint32_t)BC_DEV_SIGMA_OVERFLOW);
    if (__any(wide) && lane == 0) atomicOr(&status[1], 1u);
}

// The launches.  k_fwd_pull: each wave takes rows (or segments) wave, wave +
// waves, ... of the n + nseg, eight waves per SIMD (the loop's extra live
// values fit 64 registers for up to four words).  k_fwd_pull_row: one wave
// per row or segment, for eight words per row, whose registers leave no room
// for the loop.
template <int NW, typename S, int MODE>
__global__ __launch_bounds__(SB) __attribute__((amdgpu_waves_per_eu(8))) void k_fwd_pull(
    Topo t, const uint32_t *__restrict__ any_cur, const uint64_t *__restrict__ fcur, uint64_t *__restrict__ fnext,
    uint64_t *__restrict__ visited, S *__restrict__ sigma, uint16_t *__restrict__ sig16,
    unsigned long long *__restrict__ hacc, uint32_t *__restrict__ arrive, uint32_t *__restrict__ any_next,
    uint32_t *__restrict__ status, unsigned long long *__restrict__ lvmax_next) {
    const int lane = threadIdx.x & 63;
    const int64_t items = (int64_t)t.n + t.nseg, waves = (int64_t)gridDim.x * WPB;
    for (int64_t wid = (int64_t)blockIdx.x * WPB + (threadIdx.x >> 6); wid < items; wid += waves)
        fwd_item<NW, S, MODE>(t, wid, any_cur, fcur, fnext, visited, sigma, sig16, hacc, arrive, any_next, status,
                              lvmax_next, lane);
}
template <int NW, typename S, int MODE>
__global__ __launch_bounds__(SB) void k_fwd_pull_row(
    Topo t, const uint32_t *__restrict__ any_cur, const uint64_t *__restrict__ fcur, uint64_t *__restrict__ fnext,
    uint64_t *__restrict__ visited, S *__restrict__ sigma, uint16_t *__restrict__ sig16,
    unsigned long long *__restrict__ hacc, uint32_t *__restrict__ arrive, uint32_t *__restrict__ any_next,
    uint32_t *__restrict__ status, unsigned long long *__restrict__ lvmax_next) {
    const int64_t wid = (int64_t)blockIdx.x * WPB + (threadIdx.x >> 6);
    if (wid < (int64_t)t.n + t.nseg)
        fwd_item<NW, S, MODE>(t, wid, any_cur, fcur, fnext, visited, sigma, sig16, hacc, arrive, any_next, status,
                              lvmax_next, threadIdx.x & 63);
}

// Backward level l.  Light rows complete in their wave; split rows in the last
// segment wave to arrive.  fnext = nullptr at the deepest level.
template <int NW, typename S>
__global__ __launch_bounds__(SB) void k_bwd_pull(Topo t, const uint64_t *__restrict__ fcur,
                                                 const uint32_t *__restrict__ any_next,
                                                 const uint64_t *__restrict__ fnext, const S *__restrict__ sigma,
                                                 float *__restrict__ cval, const int32_t *__restrict__ src_lane,
                                                 double *__restrict__ bc, double *__restrict__ hacc,
                                                 uint32_t *__restrict__ arrive, double *__restrict__ delta_dump,
                                                 int accumulate, const uint32_t *__restrict__ lvf) {
    // replayed batches: lvf[0] says level l holds a vertex (cleared for a
    // batch handed back), lvf[1] level l+1 (else fnext is not read)
    if (lvf) {
        if (lvf[0] == 0) return;
        if (lvf[1] == 0) fnext = nullptr;
    }
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * WPB + (threadIdx.x >> 6);
    Item it;
    if (!item_of(t, wid, it)) return;
    const int32_t v = it.v;
    uint64_t F[NW];
    load_words<NW>(fcur + (size_t)v * NW, lane, F);
    uint64_t anyF = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) anyF |= F[q];
    if (anyF == 0) return;
    double acc[NW];
#pragma unroll
    for (int q = 0; q < NW; ++q) acc[q] = 0.0;
    if (!fnext) {
        // the deepest level: no successor, so delta = 0 and c = 1 / lambda;
        // the row's first segment finalizes it, no partial sums are needed
        if (it.first) bwd_finalize<NW, S>(v, F, acc, lane, t.B, t.n, sigma, cval, src_lane, bc, delta_dump, accumulate);
        return;
    }
    bwd_scan<NW>(t, it.beg, it.end, F, any_next, fnext, cval, lane, acc);
    if (it.h < 0) {
        bwd_finalize<NW, S>(v, F, acc, lane, t.B, t.n, sigma, cval, src_lane, bc, delta_dump, accumulate);
        return;
    }
    double *hrow = hacc + (size_t)it.h * t.B + lane;
#pragma unroll
    for (int q = 0; q < NW; ++q)
        if (acc[q] != 0.0) unsafeAtomicAdd(&hrow[q * 64], acc[q]);
    if (last_arriver(&arrive[it.h], t.heavy_nseg[it.h], lane)) {
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            acc[q] = 0.0;
            if ((F[q] >> lane) & 1) {
                acc[q] = __hip_atomic_load(&hrow[q * 64], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (acc[q] != 0.0) __hip_atomic_store(&hrow[q * 64], 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        bwd_finalize<NW, S>(v, F, acc, lane, t.B, t.n, sigma, cval, src_lane, bc, delta_dump, accumulate);
    }
}

// Backward level l, one item per (row or row segment, word q): at the fat
// levels this keeps NW times more waves in flight than a wave per row, and a
// word with no sources at this level costs its wave a single load.
template <int NW, typename S, bool EB>
__device__ __forceinline__ void bwd_item_w(const Topo &t, int64_t wid, const uint64_t *__restrict__ fcur,
                                           const uint32_t *__restrict__ any_next, const uint64_t *__restrict__ fnext,
                                           const S *__restrict__ sigma, float *__restrict__ cval,
                                           const int32_t *__restrict__ src_lane, double *__restrict__ bc,
                                           double *__restrict__ hacc, uint32_t *__restrict__ arrive,
                                           double *__restrict__ delta_dump, int accumulate, double *__restrict__ eb,
                                           int lane) {
    (void)any_next; // the per-word pull reads successors' words directly
    const int q = (int)(wid % NW);
    Item it;
    const int64_t r = wid / NW;
    uint64_t F;
    if (r < t.n) {
        // a light row: its bounds, its heavy mark and its frontier word are
        // independent loads, issued together
        const int32_t v0 = (int32_t)r;
        const int32_t hv = t.heavy_id[v0], b0 = t.rp[v0], e0 = t.rp[v0 + 1];
        F = fcur[(size_t)v0 * NW + q];
        if (hv >= 0 || F == 0) return;
        it.v = v0;
        it.beg = b0;
        it.end = e0;
        it.h = -1;
        it.first = true;
    } else {
        if (!item_of(t, r, it)) return;
        F = fcur[(size_t)it.v * NW + q];
        if (F == 0) return;
    }
    const int32_t v = it.v;
    const uint64_t F1[1] = {F};
    double acc[1] = {0.0};
    if (!fnext) {
        // the deepest level: no successor, so delta = 0 and c = 1 / lambda;
        // the row's first segment finalizes it, no partial sums are needed
        if (it.first)
            bwd_finalize<1, S>(v, F1, acc, lane, t.B, t.n, sigma + (size_t)q * 64, cval + (size_t)q * 64,
                               src_lane + q * 64, bc, delta_dump ? delta_dump + (size_t)q * 64 * t.n : nullptr,
                               accumulate);
        return;
    }
    {
        // the single-word scan over word q: shift the row base by q words
        const float *c = cval + (size_t)q * 64 + lane;
        // edge betweenness: arc v -> w carries sum over this word's sources of
        // lambda(v) c(w) (the per-arc term of Theorem 1.1)
        const double sv = eb && ((F >> lane) & 1) ? (double)sigma[(size_t)v * t.B + (size_t)q * 64 + lane] : 0.0;
        for (int32_t base = it.beg; base < it.end; base += 64) {
            const int32_t e = base + lane;
            int32_t w = 0;
            uint64_t g = 0;
            if (e < it.end) {
                w = t.col[e];
                // the successor's word straight away, not after the level's
                // vertex filter: every vertex's word of the level is written
                // (zero off the level), the level's words are small enough to
                // stay in the caches, and the filter was one more dependent
                // load in front of the gathers (80.1 against 85.9 us per
                // launch on RMAT-16)
                g = fnext[(size_t)w * NW + q] & F;
            }
            uint64_t act = __ballot(g != 0);
            // gathers per round: without edge terms the wave has the
            // registers for sixteen at full occupancy
            constexpr int D = EB ? GDEPTH : 2 * GDEPTH;
            while (act) {
                float x[D];
                int jj[D];
#pragma unroll
                for (int u = 0; u < D; ++u) {
                    x[u] = 0.f;
                    jj[u] = -1;
                    if (act) {
                        const int j = pop_lowest(act);
                        jj[u] = j;
                        if ((rl64(g, j) >> lane) & 1) x[u] = c[(size_t)rl32(w, j) * t.B];
                    }
                }
#pragma unroll
                for (int u = 0; u < D; ++u) acc[0] += (double)x[u];
                if (EB && eb) {
                    static_assert(GDEPTH == 8, "wave_sum8 reduces eight arcs");
                    double p[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) p[u] = sv * (double)x[u];
                    const double tot = wave_sum8(p, lane);
                    int mine = -1; // the arc whose sum this lane holds
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (((lane >> 3) & 7) == u) mine = jj[u];
                    if ((lane & 7) == 0 && mine >= 0 && tot != 0.0) unsafeAtomicAdd(&eb[base + mine], tot);
                }
            }
        }
    }
    const S *sig_q = sigma + (size_t)q * 64;
    float *cval_q = cval + (size_t)q * 64;
    const int32_t *src_q = src_lane + q * 64;
    if (it.h < 0) {
        bwd_finalize<1, S>(v, F1, acc, lane, t.B, t.n, sig_q, cval_q, src_q, bc,
                           delta_dump ? delta_dump + (size_t)q * 64 * t.n : nullptr, accumulate);
        return;
    }
    double *hp = hacc + (size_t)it.h * t.B + (size_t)q * 64 + lane;
    if (acc[0] != 0.0) unsafeAtomicAdd(hp, acc[0]);
    if (last_arriver(&arrive[(size_t)it.h * NW + q], t.heavy_nseg[it.h], lane)) {
        acc[0] = 0.0;
        if ((F >> lane) & 1) {
            acc[0] = __hip_atomic_load(hp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (acc[0] != 0.0) __hip_atomic_store(hp, 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        bwd_finalize<1, S>(v, F1, acc, lane, t.B, t.n, sig_q, cval_q, src_q, bc,
                           delta_dump ? delta_dump + (size_t)q * 64 * t.n : nullptr, accumulate);
    }
}

// The launches.  k_bwd_pull_w: each wave takes items wave, wave + waves, ...
// of the (n + nseg) * NW, eight waves per SIMD; a grid smaller than one wave
// per item makes a launch whose level turns out empty (replayed batches) cost
// a few thousand waves' flag reads instead of one wave per item.  With edge
// terms the loop's extra live values would spill: one item per wave.
template <int NW, typename S>
__global__ __launch_bounds__(SB) __attribute__((amdgpu_waves_per_eu(8))) void k_bwd_pull_w(
    Topo t, const uint64_t *__restrict__ fcur, const uint32_t *__restrict__ any_next,
    const uint64_t *__restrict__ fnext, const S *__restrict__ sigma, float *__restrict__ cval,
    const int32_t *__restrict__ src_lane, double *__restrict__ bc, double *__restrict__ hacc,
    uint32_t *__restrict__ arrive, double *__restrict__ delta_dump, int accumulate, const uint32_t *__restrict__ lvf) {
    // lvf as in k_bwd_pull
    if (lvf) {
        if (lvf[0] == 0) return;
        if (lvf[1] == 0) fnext = nullptr;
    }
    const int lane = threadIdx.x & 63;
    const int64_t items = ((int64_t)t.n + t.nseg) * NW, waves = (int64_t)gridDim.x * WPB;
    for (int64_t wid = (int64_t)blockIdx.x * WPB + (threadIdx.x >> 6); wid < items; wid += waves)
        bwd_item_w<NW, S, false>(t, wid, fcur, any_next, fnext, sigma, cval, src_lane, bc, hacc, arrive, delta_dump,
                                 accumulate, nullptr, lane);
}
template <int NW, typename S>
__global__ __launch_bounds__(SB) void k_bwd_pull_we(Topo t, const uint64_t *__restrict__ fcur,
                                                    const uint32_t *__restrict__ any_next,
                                                    const uint64_t *__restrict__ fnext, const S *__restrict__ sigma,
                                                    float *__restrict__ cval, const int32_t *__restrict__ src_lane,
                                                    double *__restrict__ bc, double *__restrict__ hacc,
                                                    uint32_t *__restrict__ arrive, double *__restrict__ delta_dump,
                                                    int accumulate, double *__restrict__ eb,
                                                    const uint32_t *__restrict__ lvf) {
    if (lvf) {
        if (lvf[0] == 0) return;
        if (lvf[1] == 0) fnext = nullptr;
    }
    const int64_t wid = (int64_t)blockIdx.x * WPB + (threadIdx.x >> 6);
    if (wid < ((int64_t)t.n + t.nseg) * NW)
        bwd_item_w<NW, S, true>(t, wid, fcur, any_next, fnext, sigma, cval, src_lane, bc, hacc, arrive, delta_dump,
                                accumulate, eb, threadIdx.x & 63);
}

// Per-source readout for bc_read_sssp: out[b][v] in source-major layout.  The
// dependencies are already there (the backward wrote them); unreached
// vertices get 0.
template <typename S>
__global__ __launch_bounds__(SB) void k_sp_dump(int32_t n, int32_t NW, int32_t B, int32_t count, int32_t nlev,
                                                const uint64_t *__restrict__ front, const S *__restrict__ sigma,
                                                int32_t *__restrict__ dist_out, uint64_t *__restrict__ sigma_out,
                                                double *__restrict__ delta_out) {
    const int64_t i = (int64_t)blockIdx.x * SB + threadIdx.x;
    if (i >= (int64_t)n * count) return;
    const int32_t b = (int32_t)(i / n), v = (int32_t)(i - (int64_t)b * n);
    const int q = b >> 6, bit = b & 63;
    int32_t d = -1;
    for (int32_t l = 0; l < nlev && d < 0; ++l)
        if ((front[((size_t)l * n + v) * NW + q] >> bit) & 1) d = l;
    dist_out[i] = d;
    sigma_out[i] = d >= 0 ? (uint64_t)sigma[(size_t)v * B + b] : 0;
    if (delta_out && d < 0) delta_out[i] = 0.0;
}

Topo topo(bc_ctx *ctx) {
    const SparseState &s = ctx->sp;
    Topo t;
    t.n = ctx->n;
    t.B = s.batch;
    t.rp = ctx->row_ptr;
    t.col = ctx->col;
    t.heavy_id = s.heavy_id;
    t.seg_v = s.seg_v;
    t.seg_beg = s.seg_beg;
    t.seg_end = s.seg_end;
    t.nseg = s.nseg;
    t.heavy_nseg = s.heavy_nseg;
    return t;
}

inline int32_t any_words(const bc_ctx *ctx) { return (ctx->n + 31) >> 5; }

// Union-frontier density of level l, from the host mirror of any[l].
double level_density(const bc_ctx *ctx, int32_t l) {
    const int32_t aw = any_words(ctx);
    const uint32_t *a = ctx->sp.any_host + (size_t)l * aw;
    int64_t c = 0;
    for (int32_t i = 0; i < aw; ++i) c += __builtin_popcount(a[i]);
    return ctx->n > 0 ? (double)c / ctx->n : 0.0;
}

int probe_mode(const bc_ctx *ctx) { return ctx->hy.probe ? ctx->hy.probe->mode : 0; }

// Does level l (>= 1) go by products with A?  The algebraic form takes them at
// every level; the hybrid form compares the level's density with a threshold.
// The backward knows the batch's own densities.  The forward is launched ahead
// of the host (levels are read back once per several levels), so it decides
// level l from the density level l had in the previous batch of this context;
// a level no earlier batch reached goes by pulls.
bool by_products(const bc_ctx *ctx, int32_t l, bool forward) {
    if (l < 1) return false;
    if (ctx->al.every_level) return true;
    if (!ctx->hy.products) return false;
    if (!forward && ctx->edges) return false; // edge terms need the per-arc pulls
    const int mode = probe_mode(ctx);
    if (mode != 0) return mode == 2;
    if (!forward) return level_density(ctx, l) >= ctx->hy.theta_bwd;
    const std::vector<double> &pd = ctx->hy.prev_density;
    return (size_t)l < pd.size() && pd[(size_t)l] >= ctx->hy.theta_fwd;
}

// Event pair around one level's work while a probe is attached.
struct ProbeScope {
    bc_ctx *ctx;
    hipEvent_t a = nullptr;
    ProbeScope(bc_ctx *c) : ctx(c) {
        if (ctx->hy.probe && (a = bc_event_get(ctx)) != nullptr) hipEventRecord(a, ctx->stream);
    }
    void done(bool forward, int32_t level) {
        if (!a) return;
        hipEvent_t b = bc_event_get(ctx);
        if (!b) {
            bc_event_put(ctx, a);
            a = nullptr;
            return;
        }
        hipEventRecord(b, ctx->stream);
        ctx->hy.probe->recs.push_back({forward, level, 0.0, a, b});
        a = nullptr;
    }
};

bc_status ensure_levels(bc_ctx *ctx, int32_t need) {
    SparseState &s = ctx->sp;
    if (need <= s.level_cap) return BC_OK;
    int32_t cap = std::max(s.level_cap * 2, need);
    const size_t aw = (size_t)any_words(ctx);
    const size_t lvl_words = (size_t)ctx->n * s.words;
    const size_t per_level = lvl_words * sizeof(uint64_t) + aw * sizeof(uint32_t);
    const size_t budget = size_t(32) << 30;
    if ((size_t)cap * per_level > budget) {
        cap = need;
        if ((size_t)cap * per_level > budget)
            return bc_fail(ctx, BC_ERR_UNSUPPORTED,
                           "sparse form: the graph is too deep for per-level frontier bitmaps; use the plain form");
    }
    uint64_t *nf = (uint64_t *)bc_dalloc(ctx, (size_t)cap * lvl_words * sizeof(uint64_t));
    uint32_t *na = (uint32_t *)bc_dalloc(ctx, (size_t)cap * aw * sizeof(uint32_t));
    unsigned long long *nm = (unsigned long long *)bc_dalloc(ctx, (size_t)cap * sizeof(unsigned long long));
    uint32_t *nl = (uint32_t *)bc_dalloc(ctx, (size_t)cap * sizeof(uint32_t));
    uint32_t *nh = nullptr;
    if (!nf || !na || !nm || !nl || hipHostMalloc((void **)&nh, (size_t)cap * aw * sizeof(uint32_t)) != hipSuccess) {
        bc_dfree(ctx, nf);
        bc_dfree(ctx, na);
        bc_dfree(ctx, nm);
        bc_dfree(ctx, nl);
        return bc_fail(ctx, BC_ERR_NOMEM, "sparse form: frontier allocation failed");
    }
    const int32_t old = s.level_cap;
    if (s.front) {
        BC_HIP(ctx, hipMemcpyAsync(nf, s.front, (size_t)old * lvl_words * sizeof(uint64_t), hipMemcpyDeviceToDevice,
                                   ctx->stream));
        BC_HIP(ctx, hipMemcpyAsync(na, s.any, (size_t)old * aw * sizeof(uint32_t), hipMemcpyDeviceToDevice, ctx->stream));
        BC_HIP(ctx, hipMemcpyAsync(nm, s.lvmax, (size_t)old * sizeof(unsigned long long), hipMemcpyDeviceToDevice,
                                   ctx->stream));
        BC_HIP(ctx, hipMemcpyAsync(nl, s.lvflag, (size_t)old * sizeof(uint32_t), hipMemcpyDeviceToDevice, ctx->stream));
    }
    BC_HIP(ctx, hipMemsetAsync(na + (size_t)old * aw, 0, (size_t)(cap - old) * aw * sizeof(uint32_t), ctx->stream));
    BC_HIP(ctx, hipMemsetAsync(nm + old, 0, (size_t)(cap - old) * sizeof(unsigned long long), ctx->stream));
    BC_HIP(ctx, hipMemsetAsync(nl + old, 0, (size_t)(cap - old) * sizeof(uint32_t), ctx->stream));
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (s.front) {
        bc_dfree(ctx, s.front);
        bc_dfree(ctx, s.any);
        bc_dfree(ctx, s.lvmax);
        bc_dfree(ctx, s.lvflag);
        hipHostFree(s.any_host);
    }
    s.front = nf;
    s.any = na;
    s.lvmax = nm;
    s.lvflag = nl;
    s.any_host = nh;
    s.level_cap = cap;
    return BC_OK;
}

// ---- the launches of one batch, shared by the host-driven batch and the
// recorded (replayed) batch ----------------------------------------------------

struct BatchShape {
    int32_t n, B, aw;
    size_t words;
    int pull_blocks, word_blocks;
    Topo t;
};

template <int NW>
BatchShape batch_shape(bc_ctx *ctx) {
    SparseState &s = ctx->sp;
    BatchShape b;
    b.n = ctx->n;
    b.B = s.batch;
    b.aw = any_words(ctx);
    b.words = (size_t)b.n * NW;
    b.pull_blocks = (int)(((int64_t)b.n + s.nseg + WPB - 1) / WPB);
    b.word_blocks = (int)((((int64_t)b.n + s.nseg) * NW + WPB - 1) / WPB);
    b.t = topo(ctx);
    return b;
}

// Clears the batch state and seeds the sources: d_src/count, or with ctl the
// run's batch ctl->batch.
template <int NW, typename S>
bc_status launch_batch_init(bc_ctx *ctx, const BatchShape &b, const int32_t *d_src, int32_t count,
                            const BatchCtl *ctl) {
    SparseState &s = ctx->sp;
    LaunchTimer tm(ctx, "batch_init");
    const int blocks = (int)std::min<size_t>((b.words + SB - 1) / SB, 8192);
    hipLaunchKernelGGL(k_sp_clear, dim3(std::max(blocks, 1)), dim3(SB), 0, ctx->stream, s.front, s.visited, b.words,
                       s.any, (size_t)s.level_cap * b.aw, s.lvmax, s.lvflag, s.level_cap, s.reach);
    hipLaunchKernelGGL(k_sp_seed<S>, dim3((b.B + SB - 1) / SB), dim3(SB), 0, ctx->stream, d_src, count, b.B, NW,
                       s.front, s.visited, reinterpret_cast<S *>(s.sigma), s.src, s.any, ctl,
                       (const int32_t *)ctx->comp_size, ctx->weighted ? nullptr : b.t.rp, s.reach);
    tm.done();
    BC_HIP(ctx, hipGetLastError());
    return BC_OK;
}

// Forward level l -> l+1 of an unweighted batch.  products: this level goes
// by products; next_products: level l+1 will (so its largest count is
// recorded).  *l1_pulled tracks whether level 1 -> 2 filled the 16-bit counts.
template <int NW, typename S>
bc_status launch_fwd_level(bc_ctx *ctx, const BatchShape &b, int32_t l, bool products, bool next_products,
                           uint16_t *sig16, bool *l1_pulled) {
    SparseState &s = ctx->sp;
    if (l == 0) {
        LaunchTimer tm(ctx, "fwd_push0");
        hipLaunchKernelGGL(k_fwd_push0<S>, dim3(b.B), dim3(SB), 0, ctx->stream, b.t, NW, (const int32_t *)s.src,
                           s.front + b.words, s.visited, reinterpret_cast<S *>(s.sigma));
        hipLaunchKernelGGL(k_any_from_front, dim3((ctx->n + SB - 1) / SB), dim3(SB), 0, ctx->stream, ctx->n, NW,
                           (size_t)b.aw, (const uint64_t *)(s.front + b.words), s.any + b.aw);
        tm.done();
        return BC_OK;
    }
    if (products) return algebraic_forward_level(ctx, sizeof(S) == 8, l);
    LaunchTimer tm(ctx, "fwd_pull");
    // level 1 holds the sources' neighbours, each with one shortest path (the
    // input graph is simple): its pull counts frontier bits, and level 2's
    // counts (at most a degree) also go to sig16, from which level 2 -> 3
    // gathers them
    const bool strided = NW < 8 && s.fwd_grid > 0;
    const auto kern = l == 1                 ? (strided ? k_fwd_pull<NW, S, FWD_UNIT> : k_fwd_pull_row<NW, S, FWD_UNIT>)
                      : l == 2 && *l1_pulled ? (strided ? k_fwd_pull<NW, S, FWD_HALF> : k_fwd_pull_row<NW, S, FWD_HALF>)
                                             : (strided ? k_fwd_pull<NW, S, FWD_GENERAL>
                                                        : k_fwd_pull_row<NW, S, FWD_GENERAL>);
    if (l == 1) *l1_pulled = sig16 != nullptr;
    const int grid = strided ? std::min(b.pull_blocks, s.fwd_grid) : b.pull_blocks;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(SB), 0, ctx->stream, b.t, s.any + (size_t)l * b.aw,
                       s.front + (size_t)l * b.words, s.front + (size_t)(l + 1) * b.words, s.visited,
                       reinterpret_cast<S *>(s.sigma), sig16, (unsigned long long *)s.hacc, s.arrive,
                       s.any + (size_t)(l + 1) * b.aw, ctx->status, next_products ? s.lvmax + l + 1 : nullptr);
    tm.done();
    return BC_OK;
}

// Backward level lv of an unweighted batch.  Host-driven (flags = false):
// deeper says whether level lv+1 exists.  Replayed (flags = true): the level
// flags the batch check wrote decide, on the device, whether level lv has a
// vertex and whether level lv+1 is read (front[lv+1] must exist: lv+1 <
// level_cap).
template <int NW, typename S>
bc_status launch_bwd_level(bc_ctx *ctx, const BatchShape &b, int32_t lv, bool products, bool deeper, bool flags,
                           double *ddump, bool accumulate) {
    SparseState &s = ctx->sp;
    const uint64_t *fcur = s.front + (size_t)lv * b.words;
    const uint64_t *fnext = flags || deeper ? s.front + (size_t)(lv + 1) * b.words : nullptr;
    const uint32_t *anext = fnext ? s.any + (size_t)(lv + 1) * b.aw : nullptr;
    const uint32_t *lvf = flags ? s.lvflag + lv : nullptr;
    if (products) return algebraic_backward_level(ctx, sizeof(S) == 8, fcur, fnext, 1, ddump, accumulate, lvf);
    LaunchTimer tm(ctx, "bwd_pull");
    const S *sigma = reinterpret_cast<const S *>(s.sigma);
    if (ctx->edges && accumulate) // edge terms come from the per-word pull, one wave per item
        hipLaunchKernelGGL((k_bwd_pull_we<NW, S>), dim3(b.word_blocks), dim3(SB), 0, ctx->stream, b.t, fcur, anext, fnext,
                           sigma, s.cval, s.src, ctx->bc, s.hacc, s.arrive_w, ddump, 1, ctx->eb, lvf);
    else if (s.bwd_per_word || ctx->edges) {
        const int grid = s.bwd_grid > 0 ? std::min(b.word_blocks, s.bwd_grid) : b.word_blocks;
        hipLaunchKernelGGL((k_bwd_pull_w<NW, S>), dim3(grid), dim3(SB), 0, ctx->stream, b.t, fcur, anext, fnext, sigma,
                           s.cval, s.src, ctx->bc, s.hacc, s.arrive_w, ddump, accumulate ? 1 : 0, lvf);
    } else
        hipLaunchKernelGGL((k_bwd_pull<NW, S>), dim3(b.pull_blocks), dim3(SB), 0, ctx->stream, b.t, fcur, anext, fnext,
                           sigma, s.cval, s.src, ctx->bc, s.hacc, s.arrive, ddump, accumulate ? 1 : 0, lvf);
    tm.done();
    return BC_OK;
}

// 16-bit copy of level 2's counts, in the unused upper half of the count
// array (uint32 counts fill the first half of its uint64 capacity).
template <typename S>
uint16_t *sig16_of(bc_ctx *ctx) {
    return sizeof(S) == 4 && ctx->max_degree < 65536
               ? reinterpret_cast<uint16_t *>(reinterpret_cast<uint32_t *>(ctx->sp.sigma) + (size_t)ctx->n * ctx->sp.batch)
               : nullptr;
}

// One batch of up to B sources with counts stored as S; *nlev_out receives
// the number of non-empty levels.  Forward levels are launched ahead of the
// host knowing whether they are needed (as many as the previous batch used);
// the host then reads the per-level vertex filters back with one
// synchronisation and finds the first empty level (with weights 1..M, the
// first of M consecutive empty levels: levels are then distances).  With S = uint32_t,
// *need_wide reports a count of 2^32 or more, before anything was added to BC.
// With accumulate = false, delta_dump (count rows of n, source-major) receives
// the dependencies instead of BC.
template <int NW, typename S>
bc_status run_batch_t(bc_ctx *ctx, const int32_t *d_src, int32_t count, bool accumulate, int32_t *nlev_out,
                      bool *need_wide, bool backward, double *delta_dump) {
    SparseState &s = ctx->sp;
    const int32_t guess = std::max(s.depth_guess, 2);
    *need_wide = false;
    bc_status st = ensure_levels(ctx, guess + 1);
    if (st != BC_OK) return st;
    const BatchShape b = batch_shape<NW>(ctx);
    const size_t words = b.words;
    const int32_t aw = b.aw;
    st = launch_batch_init<NW, S>(ctx, b, d_src, count, nullptr);
    if (st != BC_OK) return st;
    int32_t launched = 0, nlev = -1;
    const bool wide_now = sizeof(S) == 8;
    uint16_t *sig16 = sig16_of<S>(ctx);
    bool l1_pulled = false; // level 1 -> 2 ran as the pull that fills sig16
    // Weighted graphs (the algebraic form, Sec. 3.2): levels are distances and
    // level l+1 is formed from levels l+1-M .. l; the search ends at M
    // consecutive empty levels.  An empty level there does not end the
    // search, so those products run without level flags.
    const bool weighted = ctx->weighted;
    const int32_t M = weighted ? ctx->al.classes : 1;

    const size_t rec0 = ctx->hy.probe ? ctx->hy.probe->recs.size() : 0;
    while (nlev < 0) {
        const int32_t target = launched == 0 ? std::max(guess + M - 1, M + 1) : launched + std::max(2, M);
        st = ensure_levels(ctx, target + 1);
        if (st != BC_OK) return st;
        const BatchShape bb = batch_shape<NW>(ctx); // same shape; front may have moved
        for (int32_t l = launched; l < target; ++l) {
            if (weighted) {
                st = algebraic_forward_level(ctx, wide_now, l);
                if (st != BC_OK) return st;
                continue;
            }
            if (l == 0) { // pushed, not a level the hybrid choice covers
                st = launch_fwd_level<NW, S>(ctx, bb, 0, false, by_products(ctx, 1, true), sig16, &l1_pulled);
                if (st != BC_OK) return st;
                continue;
            }
            ProbeScope ps(ctx);
            st = launch_fwd_level<NW, S>(ctx, bb, l, by_products(ctx, l, true), by_products(ctx, l + 1, true), sig16,
                                         &l1_pulled);
            if (st != BC_OK) return st;
            ps.done(true, l);
        }
        BC_HIP(ctx, hipGetLastError());
        const int32_t first = 1; // levels whose filter is read back
        BC_HIP(ctx, hipMemcpyAsync(s.any_host + (size_t)first * aw, s.any + (size_t)first * aw,
                                   (size_t)(target - first + 1) * aw * sizeof(uint32_t), hipMemcpyDeviceToHost,
                                   ctx->stream));
        BC_HIP(ctx, hipMemcpyAsync(ctx->status_host + 1, ctx->status + 1, sizeof(uint32_t), hipMemcpyDeviceToHost,
                                   ctx->stream));
        BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (ctx->status_host[1] != 0) {
            BC_HIP(ctx, hipMemsetAsync(ctx->status + 1, 0, sizeof(uint32_t), ctx->stream));
            *need_wide = true;
            return BC_OK;
        }
        // nlev = the first level l >= 1 that starts a run of M empty levels
        int32_t run = 0;
        for (int32_t l = first; l <= target && nlev < 0; ++l) {
            const uint32_t *a = s.any_host + (size_t)l * aw;
            bool empty = true;
            for (int32_t i = 0; i < aw && empty; ++i) empty = a[i] == 0;
            run = empty ? run + 1 : 0;
            if (run == M) nlev = l - M + 1;
        }
        launched = target;
    }
    s.depth_guess = nlev;
    s.depth_max = std::max(s.depth_max, nlev);
    // Level 0 adds nothing to BC (v is the source), but with edges on its
    // arcs out of the source carry edge terms.
    // A forward-only batch (all-pairs distances and counts) runs no level.
    const int32_t lowest = !backward ? nlev : accumulate && !ctx->edges ? 1 : 0;
    double *ddump = accumulate ? nullptr : delta_dump;
    const BatchShape bb = batch_shape<NW>(ctx);
    for (int32_t lv = nlev - 1; lv >= lowest; --lv) {
        if (weighted) {
            // successors at levels lv+1 .. lv+M that exist; at the deepest
            // level none, and the product only sets c = 1 / lambda
            const uint64_t *fcur = s.front + (size_t)lv * words;
            const uint64_t *fnext = lv + 1 < nlev ? s.front + (size_t)(lv + 1) * words : nullptr;
            st = algebraic_backward_level(ctx, sizeof(S) == 8, fcur, fnext, std::min(M, nlev - 1 - lv), ddump,
                                          accumulate);
            if (st != BC_OK) return st;
            continue;
        }
        ProbeScope ps(ctx);
        const bool deeper = lv + 1 < nlev;
        st = launch_bwd_level<NW, S>(ctx, bb, lv, deeper && by_products(ctx, lv, false), deeper, false, ddump,
                                     accumulate);
        if (st != BC_OK) return st;
        ps.done(false, lv);
    }
    BC_HIP(ctx, hipGetLastError());
    if (ctx->hy.products) {
        std::vector<double> &pd = ctx->hy.prev_density;
        pd.assign((size_t)nlev, 0.0);
        for (int32_t l = 1; l < nlev; ++l) pd[(size_t)l] = level_density(ctx, l);
    }
    if (LevelProbe *p = ctx->hy.probe) {
        // Levels past the deepest were launched speculatively and did nothing;
        // level 0 of the backward is not a level the hybrid choice covers.
        size_t keep = rec0;
        for (size_t i = rec0; i < p->recs.size(); ++i) {
            LevelProbe::Rec r = p->recs[i];
            if (r.level < 1 || r.level >= nlev) {
                bc_event_put(ctx, r.a);
                bc_event_put(ctx, r.b);
                continue;
            }
            r.density = level_density(ctx, r.level);
            p->recs[keep++] = r;
        }
        p->recs.resize(keep);
    }
    ctx->max_levels = std::max(ctx->max_levels, nlev);
    *nlev_out = nlev;
    return BC_OK;
}

template <int NW>
bc_status run_batch_nw(bc_ctx *ctx, const int32_t *d_src, int32_t count, bool accumulate, int32_t *nlev_out,
                       bool backward, double *delta_dump) {
    SparseState &s = ctx->sp;
    if (!s.wide) {
        bool need_wide = false;
        bc_status st =
            run_batch_t<NW, uint32_t>(ctx, d_src, count, accumulate, nlev_out, &need_wide, backward, delta_dump);
        if (st != BC_OK || !need_wide) return st;
        s.wide = true;
    }
    bool unused = false;
    return run_batch_t<NW, uint64_t>(ctx, d_src, count, accumulate, nlev_out, &unused, backward, delta_dump);
}

// Counts start as uint32; the first batch that needs more switches the context
// to uint64 storage for good and is re-run.
bc_status run_batch(bc_ctx *ctx, const int32_t *d_src, int32_t count, bool accumulate, int32_t *nlev_out,
                    bool backward = true, double *delta_dump = nullptr) {
    switch (ctx->sp.words) {
    case 1: return run_batch_nw<1>(ctx, d_src, count, accumulate, nlev_out, backward, delta_dump);
    case 2: return run_batch_nw<2>(ctx, d_src, count, accumulate, nlev_out, backward, delta_dump);
    case 4: return run_batch_nw<4>(ctx, d_src, count, accumulate, nlev_out, backward, delta_dump);
    case 8: return run_batch_nw<8>(ctx, d_src, count, accumulate, nlev_out, backward, delta_dump);
    }
    return bc_fail(ctx, BC_ERR_INVALID_ARG, "sparse form: batch must be 64, 128, 256 or 512");
}

// ---- replayed batches -----------------------------------------------------------
//
// A run of many batches on an unweighted graph is not driven level by level
// from the host.  One batch's launch sequence -- clear, seed, forward levels
// 0 .. L-1, a check, backward levels L-1 .. lowest -- is recorded once into a
// HIP graph and replayed for every batch of the run; a device control block
// tells each replay which sources it takes.  The level-synchronous order of
// the search (Sec. 4) is kept: each level is one launch.  A forward level
// past the batch's depth costs one visited-word load per wave (every vertex
// it could reach is visited); the check at the end of the forward sets one
// flag per level from the levels' vertex filters, and a backward level whose
// flag is clear exits at once.  The check also hands a batch back when its search had not ended
// within the L levels (level L holds a vertex) or a count needs 64-bit
// storage: it puts the batch on a list and clears every level flag, so the
// batch's backward launches exit and add nothing.  The host reads the list
// when the context is next used and re-runs those batches host-driven.  L is
// the most levels any batch has had so far.  The hybrid form's per-level
// choice is the one the last host-driven batch's densities give.

// End of a replayed batch's forward.  Block l (of L + 1) sets lvflag[l] from
// level l's vertex filter; the last block to finish checks the batch: it
// completed within the L levels when level L is empty, and its counts fit
// the storage when no kernel asked for 64 bits.  Otherwise its first source
// goes on the handed-back list and every level flag is cleared, so that its
// backward launches exit and add nothing.
__global__ __launch_bounds__(SB) void k_batch_check(BatchCtl *ctl, const uint32_t *__restrict__ any, int32_t aw,
                                                    uint32_t *lvflag, int32_t L, uint32_t *status, int32_t B) {
    __shared__ int s_last;
    const int32_t l = blockIdx.x;
    const uint32_t *a = any + (size_t)l * aw;
    uint32_t x = 0;
    for (int32_t i = threadIdx.x; i < aw; i += SB) x |= a[i];
    const int nz = __syncthreads_or(x != 0);
    if (threadIdx.x == 0) {
        __hip_atomic_store(&lvflag[l], nz ? 1u : 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        s_last = atomicAdd(&ctl->arrived, 1u) == (uint32_t)L;
    }
    __syncthreads();
    if (!s_last || threadIdx.x != 0) return;
    __threadfence();
    ctl->arrived = 0u;
    auto flag = [&](int32_t k) { return __hip_atomic_load(&lvflag[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); };
    const bool deep = flag(L) != 0, wide = status[1] != 0;
    if (deep || wide) {
        ctl->redo[ctl->redo_count++] = ctl->batch * B;
        if (wide) ctl->need_wide = 1u;
        if (deep) ctl->deep = 1u;
        for (int32_t k = 0; k <= L; ++k) __hip_atomic_store(&lvflag[k], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        status[1] = 0u;
    } else {
        uint32_t nlev = (uint32_t)L;
        for (int32_t k = 1; k <= L; ++k)
            if (flag(k) == 0u) {
                nlev = (uint32_t)k;
                break;
            }
        if (nlev > ctl->max_nlev) ctl->max_nlev = nlev;
    }
    ctl->batch += 1;
}

// Which levels of a replayed batch go by products: bit 0 forward l -> l+1,
// bit 1 backward l; as by_products, the backward also deciding from the last
// host-driven batch's densities.
std::vector<uint8_t> replay_plan(const bc_ctx *ctx, int32_t L) {
    std::vector<uint8_t> plan((size_t)L + 1, 0);
    const std::vector<double> &pd = ctx->hy.prev_density;
    for (int32_t l = 1; l <= L; ++l) {
        const bool f = by_products(ctx, l, true);
        const bool b = ctx->al.every_level ||
                       (ctx->hy.products && !ctx->edges && (size_t)l < pd.size() && pd[(size_t)l] >= ctx->hy.theta_bwd);
        plan[(size_t)l] = (uint8_t)((f ? 1 : 0) | (b ? 2 : 0));
    }
    return plan;
}

template <int NW, typename S>
bc_status record_batch_t(bc_ctx *ctx, int32_t L, const std::vector<uint8_t> &plan) {
    SparseState &s = ctx->sp;
    const BatchShape b = batch_shape<NW>(ctx);
    bc_status st = launch_batch_init<NW, S>(ctx, b, nullptr, 0, s.ctl);
    uint16_t *sig16 = sig16_of<S>(ctx);
    bool l1_pulled = false;
    for (int32_t l = 0; l < L && st == BC_OK; ++l)
        st = launch_fwd_level<NW, S>(ctx, b, l, l > 0 && (plan[(size_t)l] & 1), (plan[(size_t)l + 1] & 1) != 0, sig16,
                                     &l1_pulled);
    if (st != BC_OK) return st;
    {
        LaunchTimer tm(ctx, "batch_check");
        hipLaunchKernelGGL(k_batch_check, dim3(L + 1), dim3(SB), 0, ctx->stream, s.ctl, (const uint32_t *)s.any, b.aw,
                           s.lvflag, L, ctx->status, s.batch);
        tm.done();
    }
    // level 0 adds nothing to BC, but with edges on its arcs carry edge terms
    const int32_t lowest = ctx->edges ? 0 : 1;
    for (int32_t lv = L - 1; lv >= lowest && st == BC_OK; --lv)
        st = launch_bwd_level<NW, S>(ctx, b, lv, lv >= 1 && (plan[(size_t)lv] & 2), true, true, nullptr, true);
    if (st != BC_OK) return st;
    BC_HIP(ctx, hipGetLastError());
    return BC_OK;
}

template <int NW>
bc_status record_batch_nw(bc_ctx *ctx, int32_t L, const std::vector<uint8_t> &plan) {
    return ctx->sp.wide ? record_batch_t<NW, uint64_t>(ctx, L, plan) : record_batch_t<NW, uint32_t>(ctx, L, plan);
}

bc_status record_batch(bc_ctx *ctx, int32_t L, const std::vector<uint8_t> &plan) {
    switch (ctx->sp.words) {
    case 1: return record_batch_nw<1>(ctx, L, plan);
    case 2: return record_batch_nw<2>(ctx, L, plan);
    case 4: return record_batch_nw<4>(ctx, L, plan);
    case 8: return record_batch_nw<8>(ctx, L, plan);
    }
    return bc_fail(ctx, BC_ERR_INVALID_ARG, "sparse form: batch must be 64, 128, 256 or 512");
}

void destroy_graphs(bc_ctx *ctx) {
    SparseState &s = ctx->sp;
    if (s.gexec) hipGraphExecDestroy(s.gexec);
    s.gexec = nullptr;
}

// Records one batch on the private capture stream (nothing runs) and
// instantiates it.
bc_status capture_batch(bc_ctx *ctx, int32_t L, const std::vector<uint8_t> &plan) {
    SparseState &s = ctx->sp;
    destroy_graphs(ctx);
    if (!s.cap_stream) BC_HIP(ctx, hipStreamCreateWithFlags(&s.cap_stream, hipStreamNonBlocking));
    hipStream_t saved = ctx->stream;
    hipGraph_t graph = nullptr;
    bc_status st = BC_OK;
    hipError_t e = hipStreamBeginCapture(s.cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        ctx->stream = s.cap_stream;
        ctx->recording = true;
        st = record_batch(ctx, L, plan);
        ctx->stream = saved;
        ctx->recording = false;
        const hipError_t e2 = hipStreamEndCapture(s.cap_stream, &graph);
        if (e2 != hipSuccess) e = e2;
    }
    if (st == BC_OK && e == hipSuccess) e = hipGraphInstantiate(&s.gexec, graph, nullptr, nullptr, 0);
    if (graph) hipGraphDestroy(graph);
    if (st != BC_OK || e != hipSuccess) {
        s.gexec = nullptr;
        return st != BC_OK ? st : bc_hip(ctx, e, "recording a batch into a HIP graph");
    }
    return BC_OK;
}

// The recorded batch for the current depth, count width, state and level plan.
bc_status ensure_replay(bc_ctx *ctx) {
    SparseState &s = ctx->sp;
    const int32_t L = std::max(s.depth_max, 2);
    bc_status st = ensure_levels(ctx, L + 1);
    if (st != BC_OK) return st;
    const std::vector<uint8_t> plan = replay_plan(ctx, L);
    if (s.gexec && s.g_levels == L && s.g_wide == s.wide && s.g_front == (const void *)s.front && s.g_plan == plan)
        return BC_OK;
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream)); // no replay of the old graph is in flight
    st = capture_batch(ctx, L, plan);
    if (st != BC_OK) return st;
    s.g_levels = L;
    s.g_wide = s.wide;
    s.g_front = s.front;
    s.g_plan = plan;
    return BC_OK;
}

// A batch of a replayed run that ran host-driven instead: its replay's slot
// in the control block is passed over.
__global__ void k_ctl_skip(BatchCtl *ctl) {
    if (threadIdx.x == 0) ctl->batch += 1;
}

} // namespace

bc_status sparse_prepare(bc_ctx *ctx, int32_t batch, int32_t split_degree) {
    SparseState &s = ctx->sp;
    if (batch != 64 && batch != 128 && batch != 256 && batch != 512)
        return bc_fail(ctx, BC_ERR_INVALID_ARG, "sparse form: batch must be 64, 128, 256 or 512");
    s.batch = batch;
    s.words = batch / 64;
    s.split = split_degree > 0 ? split_degree : 128;
    {
        // launch shapes of the pulls: 32 blocks of four waves per compute
        // unit, each wave striding over the items.  Measured on RMAT-16 at
        // batch 256 against one wave per item: the backward took a step from
        // 181 to 173 ms host-driven and 182 to 171 ms replayed, the forward
        // then to 172 and 169 ms; 16 and 64 blocks per unit were slower.
        int cus = 0;
        BC_HIP(ctx, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
        s.bwd_grid = 32 * std::max(cus, 1);
        s.fwd_grid = 32 * std::max(cus, 1);
    }
    const int32_t n = ctx->n;
    const size_t nn = (size_t)std::max(n, 1);
    // Heavy rows and their segments, from the host copy of row_ptr.
    const std::vector<int32_t> &rp = ctx->h_row_ptr;
    std::vector<int32_t> heavy_id((size_t)n, -1), heavy_nseg, seg_v, seg_beg, seg_end;
    int32_t nheavy = 0;
    for (int32_t v = 0; v < n; ++v) {
        const int32_t deg = rp[v + 1] - rp[v];
        if (deg <= s.split) continue;
        heavy_id[v] = nheavy++;
        heavy_nseg.push_back((deg + s.split - 1) / s.split);
        for (int32_t b = rp[v]; b < rp[v + 1]; b += s.split) {
            seg_v.push_back(v);
            seg_beg.push_back(b);
            seg_end.push_back(std::min(b + s.split, rp[v + 1]));
        }
    }
    s.nheavy = nheavy;
    s.nseg = (int32_t)seg_v.size();
    const size_t nh = std::max<size_t>((size_t)nheavy, 1), ns = std::max<size_t>(seg_v.size(), 1);
    s.heavy_id = (int32_t *)bc_dalloc(ctx, nn * sizeof(int32_t));
    s.heavy_nseg = (int32_t *)bc_dalloc(ctx, nh * sizeof(int32_t));
    s.arrive = (uint32_t *)bc_dalloc(ctx, nh * sizeof(uint32_t));
    s.arrive_w = (uint32_t *)bc_dalloc(ctx, nh * s.words * sizeof(uint32_t));
    s.seg_v = (int32_t *)bc_dalloc(ctx, ns * sizeof(int32_t));
    s.seg_beg = (int32_t *)bc_dalloc(ctx, ns * sizeof(int32_t));
    s.seg_end = (int32_t *)bc_dalloc(ctx, ns * sizeof(int32_t));
    s.hacc = (double *)bc_dalloc(ctx, nh * batch * sizeof(double));
    s.visited = (uint64_t *)bc_dalloc(ctx, nn * s.words * sizeof(uint64_t));
    s.sigma = (uint64_t *)bc_dalloc(ctx, nn * batch * sizeof(uint64_t));
    s.cval = (float *)bc_dalloc(ctx, nn * batch * sizeof(float));
    s.src = (int32_t *)bc_dalloc(ctx, batch * sizeof(int32_t));
    s.ctl = (BatchCtl *)bc_dalloc(ctx, sizeof(BatchCtl));
    s.reach = (unsigned long long *)bc_dalloc(ctx, 256);
    if (!s.heavy_id || !s.heavy_nseg || !s.arrive || !s.arrive_w || !s.seg_v || !s.seg_beg || !s.seg_end || !s.hacc || !s.visited ||
        !s.sigma || !s.cval || !s.src || !s.ctl || !s.reach)
        return bc_fail(ctx, BC_ERR_NOMEM, "sparse form: state allocation failed");
    if (n > 0)
        BC_HIP(ctx, hipMemcpyAsync(s.heavy_id, heavy_id.data(), nn * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
    if (nheavy) {
        BC_HIP(ctx, hipMemcpyAsync(s.heavy_nseg, heavy_nseg.data(), (size_t)nheavy * sizeof(int32_t),
                                   hipMemcpyHostToDevice, ctx->stream));
        BC_HIP(ctx, hipMemcpyAsync(s.seg_v, seg_v.data(), seg_v.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
        BC_HIP(ctx, hipMemcpyAsync(s.seg_beg, seg_beg.data(), seg_v.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
        BC_HIP(ctx, hipMemcpyAsync(s.seg_end, seg_end.data(), seg_v.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
    }
    BC_HIP(ctx, hipMemsetAsync(s.arrive, 0, nh * sizeof(uint32_t), ctx->stream));
    BC_HIP(ctx, hipMemsetAsync(s.arrive_w, 0, nh * s.words * sizeof(uint32_t), ctx->stream));
    BC_HIP(ctx, hipMemsetAsync(s.hacc, 0, nh * batch * sizeof(double), ctx->stream));
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream)); // host vectors above go out of scope
    return ensure_levels(ctx, 16);
}

bc_status sparse_batch(bc_ctx *ctx, const int32_t *d_src, int32_t count, bool accumulate) {
    int32_t nlev = 0;
    return run_batch(ctx, d_src, count, accumulate, &nlev);
}

bc_status sparse_release(bc_ctx *ctx) {
    SparseState &s = ctx->sp;
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    sparse_graphs_release(ctx);
    for (void *p : {(void *)s.front, (void *)s.any, (void *)s.lvmax, (void *)s.lvflag, (void *)s.visited,
                    (void *)s.sigma, (void *)s.cval, (void *)s.src, (void *)s.heavy_id,
                    (void *)s.heavy_nseg, (void *)s.arrive, (void *)s.arrive_w, (void *)s.seg_v, (void *)s.seg_beg,
                    (void *)s.seg_end, (void *)s.hacc, (void *)s.ctl, (void *)s.redo, (void *)s.reach})
        if (p) bc_dfree(ctx, p);
    if (s.any_host) hipHostFree(s.any_host);
    s = SparseState{};
    return BC_OK;
}

bc_status sparse_run(bc_ctx *ctx, const int32_t *d_src, int64_t count) {
    SparseState &s = ctx->sp;
    const int32_t B = s.batch;
    const bool replay = !ctx->weighted && !ctx->host_driven && count < (int64_t(1) << 31) - B;
    int64_t b0 = 0;
    // Host-driven batches: every batch without replay; with replay the first
    // batch a state runs, which gives the depth and the level densities.
    for (; b0 < count && (!replay || s.depth_max == 0); b0 += B) {
        int32_t nlev = 0;
        bc_timing_batch(ctx); // with sampled timing, this batch's launches are timed or not as a whole
        bc_timing_eager(ctx);
        bc_status st = run_batch(ctx, d_src + b0, (int32_t)std::min<int64_t>(B, count - b0), true, &nlev);
        if (st != BC_OK) return st;
    }
    if (b0 >= count) return BC_OK;
    bc_status st = ensure_replay(ctx);
    if (st != BC_OK) return st;
    const int64_t rest = count - b0, nb = (rest + B - 1) / B;
    if (nb > s.redo_cap) {
        int32_t *r = (int32_t *)bc_dalloc(ctx, (size_t)nb * sizeof(int32_t));
        if (!r) return bc_fail(ctx, BC_ERR_NOMEM, "sparse form: allocation of the handed-back list failed");
        bc_dfree(ctx, s.redo);
        s.redo = r;
        s.redo_cap = nb;
    }
    hipLaunchKernelGGL(k_run_init, dim3(1), dim3(64), 0, ctx->stream, s.ctl, d_src + b0, (int32_t)rest, s.redo);
    BC_HIP(ctx, hipGetLastError());
    s.g_pending = true; // from here on the device holds checks the host must read
    for (int64_t i = 0; i < nb; ++i) {
        bc_timing_batch(ctx);
        if (ctx->timing && ctx->timing_sel) {
            // a timed batch runs host-driven, so that its launches carry events
            bc_timing_eager(ctx);
            const int64_t off = b0 + i * B;
            int32_t nlev = 0;
            st = run_batch(ctx, d_src + off, (int32_t)std::min<int64_t>(B, count - off), true, &nlev);
            if (st != BC_OK) return st;
            hipLaunchKernelGGL(k_ctl_skip, dim3(1), dim3(64), 0, ctx->stream, s.ctl);
            BC_HIP(ctx, hipGetLastError());
            // it may have grown the level storage or switched to 64-bit counts
            if ((st = ensure_replay(ctx)) != BC_OK) return st;
            continue;
        }
        BC_HIP(ctx, hipGraphLaunch(s.gexec, ctx->stream));
    }
    return BC_OK;
}

bc_status sparse_settle(bc_ctx *ctx) {
    SparseState &s = ctx->sp;
    if (!s.g_pending) return BC_OK;
    s.g_pending = false;
    BatchCtl c{};
    BC_HIP(ctx, hipMemcpyAsync(&c, s.ctl, sizeof c, hipMemcpyDeviceToHost, ctx->stream));
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    s.depth_max = std::max(s.depth_max, (int32_t)c.max_nlev);
    s.depth_guess = std::max(s.depth_guess, (int32_t)c.max_nlev);
    ctx->max_levels = std::max(ctx->max_levels, (int32_t)c.max_nlev);
    if (c.redo_count == 0) return BC_OK;
    std::vector<int32_t> redo(c.redo_count);
    BC_HIP(ctx, hipMemcpy(redo.data(), s.redo, redo.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (c.need_wide) s.wide = true; // sticky, as on the host-driven path
    for (const int32_t b0 : redo) {
        int32_t nlev = 0;
        bc_status st = run_batch(ctx, c.src + b0, std::min(s.batch, c.total - b0), true, &nlev);
        if (st != BC_OK) return st;
    }
    return BC_OK;
}

void sparse_graphs_release(bc_ctx *ctx) {
    SparseState &s = ctx->sp;
    hipStreamSynchronize(ctx->stream); // no replay is in flight
    destroy_graphs(ctx);
    if (s.cap_stream) hipStreamDestroy(s.cap_stream);
    s.cap_stream = nullptr;
    s.g_pending = false;
}

bc_status sparse_dump(bc_ctx *ctx, const int32_t *d_src, int32_t count,
                      int32_t *dist_dump, uint64_t *sigma_dump, double *delta_dump) {
    SparseState &s = ctx->sp;
    int32_t nlev = 0;
    bc_status st = run_batch(ctx, d_src, count, false, &nlev, delta_dump != nullptr, delta_dump);
    if (st != BC_OK) return st;
    const int64_t cells = (int64_t)ctx->n * count;
    const unsigned blocks = (unsigned)((cells + SB - 1) / SB);
    if (s.wide)
        hipLaunchKernelGGL(k_sp_dump<uint64_t>, dim3(blocks), dim3(SB), 0, ctx->stream, ctx->n, s.words, s.batch, count,
                           nlev, s.front, (const uint64_t *)s.sigma, dist_dump, sigma_dump, delta_dump);
    else
        hipLaunchKernelGGL(k_sp_dump<uint32_t>, dim3(blocks), dim3(SB), 0, ctx->stream, ctx->n, s.words, s.batch, count,
                           nlev, s.front, (const uint32_t *)s.sigma, dist_dump, sigma_dump, delta_dump);
    BC_HIP(ctx, hipGetLastError());
    return BC_OK;
}
