// The sampled forward of Sec. 4.1.1 (Algorithm 1) for unweighted graphs,
// distances only.  With a distinguished set S (the requested sources first,
// then the caller's random sample) it runs four stages:
//   limited searches  a breadth-first search from every x in S that stops
//                     after k hops gives d'(x, v): the hop distance when it
//                     is at most k, otherwise none;
//   graph on S        H on the vertices of S, the weight of x-y being d'(x, y);
//   closure           all-pairs distances D_H of H (Floyd-Warshall);
//   combination       d(s, v) = min over x in S of D_H(s, x) + d'(x, v).
// The algorithm's count of minimising vertices is not a count of shortest
// paths and is not computed.
//
// Layout (sp = |S| rounded up to 64, W = sp / 64 bitmap words):
//   d'    uint16 dT[v][sp], vertex-major: dT[v][x] = d'(S_x, v), DINF = none
//   bits  visited sets and the new bits of each level (a ring of 8 levels,
//         the last being the frontier) as uint64 [v][W]: bit x of vertex v's
//         words is row x of S
//   H     int32 [sp][sp], HINF = no path (HINF + HINF fits int32); D_H in place
// The limited searches advance every row of S together, one launch per level:
// a wave takes a chunk of at most CH arcs of one vertex, lane w pulls word w of
// each neighbour's frontier; vertices with more than CH arcs leave one partial
// OR per chunk, merged by a second launch.  Every 8 levels the new bits become
// d' entries, sixteen bytes per thread.  Floyd-Warshall runs in 64 x 64
// tiles: per pivot block, the diagonal tile, then the column strip and then
// the whole (symmetric) matrix as min-plus products.  The combination is the
// min-plus product of the sources' rows of D_H with d', in LDS-staged
// 128 x 128 tiles.
#include "bc_internal.h"

#include <algorithm>
#include <cmath>
#include <unordered_map>

namespace {

constexpr int SB = 256;
constexpr uint16_t DINF = 0xFFFF;
constexpr int32_t HINF = 1 << 29;
constexpr int CH = 128; // arcs per chunk of a search level
constexpr int TB = 64;  // Floyd-Warshall tile
constexpr int KC = 32;  // k step of the min-plus products

inline unsigned blocks_for(size_t count) { return (unsigned)((count + SB - 1) / SB); }

// Bits of word w that are rows of S.
__device__ inline uint64_t word_rows(int32_t w, int32_t ns) {
    const int32_t r = ns - 64 * w;
    return r >= 64 ? ~0ull : r <= 0 ? 0ull : ((1ull << r) - 1);
}

// Level 0: row i of S starts at its own vertex (S has no repeats, so each
// vertex's words hold at most one bit here; the bitmaps were cleared).
__global__ __launch_bounds__(SB) void k_ls_sources(int32_t ns, const int32_t *__restrict__ S, int32_t W,
                                                   uint64_t *__restrict__ F, uint64_t *__restrict__ V) {
    const int32_t i = blockIdx.x * SB + threadIdx.x;
    if (i >= ns) return;
    const int32_t v = S[i];
    const uint64_t bit = 1ull << (i & 63);
    F[(size_t)v * W + (i >> 6)] = bit;
    V[(size_t)v * W + (i >> 6)] = bit;
}

// New bits of vertex v at level L: they are its next-frontier word (kept for
// the flush into d') and join its visited word.
__device__ inline void ls_settle(int32_t v, int lane, int32_t W, uint64_t acc, uint64_t vis, uint64_t rows,
                                 int32_t L, uint64_t *__restrict__ N, uint64_t *__restrict__ V,
                                 uint32_t *__restrict__ found) {
    const uint64_t nw = acc & ~vis & rows;
    if (lane < W) {
        N[(size_t)v * W + lane] = nw;
        if (nw) V[(size_t)v * W + lane] = vis | nw;
    }
    if (__builtin_amdgcn_ballot_w64(nw != 0) != 0 && lane == 0) found[L] = 1;
}

// d' from the new-bit words of levels L0 .. L0 + nl - 1 (ring slot L % RING,
// nl <= RING).  A block takes 32 words: it stages their slot words in LDS (one
// coalesced load per thread), then thread (word, g) owns the sixteen bytes of
// entries 64w + 8g .. + 7 of row v of dT, so a wave stores one contiguous
// kilobyte.  Levels that found nothing are skipped (their slots were not
// rewritten).  The slots' bits are disjoint, so the slot index of an entry is
// read off three OR-planes of the slot words (bit j of the index: the OR of
// the slots whose index has bit j).  The first flush writes every entry (DINF
// where no level set it); later ones read, merge and write back the groups
// that gained entries.
constexpr int RING = 8;
constexpr int FW_WORDS = SB / 8; // words per block of the flush
__global__ __launch_bounds__(SB) void k_ls_flush(int32_t n, int32_t W, int32_t sp, const uint64_t *__restrict__ ring,
                                                 int32_t L0, int32_t nl, int32_t first,
                                                 const uint32_t *__restrict__ found, uint16_t *__restrict__ dT) {
    __shared__ uint64_t sw[RING][FW_WORDS];
    uint32_t live = 0; // bit q: level L0 + q found something (level 0: the sources)
    for (int32_t q = 0; q < nl; ++q)
        if (L0 + q == 0 || found[L0 + q]) live |= 1u << q;
    if (!first && !live) return;
    const size_t words = (size_t)n * W;
    const size_t base = (size_t)blockIdx.x * FW_WORDS;
    {
        const int q = threadIdx.x / FW_WORDS, i = threadIdx.x % FW_WORDS;
        uint64_t x = 0;
        if (((live >> q) & 1u) && base + i < words) x = ring[(size_t)((L0 + q) % RING) * words + base + i];
        sw[q][i] = x;
    }
    __syncthreads();
    const int i = threadIdx.x >> 3, g = threadIdx.x & 7;
    const size_t vw = base + i;
    if (vw >= words) return;
    uint32_t ga = 0, g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
    for (int q = 0; q < RING; ++q) {
        const uint32_t x = (uint32_t)(sw[q][i] >> (8 * g)) & 0xFFu;
        ga |= x;
        if (q & 1) g0 |= x;
        if (q & 2) g1 |= x;
        if (q & 4) g2 |= x;
    }
    if (!first && !ga) return;
    const int32_t v = (int32_t)(vw / W), w = (int32_t)(vw % W);
    uint4 *dst = (uint4 *)(dT + (size_t)v * sp + 64 * w + 8 * g);
    uint32_t out[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
    if (!first) {
        const uint4 o = *dst;
        out[0] = o.x;
        out[1] = o.y;
        out[2] = o.z;
        out[3] = o.w;
    }
#pragma unroll
    for (int b = 0; b < 8; ++b)
        if ((ga >> b) & 1u) {
            const uint32_t lv = (uint32_t)L0 + (((g0 >> b) & 1u) | (((g1 >> b) & 1u) << 1) | (((g2 >> b) & 1u) << 2));
            const int sh = 16 * (b & 1);
            out[b >> 1] = (out[b >> 1] & ~(0xFFFFu << sh)) | (lv << sh);
        }
    *dst = make_uint4(out[0], out[1], out[2], out[3]);
}

// Level L: one wave per chunk (v, first arc); chunks below nsplit belong to
// vertices with more than CH arcs and leave their OR in P.
__global__ __launch_bounds__(SB) void k_ls_level(int32_t nchunks, int32_t nsplit, const int2 *__restrict__ chunks,
                                                 const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                 int32_t W, int32_t ns, int32_t L, const uint64_t *__restrict__ F, uint64_t *__restrict__ N,
                                                 uint64_t *__restrict__ V, uint64_t *__restrict__ P,
                                                 uint32_t *__restrict__ found) {
    if (L > 1 && found[L - 1] == 0) return; // empty frontier: nothing to do, the flush skips this level
    const int lane = threadIdx.x & 63;
    const int32_t c = __builtin_amdgcn_readfirstlane(blockIdx.x * (SB / 64) + (threadIdx.x >> 6));
    if (c >= nchunks) return;
    const int2 ch = chunks[c];
    const int32_t v = ch.x;
    const uint64_t rows = word_rows(lane, ns);
    const uint64_t vis = lane < W ? V[(size_t)v * W + lane] : 0;
    uint64_t acc = 0;
    if (__builtin_amdgcn_ballot_w64(vis != rows) != 0) {
        const int32_t e1 = min(ch.y + CH, rp[v + 1]);
        const uint64_t *Fl = F + lane;
        int32_t e = ch.y;
        for (; e + 8 <= e1; e += 8) {
            int32_t u[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) u[q] = col[e + q];
            if (lane < W) {
                uint64_t a = 0;
#pragma unroll
                for (int q = 0; q < 8; ++q) a |= Fl[(size_t)u[q] * W];
                acc |= a;
            }
        }
        for (; e < e1; ++e) {
            const int32_t u = col[e];
            if (lane < W) acc |= Fl[(size_t)u * W];
        }
    }
    if (c < nsplit) {
        if (lane < W) P[(size_t)c * W + lane] = acc;
        return;
    }
    ls_settle(v, lane, W, acc, vis, rows, L, N, V, found);
}

// Level L for the split vertices: OR of their chunks' partial results.
__global__ __launch_bounds__(SB) void k_ls_finish(int32_t nsv, const int32_t *__restrict__ sv,
                                                  const int32_t *__restrict__ sc, int32_t W, int32_t ns, int32_t L, const uint64_t *__restrict__ P, uint64_t *__restrict__ N,
                                                  uint64_t *__restrict__ V, uint32_t *__restrict__ found) {
    if (L > 1 && found[L - 1] == 0) return;
    const int lane = threadIdx.x & 63;
    const int32_t j = __builtin_amdgcn_readfirstlane(blockIdx.x * (SB / 64) + (threadIdx.x >> 6));
    if (j >= nsv) return;
    const int32_t v = sv[j];
    uint64_t acc = 0;
    if (lane < W) {
        const int32_t ce = sc[j + 1];
        int32_t c = sc[j];
        for (; c + 4 <= ce; c += 4)
            acc |= P[(size_t)c * W + lane] | P[(size_t)(c + 1) * W + lane] | P[(size_t)(c + 2) * W + lane] |
                   P[(size_t)(c + 3) * W + lane];
        for (; c < ce; ++c) acc |= P[(size_t)c * W + lane];
    }
    const uint64_t vis = lane < W ? V[(size_t)v * W + lane] : 0;
    ls_settle(v, lane, W, acc, vis, word_rows(lane, ns), L, N, V, found);
}

// The graph on S: H[j][i] = d'(S_i, S_j) = dT[S_j][i] (symmetric: the graph is
// undirected); 0 on the diagonal, HINF where no path was found and in the
// padding.
__global__ __launch_bounds__(SB) void k_build_h(int32_t ns, int32_t sp, const int32_t *__restrict__ S,
                                                const uint16_t *__restrict__ dT, int32_t *__restrict__ H) {
    const size_t id = (size_t)blockIdx.x * SB + threadIdx.x;
    if (id >= (size_t)sp * sp) return;
    const int32_t j = (int32_t)(id / sp), i = (int32_t)(id % sp);
    int32_t h = HINF;
    if (i == j) h = 0;
    else if (i < ns && j < ns) {
        const uint16_t d = dT[(size_t)S[j] * sp + i];
        h = d == DINF ? HINF : (int32_t)d;
    }
    H[id] = h;
}

// The closure in 64 x 64 tiles, rounds r = 0 .. sp/64 - 1 over the pivot blocks.
// Every step only lowers an entry to the length of some walk, and every
// entry ends at the shortest one, so each phase may see entries of a tile
// before or after another phase's update of the same values.
//
// Phase 1: the diagonal tile (r, r) closed on its own: repeated min-plus
// squaring of the tile (diagonal 0, so k squarings give the shortest walks of
// at most 2^k edges; 6 cover every simple path of 64 vertices), stopping once
// a squaring changes nothing.  The tile is in LDS s[64][TP] and in c (thread
// t: rows 4 (t >> 4) .., columns 4 (t & 15) ..); both hold the result.
constexpr int TP = TB + 4; // LDS pitch of a closed tile (16-byte aligned rows)
__device__ void close_tile(int32_t *s, int32_t (&c)[4][4]) {
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
    for (int it = 0; it < 6; ++it) {
        int32_t nc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) nc[i][j] = c[i][j];
        for (int k = 0; k < TB; k += 2) {
            int2 a[4];
            int4 b0 = *(const int4 *)&s[k * TP + tx * 4], b1 = *(const int4 *)&s[(k + 1) * TP + tx * 4];
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] = *(const int2 *)&s[(ty * 4 + q) * TP + k];
            const int32_t r0[4] = {b0.x, b0.y, b0.z, b0.w}, r1[4] = {b1.x, b1.y, b1.z, b1.w};
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) nc[i][j] = min(min(nc[i][j], a[i].x + r0[j]), a[i].y + r1[j]);
        }
        int changed = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) changed |= nc[i][j] != c[i][j];
        __syncthreads(); // every read of this squaring is done
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                c[i][j] = nc[i][j];
                s[(ty * 4 + i) * TP + tx * 4 + j] = nc[i][j];
            }
        if (!__syncthreads_or(changed)) break;
    }
}

// Phase 1 as its own launch (the first pivot block; later diagonal tiles are
// closed inside the previous round's phase 3).
__global__ __launch_bounds__(SB) void k_fw_diag(int32_t sp, int32_t r, int32_t *__restrict__ D) {
    __shared__ __attribute__((aligned(16))) int32_t s[TB * TP];
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
    int32_t *base = D + (size_t)r * TB * sp + (size_t)r * TB;
    int32_t c[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            c[i][j] = base[(size_t)(ty * 4 + i) * sp + tx * 4 + j];
            s[(ty * 4 + i) * TP + tx * 4 + j] = c[i][j];
        }
    __syncthreads();
    close_tile(s, c);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) base[(size_t)(ty * 4 + i) * sp + tx * 4 + j] = c[i][j];
}

inline __device__ int32_t as_dist(int32_t x) { return x; }
inline __device__ int32_t as_dist(uint16_t x) { return x == DINF ? HINF : (int32_t)x; }

enum MinPlusMode { MP_OUT = 0, MP_LOWER = 1, MP_LOWER_SYM = 2 };

// Min-plus product over k of A[m][k] + B[n][k]: A int32 [M][lda], B [N][ldb]
// (int32, or uint16 distances with DINF), both with k contiguous, K a
// multiple of KC, rows 16-byte aligned; with brow, column n takes B row
// brow[n].  Tiles of T = 16R rows and columns; 256 threads, each an R x R
// block, through k-major LDS in KC steps (the next step's operands load while
// this one computes), two k per step so that the compiler fuses the two
// minima (v_min3).
//   MP_OUT        C = the product, -1 where it stays HINF or above
//   MP_LOWER      C = min(C, product), stored only where it decreases; with
//                 CT, also CT[n][m] where the result is below it
//   MP_LOWER_SYM  as MP_LOWER on a symmetric C (M = N): the blocks take the
//                 tiles (bm, bn) with bm <= bn except those in tile row or
//                 column `blk`, and store each decrease at (m, n) and (n, m);
//                 with R = 4, the block of diagonal tile (closeb, closeb) then
//                 closes that tile (phase 1 of the next round, which no other
//                 block of this launch reads)
// In the lowering modes an entry that does not decrease is never written, so
// other blocks may read it concurrently.  With a gate, the launch does nothing
// unless *gate is nonzero.
template <int R, int MODE, typename BT>
__global__ __launch_bounds__(SB) void k_minplus(int32_t M, int32_t N, int32_t K, const int32_t *A, int64_t lda,
                                                const BT *B, int64_t ldb, const int32_t *brow, int32_t *C,
                                                int64_t ldc, int32_t *CT, int32_t blk, int32_t closeb,
                                                const uint32_t *gate) {
    constexpr int T = 16 * R, P = T + 4;
    constexpr bool B16 = sizeof(BT) == 2;
    if (gate && *gate == 0) return; // the 16-bit product below runs instead
    __shared__ __attribute__((aligned(16))) int32_t smem[2 * KC * P];
    int32_t(*sA)[P] = (int32_t(*)[P])smem;
    int32_t(*sB)[P] = (int32_t(*)[P])(smem + KC * P);
    static_assert(R != 4 || 2 * KC * P >= TB * TP, "a closed tile fits the staging area");
    const int t = threadIdx.x;
    int32_t bm = blockIdx.y, bn = blockIdx.x;
    if (MODE == MP_LOWER_SYM) {
        // blockIdx.x enumerates the tiles (bm, bn) with bm <= bn
        const int32_t id = blockIdx.x;
        int32_t j = (int32_t)((sqrtf(8.0f * (float)id + 1.0f) - 1.0f) * 0.5f);
        while (j * (j + 1) / 2 > id) --j;
        while ((j + 1) * (j + 2) / 2 <= id) ++j;
        bn = j;
        bm = id - j * (j + 1) / 2;
        if (bm == blk || bn == blk) return; // the strips are final after phase 2
    }
    const int32_t m0 = bm * T, n0 = bn * T;
    const int ty = t >> 4, tx = t & 15;
    // staging registers: A rows (t >> 3) + 32p, four int32 at k (t & 7) * 4;
    // B likewise, or (16-bit) rows (t >> 2) + 64p, eight uint16 at k (t & 3) * 8
    constexpr int NA = T / 32, NB = B16 ? T / 64 : T / 32;
    int4 ra[NA];
    uint4 rb[NB];
    const BT *brows[NB];
#pragma unroll
    for (int p = 0; p < NB; ++p) {
        const int32_t n = n0 + (B16 ? (t >> 2) + 64 * p : (t >> 3) + 32 * p);
        brows[p] = n < N ? B + (size_t)(brow ? brow[n] : n) * ldb : nullptr;
    }
    auto load = [&](int32_t k0) {
#pragma unroll
        for (int p = 0; p < NA; ++p) {
            const int32_t m = m0 + (t >> 3) + 32 * p;
            ra[p] = m < M ? *(const int4 *)(A + (size_t)m * lda + k0 + (t & 7) * 4)
                          : make_int4(HINF, HINF, HINF, HINF);
        }
#pragma unroll
        for (int p = 0; p < NB; ++p) {
            const int kk = B16 ? (t & 3) * 8 : (t & 7) * 4;
            if (brows[p]) rb[p] = *(const uint4 *)(brows[p] + k0 + kk);
            else rb[p] = B16 ? make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu)
                             : make_uint4(HINF, HINF, HINF, HINF);
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int p = 0; p < NA; ++p) {
            const int row = (t >> 3) + 32 * p, k = (t & 7) * 4;
            sA[k][row] = ra[p].x;
            sA[k + 1][row] = ra[p].y;
            sA[k + 2][row] = ra[p].z;
            sA[k + 3][row] = ra[p].w;
        }
#pragma unroll
        for (int p = 0; p < NB; ++p) {
            const uint32_t wv[4] = {rb[p].x, rb[p].y, rb[p].z, rb[p].w};
            if constexpr (B16) {
                const int row = (t >> 2) + 64 * p, k = (t & 3) * 8;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    sB[k + 2 * q][row] = as_dist((uint16_t)(wv[q] & 0xFFFF));
                    sB[k + 2 * q + 1][row] = as_dist((uint16_t)(wv[q] >> 16));
                }
            } else {
                const int row = (t >> 3) + 32 * p, k = (t & 7) * 4;
#pragma unroll
                for (int q = 0; q < 4; ++q) sB[k + q][row] = (int32_t)wv[q];
            }
        }
    };
    load(0);
    int32_t c[R][R], c0[MODE == MP_OUT ? 1 : R][MODE == MP_OUT ? 1 : R],
        ct0[MODE == MP_LOWER ? R : 1][MODE == MP_LOWER ? R : 1];
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) {
            int32_t x = HINF;
            if constexpr (MODE != MP_OUT) {
                const int32_t m = m0 + ty * R + i, n = n0 + tx * R + j;
                const bool in = m < M && n < N;
                if (in) x = C[(size_t)m * ldc + n];
                c0[i][j] = x;
                // the transposed entries: written only by this block, at the end
                if constexpr (MODE == MP_LOWER) ct0[i][j] = in && CT ? CT[(size_t)n * ldc + m] : HINF;
            }
            c[i][j] = x;
        }
    for (int32_t k0 = 0; k0 < K; k0 += KC) {
        stage();
        __syncthreads();
        if (k0 + KC < K) load(k0 + KC);
        constexpr int UNR = R == 8 ? 2 : 1;
#pragma unroll UNR
        for (int k = 0; k < KC; k += 2) {
            int32_t a0[R], a1[R], b0[R], b1[R];
#pragma unroll
            for (int h = 0; h < R; h += 4) {
                *(int4 *)&a0[h] = *(const int4 *)&sA[k][ty * R + h];
                *(int4 *)&a1[h] = *(const int4 *)&sA[k + 1][ty * R + h];
                *(int4 *)&b0[h] = *(const int4 *)&sB[k][tx * R + h];
                *(int4 *)&b1[h] = *(const int4 *)&sB[k + 1][tx * R + h];
            }
#pragma unroll
            for (int i = 0; i < R; ++i)
#pragma unroll
                for (int j = 0; j < R; ++j) c[i][j] = min(min(c[i][j], a0[i] + b0[j]), a1[i] + b1[j]);
        }
        __syncthreads();
    }
    if constexpr (MODE == MP_LOWER_SYM && R == 4) {
        if (bm == closeb && bn == closeb) {
#pragma unroll
            for (int i = 0; i < R; ++i)
#pragma unroll
                for (int j = 0; j < R; ++j) smem[(ty * R + i) * TP + tx * R + j] = c[i][j];
            __syncthreads();
            close_tile(smem, c);
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int32_t m = m0 + ty * R + i;
        if (m >= M) continue;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int32_t n = n0 + tx * R + j;
            if (n >= N) continue;
            if constexpr (MODE == MP_OUT) {
                C[(size_t)m * ldc + n] = c[i][j] >= HINF ? -1 : c[i][j];
            } else {
                // (n, m) equals (m, n) before the update: the tiles read here
                // hold no strip entry, and the matrix is symmetric elsewhere
                if (c[i][j] < c0[i][j]) {
                    C[(size_t)m * ldc + n] = c[i][j];
                    if (MODE == MP_LOWER_SYM && bm != bn) C[(size_t)n * ldc + m] = c[i][j];
                }
                if constexpr (MODE == MP_LOWER)
                    if (CT && c[i][j] < ct0[i][j]) CT[(size_t)n * ldc + m] = c[i][j];
            }
        }
    }
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// The sources' rows of D_H as uint16 (DINF where none) for the 16-bit final
// product; *wide = 1 when some finite value exceeds cap = 65534 - k, so that a
// sum could pass 65534 (the 32-bit product runs then).
__global__ __launch_bounds__(SB) void k_dh16(int32_t M, int32_t sp, const int32_t *__restrict__ DH, int32_t cap,
                                             uint16_t *__restrict__ A16, uint32_t *__restrict__ wide) {
    const size_t id = (size_t)blockIdx.x * SB + threadIdx.x;
    if (id >= (size_t)M * sp) return;
    const int32_t d = DH[id];
    const bool fin = d < HINF;
    A16[id] = fin ? (uint16_t)min(d, (int32_t)DINF) : DINF;
    if (fin && d > cap) *wide = 1;
}

// The combination in 16-bit arithmetic: C[m][n] = min over k of A[m][k] + B[n'][k], A
// and B uint16 [rows][sp] with k contiguous, DINF = none, n' = brow[n] (or n); each sum saturates at
// 65535 (v_pk_add_u16 with clamp) and two columns share one register
// (v_pk_min_u16), one instruction per term for the add and the minimum.
// Exact while every finite D_H entry plus every finite d' stays below 65535,
// which the gate guarantees: the launch does nothing when *wide is set.  Tiles
// of 128 x 128 through k-major LDS in steps of 64; each thread an 8 x 8 block;
// result -1 where no walk was found.
constexpr int KH = 64, PH = 128 + 8; // k step and LDS pitch (uint16) of the 16-bit product

// Eight k values of rows r and r + 1 (x0, x1: one 16-byte load each) into the
// k-major tile, each k as one 32-bit word holding both rows.
__device__ inline void stage_pairs(uint16_t (*s)[PH], int kk, int r, uint4 x0, uint4 x1) {
    const uint32_t u0[4] = {x0.x, x0.y, x0.z, x0.w}, u1[4] = {x1.x, x1.y, x1.z, x1.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        *(uint32_t *)&s[kk + 2 * q][r] = (u0[q] & 0xFFFFu) | (u1[q] << 16);
        *(uint32_t *)&s[kk + 2 * q + 1][r] = (u0[q] >> 16) | (u1[q] & 0xFFFF0000u);
    }
}
__global__ __launch_bounds__(SB) void k_minplus16(int32_t M, int32_t N, int32_t K, const uint16_t *__restrict__ A,
                                                  const uint16_t *__restrict__ B, int64_t ld,
                                                  const int32_t *__restrict__ brow, int32_t *__restrict__ C,
                                                  int64_t ldc, const uint32_t *__restrict__ wide) {
    if (*wide != 0) return;
    __shared__ __attribute__((aligned(16))) uint16_t sA[KH][PH];
    __shared__ __attribute__((aligned(16))) uint16_t sB[KH][PH];
    const int t = threadIdx.x;
    const int32_t m0 = blockIdx.y * 128, n0 = blockIdx.x * 128;
    const int ty = t >> 4, tx = t & 15;
    u16x2 c[8][4];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) c[i][j] = (u16x2){DINF, DINF};
    // staging: thread t loads rows 2 (t & 63) and 2 (t & 63) + 1 at k chunks
    // ((t >> 6) + 4p) * 8 and writes each k as one 32-bit pair of rows
    const int pr = 2 * (t & 63);
    const uint16_t *bp0 = n0 + pr < N ? B + (size_t)(brow ? brow[n0 + pr] : n0 + pr) * ld : nullptr;
    const uint16_t *bp1 = n0 + pr + 1 < N ? B + (size_t)(brow ? brow[n0 + pr + 1] : n0 + pr + 1) * ld : nullptr;
    // the next k step's staging words, loaded while this one computes:
    // rows pr and pr + 1 of A and of B at k chunks kk0 and kk1
    const int kk0 = (t >> 6) * 8, kk1 = kk0 + 32;
    const uint4 none = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
    const uint16_t *ap0 = m0 + pr < M ? A + (size_t)(m0 + pr) * ld : nullptr;
    const uint16_t *ap1 = m0 + pr + 1 < M ? A + (size_t)(m0 + pr + 1) * ld : nullptr;
    uint4 a00, a01, a10, a11, b00, b01, b10, b11; // [chunk][row of the pair]
#define MP16_LOAD(k0)                                                                                          \
    do {                                                                                                       \
        a00 = ap0 ? *(const uint4 *)(ap0 + (k0) + kk0) : none;                                                 \
        a01 = ap1 ? *(const uint4 *)(ap1 + (k0) + kk0) : none;                                                 \
        a10 = ap0 ? *(const uint4 *)(ap0 + (k0) + kk1) : none;                                                 \
        a11 = ap1 ? *(const uint4 *)(ap1 + (k0) + kk1) : none;                                                 \
        b00 = bp0 ? *(const uint4 *)(bp0 + (k0) + kk0) : none;                                                 \
        b01 = bp1 ? *(const uint4 *)(bp1 + (k0) + kk0) : none;                                                 \
        b10 = bp0 ? *(const uint4 *)(bp0 + (k0) + kk1) : none;                                                 \
        b11 = bp1 ? *(const uint4 *)(bp1 + (k0) + kk1) : none;                                                 \
    } while (0)
    MP16_LOAD(0);
    for (int32_t k0 = 0; k0 < K; k0 += KH) {
        stage_pairs(sA, kk0, pr, a00, a01);
        stage_pairs(sA, kk1, pr, a10, a11);
        stage_pairs(sB, kk0, pr, b00, b01);
        stage_pairs(sB, kk1, pr, b10, b11);
        __syncthreads();
        if (k0 + KH < K) MP16_LOAD(k0 + KH);
#pragma unroll 4
        for (int k = 0; k < KH; ++k) {
            const uint4 av = *(const uint4 *)&sA[k][ty * 8];
            const uint4 bv = *(const uint4 *)&sB[k][tx * 8];
            const uint32_t aw[4] = {av.x, av.y, av.z, av.w};
            const u16x2 b[4] = {__builtin_bit_cast(u16x2, bv.x), __builtin_bit_cast(u16x2, bv.y),
                                __builtin_bit_cast(u16x2, bv.z), __builtin_bit_cast(u16x2, bv.w)};
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const unsigned short ai = (unsigned short)((i & 1) ? (aw[i >> 1] >> 16) : (aw[i >> 1] & 0xFFFF));
                const u16x2 a2 = (u16x2){ai, ai};
#pragma unroll
                for (int j = 0; j < 4; ++j) c[i][j] = __builtin_elementwise_min(c[i][j], __builtin_elementwise_add_sat(a2, b[j]));
            }
        }
        __syncthreads();
    }
#undef MP16_LOAD
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int32_t m = m0 + ty * 8 + i;
        if (m >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int32_t n = n0 + tx * 8 + 2 * j;
            const int32_t lo = c[i][j].x, hi = c[i][j].y;
            if (n < N) C[(size_t)m * ldc + n] = lo == DINF ? -1 : lo;
            if (n + 1 < N) C[(size_t)m * ldc + n + 1] = hi == DINF ? -1 : hi;
        }
    }
}

// out[i] = in[row[i]]: rows in the requested order, repeats included.
__global__ __launch_bounds__(SB) void k_pick_rows(int32_t n, int32_t count, const int32_t *__restrict__ row,
                                                  const int32_t *__restrict__ in, int32_t *__restrict__ out) {
    const int32_t v = blockIdx.x * SB + threadIdx.x;
    if (v >= n) return;
    for (int32_t i = blockIdx.y; i < count; i += gridDim.y) out[(size_t)i * n + v] = in[(size_t)row[i] * n + v];
}

} // namespace

bc_status sampled_distances(bc_ctx *ctx, const int32_t *h_sources, int32_t count, const int32_t *h_sample,
                            int32_t nsample, int32_t limit, int32_t *out, bool out_on_device) {
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
    bool in_order = true; // row_of[i] == i: no repeats among the sources
    for (int32_t i = 0; i < count; ++i) {
        nreq = std::max(nreq, row_of[(size_t)i] + 1);
        in_order = in_order && row_of[(size_t)i] == i;
    }
    if (ns > BC_SAMPLED_MAX_S)
        return bc_fail(ctx, BC_ERR_UNSUPPORTED, "sampled forward: more than BC_SAMPLED_MAX_S distinguished vertices");
    const int32_t k = limit > 0 ? limit : std::max(1, (int32_t)std::ceil(std::sqrt((double)n)));
    if (k > 65534) return bc_fail(ctx, BC_ERR_INVALID_ARG, "sampled forward: limit above 65534");
    const int32_t sp = (ns + 63) / 64 * 64, W = sp / 64;

    // chunks of at most CH arcs: first those of vertices with more arcs (their
    // partial ORs go to P), then one per remaining vertex (even with no arcs,
    // so that every vertex's next-frontier words are written each level)
    std::vector<int32_t> rp((size_t)n + 1);
    hipError_t e = hipMemcpyAsync(rp.data(), ctx->row_ptr, sizeof(int32_t) * rp.size(), hipMemcpyDeviceToHost,
                                  ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return bc_hip(ctx, e, "sampled forward: row offsets");
    std::vector<int2> chunks;
    std::vector<int32_t> sv, sc;
    chunks.reserve((size_t)n + (size_t)(rp[(size_t)n] / CH));
    for (int32_t v = 0; v < n; ++v)
        if (rp[(size_t)v + 1] - rp[(size_t)v] > CH) {
            sv.push_back(v);
            sc.push_back((int32_t)chunks.size());
            for (int32_t a = rp[(size_t)v]; a < rp[(size_t)v + 1]; a += CH) chunks.push_back(make_int2(v, a));
        }
    const int32_t nsplit = (int32_t)chunks.size(), nsv = (int32_t)sv.size();
    sc.push_back(nsplit);
    for (int32_t v = 0; v < n; ++v)
        if (rp[(size_t)v + 1] - rp[(size_t)v] <= CH) chunks.push_back(make_int2(v, rp[(size_t)v]));
    const int32_t nchunks = (int32_t)chunks.size();

    const size_t bits = (size_t)n * W;
    int32_t *dS = (int32_t *)bc_dalloc(ctx, sizeof(int32_t) * (size_t)sp);
    uint16_t *dT = (uint16_t *)bc_dalloc(ctx, sizeof(uint16_t) * (size_t)sp * n);
    int32_t *H = (int32_t *)bc_dalloc(ctx, sizeof(int32_t) * (size_t)sp * sp);
    uint64_t *ring = (uint64_t *)bc_dalloc(ctx, sizeof(uint64_t) * bits * RING);
    uint64_t *visited = (uint64_t *)bc_dalloc(ctx, sizeof(uint64_t) * bits);
    uint64_t *part = (uint64_t *)bc_dalloc(ctx, sizeof(uint64_t) * (size_t)std::max(nsplit, 1) * W);
    int2 *dchunks = (int2 *)bc_dalloc(ctx, sizeof(int2) * (size_t)nchunks);
    int32_t *dsv = (int32_t *)bc_dalloc(ctx, sizeof(int32_t) * (size_t)(2 * nsv + 1));
    uint32_t *found = (uint32_t *)bc_dalloc(ctx, sizeof(uint32_t) * (size_t)(k + 2)); // [k + 1]: the wide flag
    uint32_t *wide = found + (k + 1);
    uint16_t *a16 = (uint16_t *)bc_dalloc(ctx, sizeof(uint16_t) * (size_t)std::max(nreq, 1) * sp);
    // caller-numbered rows: straight into a device output when no source repeats
    const bool direct = out_on_device && in_order;
    int32_t *outc = direct ? out : (int32_t *)bc_dalloc(ctx, sizeof(int32_t) * (size_t)std::max(nreq, 1) * n);
    int32_t *drow = out_on_device && !in_order ? (int32_t *)bc_dalloc(ctx, sizeof(int32_t) * (size_t)count)
                                               : nullptr;
    std::vector<uint32_t> found_h((size_t)k + 1);
    auto cleanup = [&]() {
        for (void *q : {(void *)dS, (void *)dT, (void *)H, (void *)ring, (void *)visited, (void *)part,
                        (void *)dchunks, (void *)dsv, (void *)found, (void *)a16})
            bc_dfree(ctx, q);
        if (!direct) bc_dfree(ctx, outc);
        bc_dfree(ctx, drow);
    };
    if (!dS || !dT || !H || !ring || !visited || !part || !dchunks || !dsv || !found || !a16 || !outc ||
        (out_on_device && !in_order && !drow)) {
        cleanup();
        return bc_fail(ctx, BC_ERR_NOMEM, "sampled forward: allocation failed");
    }
    auto fail_hip = [&](hipError_t err, const char *what) {
        cleanup();
        return bc_hip(ctx, err, what);
    };
    std::vector<int32_t> svsc(sv);
    svsc.insert(svsc.end(), sc.begin(), sc.end());
    e = hipMemcpyAsync(dS, S.data(), sizeof(int32_t) * (size_t)ns, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dchunks, chunks.data(), sizeof(int2) * chunks.size(), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dsv, svsc.data(), sizeof(int32_t) * svsc.size(), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(ring, 0, sizeof(uint64_t) * bits, ctx->stream); // level 0
    if (e == hipSuccess) e = hipMemsetAsync(visited, 0, sizeof(uint64_t) * bits, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(found, 0, sizeof(uint32_t) * (size_t)(k + 2), ctx->stream);
    if (e != hipSuccess) return fail_hip(e, "sampled forward: upload");
    bc_status st = map_ids_to_internal(ctx, dS, ns);
    if (st != BC_OK) {
        cleanup();
        return st;
    }
    hipLaunchKernelGGL(k_ls_sources, dim3(blocks_for((size_t)ns)), dim3(SB), 0, ctx->stream, ns, dS, W, ring,
                       visited);
    // limited searches: every row of S advances one level per launch; level L's new bits
    // go to ring slot L % RING (the next level's frontier), and every RING
    // levels (and at the end) they are written into d'
    {
        LaunchTimer tm(ctx, "limited_bfs");
        const unsigned level_blocks = (unsigned)((nchunks + SB / 64 - 1) / (SB / 64));
        const unsigned finish_blocks = (unsigned)((nsv + SB / 64 - 1) / (SB / 64));
        const unsigned flush_blocks = (unsigned)((bits + FW_WORDS - 1) / FW_WORDS);
        int32_t flushed = 0; // levels below this one are in d'
        for (int32_t L = 1; L <= k; ++L) {
            const uint64_t *f = ring + (size_t)((L - 1) % RING) * bits;
            uint64_t *g = ring + (size_t)(L % RING) * bits;
            hipLaunchKernelGGL(k_ls_level, dim3(level_blocks), dim3(SB), 0, ctx->stream, nchunks, nsplit, dchunks,
                               ctx->row_ptr, ctx->col, W, ns, L, f, g, visited, part, found);
            if (nsv > 0)
                hipLaunchKernelGGL(k_ls_finish, dim3(finish_blocks), dim3(SB), 0, ctx->stream, nsv, dsv,
                                   dsv + nsv, W, ns, L, part, g, visited, found);
            if (L % RING == RING - 1 || L == k) {
                e = hipMemcpyAsync(found_h.data(), found, sizeof(uint32_t) * (size_t)(k + 1), hipMemcpyDeviceToHost,
                                   ctx->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
                if (e != hipSuccess) return fail_hip(e, "sampled forward: level read-back");
                bool news = flushed == 0; // the first flush also writes every unreached entry
                for (int32_t q = flushed; q <= L; ++q) news = news || found_h[(size_t)q] != 0;
                if (news)
                    hipLaunchKernelGGL(k_ls_flush, dim3(flush_blocks), dim3(SB), 0, ctx->stream, n, W, sp,
                                       (const uint64_t *)ring, flushed, L - flushed + 1, flushed == 0 ? 1 : 0,
                                       (const uint32_t *)found, dT);
                flushed = L + 1;
                if (found_h[(size_t)L] == 0) break; // a level found nothing new: the searches are over
            }
        }
        tm.done();
    }
    // the graph on S and its closure
    hipLaunchKernelGGL(k_build_h, dim3(blocks_for((size_t)sp * sp)), dim3(SB), 0, ctx->stream, ns, sp, dS, dT, H);
    {
        LaunchTimer tm(ctx, "floyd_warshall");
        const int32_t nb = sp / TB;
        const unsigned tri = (unsigned)(nb * (nb + 1) / 2);
        // phase 1 of the first round; each later diagonal tile is closed by the
        // previous round's phase 3
        hipLaunchKernelGGL(k_fw_diag, dim3(1), dim3(SB), 0, ctx->stream, sp, 0, H);
        for (int32_t r = 0; r < nb; ++r) {
            int32_t *strip = H + (size_t)r * TB;                  // column strip: rows 0..sp-1, columns of block r
            const int32_t *diag = H + (size_t)r * TB * sp + (size_t)r * TB;
            // phase 2: strip <- min(strip, strip (x) diagonal); the diagonal's own rows do not change
            // (and the row strip, its transpose)
            hipLaunchKernelGGL((k_minplus<4, MP_LOWER, int32_t>), dim3(1, nb), dim3(SB), 0, ctx->stream, sp, TB, TB,
                               (const int32_t *)strip, (int64_t)sp, diag, (int64_t)sp, nullptr, strip, (int64_t)sp,
                               H + (size_t)r * TB * sp, -1, -1, nullptr);
            // phase 3: every entry outside the strips <- min(entry, strip (x) strip), upper
            // tiles mirrored; then the next diagonal tile is closed
            hipLaunchKernelGGL((k_minplus<4, MP_LOWER_SYM, int32_t>), dim3(tri), dim3(SB), 0, ctx->stream, sp, sp, TB,
                               (const int32_t *)strip, (int64_t)sp, (const int32_t *)strip, (int64_t)sp, nullptr,
                               H, (int64_t)sp, nullptr, r, r + 1 < nb ? r + 1 : -1, nullptr);
        }
        tm.done();
    }
    // combination: the sources' rows of D_H (rows 0 .. nreq-1) min-plus d', in 16-bit
    // arithmetic when every finite sum stays below 65535, else in 32-bit; column
    // v of a row is the caller's vertex v (its d' row is that of new_of_old[v])
    if (nreq > 0) {
        LaunchTimer tm(ctx, "sampled_min");
        const dim3 grid((n + 127) / 128, (nreq + 127) / 128);
        hipLaunchKernelGGL(k_dh16, dim3(blocks_for((size_t)nreq * sp)), dim3(SB), 0, ctx->stream, nreq, sp,
                           (const int32_t *)H, 65534 - k, a16, wide);
        hipLaunchKernelGGL(k_minplus16, grid, dim3(SB), 0, ctx->stream, nreq, n, sp, (const uint16_t *)a16,
                           (const uint16_t *)dT, (int64_t)sp, (const int32_t *)ctx->new_of_old, outc, (int64_t)n,
                           (const uint32_t *)wide);
        hipLaunchKernelGGL((k_minplus<8, MP_OUT, uint16_t>), grid, dim3(SB), 0, ctx->stream, nreq, n, sp,
                           (const int32_t *)H, (int64_t)sp, (const uint16_t *)dT, (int64_t)sp,
                           (const int32_t *)ctx->new_of_old, outc, (int64_t)n, nullptr, -1, -1,
                           (const uint32_t *)wide);
        tm.done();
    }
    e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "sampled forward");
    if (nreq > 0) {
        if (out_on_device && !direct) {
            e = hipMemcpyAsync(drow, row_of.data(), sizeof(int32_t) * (size_t)count, hipMemcpyHostToDevice,
                               ctx->stream);
            if (e != hipSuccess) return fail_hip(e, "sampled forward: row upload");
            hipLaunchKernelGGL(k_pick_rows, dim3(blocks_for((size_t)n), std::min(count, 65535)), dim3(SB), 0, ctx->stream, n, count,
                               drow, outc, out);
            e = hipGetLastError();
            if (e != hipSuccess) return fail_hip(e, "sampled forward: row order");
        }
        e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return fail_hip(e, "sampled forward");
        if (!out_on_device) {
            // requested order, repeats included
            std::vector<int32_t> rows((size_t)nreq * n);
            e = hipMemcpy(rows.data(), outc, sizeof(int32_t) * rows.size(), hipMemcpyDeviceToHost);
            if (e != hipSuccess) return fail_hip(e, "sampled forward: copy out");
            for (int32_t i = 0; i < count; ++i)
                std::copy(rows.begin() + (size_t)row_of[i] * n, rows.begin() + (size_t)(row_of[i] + 1) * n,
                          out + (size_t)i * n);
        }
    }
    cleanup();
    return BC_OK;
}
