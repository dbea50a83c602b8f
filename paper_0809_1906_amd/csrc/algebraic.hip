// Algebraic form (Sec. 3.1): a batch of B sources is a frontier matrix and each
// level is a product with the 0/1 adjacency matrix A on MFMA (int8 forward,
// BF16 backward).
//
// Forward (Compute Path Count, first-hit reading): with F_l[v][b] = lambda(s_b, v)
// where d(s_b, v) = l and 0 elsewhere,
//     F_{l+1} = Mask_unvisited(A . F_l),
// i.e. for every w not yet reached from s_b, lambda(s_b, w) = sum over
// neighbours v at level l of lambda(s_b, v).  Counts are carried exactly:
// F_l is split into 7-bit limbs F^(k) (non-negative int8), every product
// A . F^(k) is an int8 MFMA with int32 accumulation -- exact; each output is an
// integer of at most 127 * deg(w) < 2^24 (deg <= 65792 is checked at create),
// so its FP32 copy for the epilogue is exact too -- and the limbs are
// recombined as sum_k 2^(7k) P^(k) in 64-bit integers, with a carry out of 64
// bits reported as an overflowing count.  The number of limbs comes
// from the largest count of level l, which the kernel that wrote level l
// recorded on the device, so no host round trip precedes the products.
//
// Backward (Compute Dependency): with C_{l+1}[w][b] = (1 + delta(w,b)) /
// lambda(s_b, w) for w at level l+1 (the "(D_l + Delta_l) div Lambda" matrix of
// the paper, one level deeper), Delta_l = Mask_l(A . C_{l+1}) mult Lambda.
// C is FP32; it is split exactly into three BF16 planes hi + mid + lo
// (3 x 8 significand bits cover FP32's 24) and the three products are summed
// in the same FP32 accumulators, which gives FP32-GEMM accuracy against a 0/1
// matrix.  The dependencies are added into BC in the epilogue (column sums of
// Delta without the diagonal: level 0 is never accumulated).
//
// Integer weights 1..M (Sec. 3.2): levels are distances, A_c is the 0/1
// matrix of the edges of weight c, and
//     F_L = Mask_unvisited(sum_{c=1..M} A_c . F_{L-c}),
// a vertex's first non-empty level being its distance (every weight is at
// least 1, so levels L-M .. L-1 are complete when level L is formed).  The
// backward takes, for v at level L, delta(v) = lambda(v) * sum_c (A_c .
// C_{L+c})[v]: the w with d(w) = d(v) + c over an edge of weight c are exactly
// v's successors in the shortest-path DAG.  Both sums are one product with
// the class matrices side by side, [A_1 | ... | A_M] (rows = vertices, K =
// M * npad), against the stacked planes [X_1; ...; X_M] of the levels involved;
// unit weights are M = 1.  The exactness bound is unchanged: an output sums at
// most deg(w) non-zero terms of at most 127.
//
// Data layout: A is a bit matrix in panels of 128 columns, [M * npad / 128]
// [npad][4] words (npad = n rounded up to 256, a multiple of the block's row
// count): a row's 16 B of one panel lie beside the next row's, so the bits of
// 32 consecutive rows for one pipeline stage share four cache lines.  Word i
// of a row's panel holds the panel's columns 32i .. 32i + 31, column 32i + 2p
// at bit p and 32i + 2p + 1 at bit 16 + p (p < 16): masked with 0x10001 << p
// and multiplied by 0x3F80 >> p, a word gives the BF16 pair (0 or 1, 0 or 1)
// of columns 2p, 2p + 1 in one 24-bit multiply.  Each wave loads the bits of
// its own rows into registers and expands them into MFMA A operands there:
// the adjacency costs 1/16 of a BF16 matrix's bytes and no LDS traffic, and
// LDS holds only the planes, which the block's waves share.  The forward's
// int8 operands take a second copy of the bits in another order: column
// 32i + 16h + 4d + j (h < 2, d < 4, j < 4) at bit 8j + 2d + h of word i, so
// a shift by 2d + h and a mask with 0x01010101 give the four bytes (0 or 1)
// of columns 16h + 4d .. +3, one dword of an int8 A operand.  Planes are
// k-packed in 16-byte cells, plane[v / 8][b][v % 8] in BF16 and
// plane[v / 16][b][v % 16] in int8, so each MFMA B-operand lane reads one
// cell.  Every product is
// C[w][b] = sum_v A[w][v] X[v][b] with rows = vertices and columns = sources;
// in the 32x32 MFMA output the 32 lanes of each half-wave hold 32 consecutive
// sources of one vertex, so two ballots give a 64-bit frontier word.
// The frontier bitmaps, visited words, counts and c values are the batched
// sparse form's state (sparse.hip): levels can switch between the two forms.
#include "bc_internal.h"

#include <algorithm>

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

constexpr int GN = 128;  // columns (sources) per block (two bitmap words)
constexpr int GK = 32;   // k (vertices) per k-tile of the skip flags
constexpr int WM = 64;   // rows per wave: 2 MFMA row tiles of 32
constexpr int RT = WM / 32;
constexpr int PB = 256;  // threads per block of the element-wise kernels
constexpr int NPAD = 256; // n is padded to a multiple of this (of every block's rows too)

enum { EPI_ONLY = 0, EPI_FIRST = 1, EPI_MID = 2, EPI_LAST = 3 };

struct GemmArgs {
    const uint32_t *abits; // [K / 128][npad][4] adjacency bit words (layout above)
    const uint32_t *abits8;// the same bits in the int8 operand order (forward)
    const __bf16 *planes;  // planes of 16-byte cells: [K/8][B][8] BF16 or [K/16][B][16] int8
    const uint32_t *kflags;// [K/GK][B/GN]: some plane entry of this k-tile is non-zero
    int32_t npad, n, B, NW;
    int32_t K;             // M * npad: the class matrices side by side
    size_t plane_elems;    // K * B
    int32_t ksplit;        // forward: 1, or 2 blocks per tile, each over half of K
    int32_t ntiles;        // grid_blocks<BM>(npad, B): tiles of one product
    float *ws;             // split tiles' partial sums, [8][ntiles][2][64][forward block threads]
    uint32_t *arrive;      // [8][ntiles]
    unsigned long long *ktiles; // [0] k-tiles multiplied, [1] k-tiles in the blocks' ranges (per direction)
    const uint32_t *gate;  // backward of a replayed batch: flag of level l, whose vertices it
                           // writes; zero = every block exits
};

struct EpiArgs {
    uint64_t *part;        // [npad][B] partial limb sums
    const uint64_t *fcur;  // backward: front[l]
    uint64_t *fnext;       // forward: front[l+1]
    uint64_t *visited;
    void *sigma;           // uint32_t or uint64_t [n][B]
    float *cval;           // [n][B]
    const int32_t *src_lane;
    double *bc, *delta_dump;
    uint32_t *any_next, *status;
    const unsigned long long *lvmax_cur; // forward: largest count of level l (then l-1, ...)
    unsigned long long *lvmax_next;      // forward: largest count of level l+1
    int32_t classes, level;              // forward: M, and l (levels l+1-M .. l feed level l+1)
    unsigned long long *planes_issued;   // products issued (limb or coefficient planes)
    unsigned long long *reach;           // forward, every level by products: [0] pairs the batch's
                                         // sources can reach, [1] pairs reached, [2] set when the
                                         // two were equal before this level's products
    int accumulate;
};

// Every (vertex, source) pair the batch can reach has been reached: the next
// level is empty, and the products that would find that out are skipped.
// Read only while no kernel adds to reach[1] (the planes kernel before a
// level's products, which records the answer in reach[2] for them: the
// products' own epilogues add to reach[1] while later blocks start).
__device__ __forceinline__ bool search_over(const unsigned long long *reach) {
    return reach && __hip_atomic_load(&reach[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                        __hip_atomic_load(&reach[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_count(uint64_t *p, uint64_t x, bool &) { *p = x; }
__device__ __forceinline__ void store_count(uint32_t *p, uint64_t x, bool &wide) {
    wide |= x > 0xFFFFFFFFull;
    *p = (uint32_t)x;
}

// 7-bit limbs needed for a count (at least one; ten cover 64 bits).
constexpr int LIMB_BITS = 7;
__device__ __forceinline__ int limbs_of(uint64_t mx) {
    int L = 1;
    while (L < 10 && (mx >> (LIMB_BITS * L)) != 0) ++L;
    return L;
}

// Limbs for the product forming level l+1: the largest count of the levels
// l+1-M .. l that feed it (levels below 0 do not exist).
__device__ __forceinline__ int limbs_feeding(const unsigned long long *lvmax_l, int32_t l, int32_t M) {
    unsigned long long mx = 0;
    for (int32_t c = 0; c < M && c <= l; ++c) mx = max(mx, lvmax_l[-c]);
    return limbs_of(mx);
}

// ---- the product -------------------------------------------------------------------

// Block shapes: BM rows by GN sources in 2 BM threads, waves of 64 x 64 in
// BM / 64 rows by 2 columns (BM = 128: 4 waves, BM = 256: 8 waves).

// Plane tile of one stage in LDS: [NP][KS / KC][GN] cells of 16 B (KC = 8
// BF16 or 16 int8 k per cell, one MFMA B-operand lane each; 32 consecutive
// sources of one k-group contiguous), counted in BF16 units.
template <int NP, int KS, int KC = 8>
constexpr int lds_x() { return NP * (KS / KC) * GN * 8; }
// Two LDS buffers (one barrier per stage, the next stage stored while the
// current one is multiplied) when they fit: 2 x 32 KB for 128-row blocks (two
// per compute unit), 2 x 48 KB for 256-row blocks (one per unit); else one.
template <int NP, int KS, int BM, int KC = 8>
constexpr int stages() { return lds_x<NP, KS, KC>() * 2 * 2 <= (BM == 256 ? 196608 : 65536) ? 2 : 1; }
// Stage depths (k per stage): forward one int8 plane 256 deep (32 KB),
// backward three BF16 planes 64 deep (48 KB, one buffer).  Measured on
// ER-16384 (B = 512): backward 32-deep stages with two buffers, and 256-row
// backward blocks with two 48 KB buffers, were both slower (by 8% and 3%).
constexpr int FWD_KS = 256;
constexpr int FWD_KC = 16;
constexpr int BWD_KS = 64;
// Forward block rows: 128 or 256, whichever the tuner measured faster on the
// graph (AlgebraicState::fwd_rows); the backward takes 128.
constexpr int BWD_BM = 128;

// A stage's plane tile held in registers between its global loads and its LDS
// stores: the block's T threads cover T / GN k-groups of GN sources at a time,
// 16 B per thread and k-group.
template <int NP, int KS_, int T_, int KC = 8>
struct Stage {
    static constexpr int KS = KS_, XG = T_ / GN, XJ = KS / KC / XG;
    static_assert(XJ >= 1, "stage shape");
    u32x4 x[NP * XJ];
};

// A wave's adjacency bits of one stage: for each 32-row MFMA tile rt, the
// words of row (lane % 32) of that tile that the wave multiplies: the stage's
// KS / 32, or with the stage's k range split between the two waves of a row
// pair (KH), the KS / 64 of the wave's half.
template <int KS, bool KH>
struct ABits {
    static constexpr int W = KH ? KS / 64 : KS / 32;
    static_assert(W == 2 || W == 4, "stage depth");
    uint32_t w[RT][W];
};

template <int NP, int KS, int TT, int KC>
__device__ __forceinline__ void load_stage(const GemmArgs &g, const __bf16 *planes, int ks, int b0, int tid,
                                           Stage<NP, KS, TT, KC> &st) {
    using T = Stage<NP, KS, TT, KC>;
    const int c = tid & (GN - 1), i0 = tid / GN; // k-groups i0, i0 + XG, ..., column c
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int j = 0; j < T::XJ; ++j)
            st.x[p * T::XJ + j] = *reinterpret_cast<const u32x4 *>(
                planes + (size_t)p * g.plane_elems + (((size_t)ks * (KS / KC) + i0 + T::XG * j) * g.B + b0 + c) * 8);
}

// rows0: the wave's first row.  The wave's columns of stage ks start at k0 =
// ks KS (+ KS / 2 for the second half with KH), word (k0 % 128) / 32 of panel
// k0 / 128: 16 B or 8 B, aligned.  I8: the bits in the int8 operand order.
template <int KS, bool KH, bool I8 = false>
__device__ __forceinline__ void load_abits(const GemmArgs &g, int ks, int rows0, int lane, int half,
                                           ABits<KS, KH> &ab) {
    constexpr int W = ABits<KS, KH>::W;
    const int k0 = ks * KS + (KH ? half * (KS / 2) : 0);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const uint32_t *p = (I8 ? g.abits8 : g.abits) +
                            ((size_t)(k0 / 128) * g.npad + rows0 + rt * 32 + (lane & 31)) * 4 + (k0 % 128) / 32;
        if constexpr (W == 4) {
            const u32x4 v = *reinterpret_cast<const u32x4 *>(p);
            ab.w[rt][0] = v[0];
            ab.w[rt][1] = v[1];
            ab.w[rt][2] = v[2];
            ab.w[rt][3] = v[3];
        } else {
            const uint2 v = *reinterpret_cast<const uint2 *>(p);
            ab.w[rt][0] = v.x;
            ab.w[rt][1] = v.y;
        }
    }
}

template <int NP, int KS, int TT, int KC>
__device__ __forceinline__ void store_stage(__bf16 *sX, int tid, const Stage<NP, KS, TT, KC> &st) {
    using T = Stage<NP, KS, TT, KC>;
    const int c = tid & (GN - 1), i0 = tid / GN;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int j = 0; j < T::XJ; ++j)
            *reinterpret_cast<u32x4 *>(sX + (((size_t)p * (KS / KC) + i0 + T::XG * j) * GN + c) * 8) =
                st.x[p * T::XJ + j];
}

// MFMA A operand (32 x 16 BF16, lane l: row l % 32, columns 8 (l / 32) .. +7)
// from a word of bits: columns 16 h + 8 (l / 32) + j, j < 8, of the word's
// half h are its pairs 8 h + 4 (l / 32) + j / 2, which the shift brings to
// pairs 0 .. 3 (bits 0 .. 3 and 16 .. 19).
__device__ __forceinline__ bf16x8 expand_bits(uint32_t w, int shift) {
    const uint32_t y = w >> shift;
    u32x4 o;
    o[0] = __umul24(y & 0x10001u, 0x3F80u);
    o[1] = __umul24(y & 0x20002u, 0x1FC0u);
    o[2] = __umul24(y & 0x40004u, 0xFE0u);
    o[3] = __umul24(y & 0x80008u, 0x7F0u);
    return __builtin_bit_cast(bf16x8, o);
}

// int8 MFMA A operand (32 x 32, lane l: row l % 32, columns 16 (l / 32) ..
// +15, one byte each) from a word in the int8 order: dword d holds columns
// 16 h + 4d .. +3 (h = l / 32), at bits 8j + 2d + h of the word.
__device__ __forceinline__ i32x4 expand_i8(uint32_t w, int h) {
    i32x4 o;
#pragma unroll
    for (int d = 0; d < 4; ++d) o[d] = (int)((w >> (2 * d + h)) & 0x01010101u);
    return o;
}

// The wave's rows (RT tiles of 32) by its CT column tiles of 32 sources
// starting at source wn of the block: A from the wave's bits, X from LDS.
// Without KH the wave multiplies the stage's KS / 16 k-steps for 64 sources
// (CT = 2); with KH, its half of them (from k-step half KS / 32) for all 128
// sources (CT = 4).
template <int NP, int KS, bool KH, bool I8 = false>
__device__ __forceinline__ void mma_stage(const __bf16 *sX, const ABits<KS, KH> &ab, int lane, int wn, int half,
                                          f32x16 (&acc)[RT][KH ? 4 : 2]) {
    // k-steps of 16 (BF16) or 32 (int8) k: two cell rows of 16 B each
    constexpr int KC = I8 ? 16 : 8, KSTEP = 2 * KC;
    constexpr int CT = KH ? 4 : 2, STEPS = KH ? KS / KSTEP / 2 : KS / KSTEP;
    static_assert(!I8 || NP == 1, "int8 products take one plane");
    const int hs = (lane >> 5) * 4;
    const __bf16 *x = sX + (((size_t)(KH ? half * STEPS * 2 : 0) + (lane >> 5)) * GN + wn + (lane & 31)) * 8;
    // B operands of k-step kh + 1 are read while step kh multiplies
    u32x4 b[2][NP][CT];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
            b[0][p][ct] = *reinterpret_cast<const u32x4 *>(x + ((size_t)p * (KS / KC) * GN + ct * 32) * 8);
#pragma unroll
    for (int kh = 0; kh < STEPS; ++kh) {
        const int cur = kh & 1;
        if (kh + 1 < STEPS) {
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int ct = 0; ct < CT; ++ct)
                    b[cur ^ 1][p][ct] = *reinterpret_cast<const u32x4 *>(
                        x + (((size_t)p * (KS / KC) + (kh + 1) * 2) * GN + ct * 32) * 8);
        }
        __builtin_amdgcn_sched_barrier(0); // the reads stay ahead of this step's products
        if constexpr (I8) {
            // int32 sums kept in the FP32-typed accumulators' bits
            i32x4 a[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) a[rt] = expand_i8(ab.w[rt][kh], lane >> 5);
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
                    acc[rt][ct] = __builtin_bit_cast(
                        f32x16, __builtin_amdgcn_mfma_i32_32x32x32_i8(a[rt], __builtin_bit_cast(i32x4, b[cur][0][ct]),
                                                                      __builtin_bit_cast(i32x16, acc[rt][ct]), 0, 0,
                                                                      0));
        } else {
            bf16x8 a[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) a[rt] = expand_bits(ab.w[rt][kh >> 1], hs + 8 * (kh & 1));
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            a[rt], __builtin_bit_cast(bf16x8, b[cur][p][ct]), acc[rt][ct], 0, 0, 0);
        }
    }
}

// Block -> (row block, column block), XCD-aware.  Consecutive blocks go to
// consecutive XCDs (each with its own L2), so block L runs on XCD L % 8; the
// blocks of one XCD take (row block, column block) pairs with the column
// fastest, so all column blocks of a row block run on the same XCD at about
// the same time and share its adjacency rows in that L2.  Row blocks past the
// matrix (padding to a multiple of 8) return at once.
struct Tile {
    int row, col;
};
__device__ __forceinline__ Tile tile_of(int B) {
    const int C = B / GN;
    const int L = blockIdx.x, x = L & 7, t = L >> 3;
    // uniform over the block: keep it in scalar registers
    return Tile{__builtin_amdgcn_readfirstlane((t / C) * 8 + x), __builtin_amdgcn_readfirstlane(t % C)};
}
template <int BM>
inline unsigned grid_blocks(int npad, int B) { return (unsigned)(((npad / BM + 7) / 8) * 8 * (B / GN)); }

// With K split in two: blocks L and L + 8 (the same XCD) take the two halves
// of one tile; otherwise as tile_of.  *tile is the tile's index in
// [0, grid_blocks).
__device__ __forceinline__ Tile tile_of_split(int B, int &half, int &tile) {
    const int C = B / GN;
    const int L = blockIdx.x, x = L & 7, t = L >> 3, tt = t >> 1;
    half = __builtin_amdgcn_readfirstlane(t & 1);
    const int row = (tt / C) * 8 + x, col = tt % C;
    tile = __builtin_amdgcn_readfirstlane(row * C + col);
    return Tile{__builtin_amdgcn_readfirstlane(row), __builtin_amdgcn_readfirstlane(col)};
}

// Stages with a non-zero flag among their TPS k-tiles, 64 at a time: lane i
// of each wave reads the flags of stage base + i, and the ballot is the
// wave's window (one round trip per 64 stages, not one per stage).
template <int TPS>
__device__ __forceinline__ uint64_t stage_window(const uint32_t *flags, int ntn, int base, int nks, int lane) {
    const int st = base + lane;
    uint32_t f = 0;
    if (st < nks) {
#pragma unroll
        for (int t = 0; t < TPS; ++t) f |= flags[((size_t)st * TPS + t) * ntn];
    }
    return __ballot(f != 0);
}

// The next stage from ks on (of nks) with a non-zero flag; [base, base + 64)
// is the window in `bits`, refilled once ks passes it.
template <int TPS>
__device__ __forceinline__ int next_stage(const uint32_t *flags, int ntn, int ks, int nks, int lane, int &base,
                                          uint64_t &bits) {
    while (ks < nks) {
        if (ks >= base + 64) {
            base = ks;
            bits = stage_window<TPS>(flags, ntn, base, nks, lane);
        }
        const uint64_t m = bits >> (ks - base);
        if (m) return ks + __builtin_ctzll(m);
        ks = base + 64;
    }
    return nks;
}

// acc[w][b] = sum over stages with a non-zero k-tile flag of A[w][k] X_p[k][b],
// summed over the NP planes starting at `planes`, for the block's BM rows
// (from w0) and GN sources (from b0); wave wv holds rows w0 + WM (wv / WC) +
// [0, WM) and sources b0 + WN (wv % WC) + [0, WN).  The next stage's planes
// and bits are loaded (into registers) during the current stage's products.
// kt0 and kt1 are k-tiles, multiples of the stage's k-tiles.  I8: int8
// planes and products (exact int32 sums, returned converted to FP32).
template <int NP, int KS, int BM, bool KH = false, bool I8 = false>
__device__ __forceinline__ void gemm_tile(const GemmArgs &g, const __bf16 *planes, int w0, int b0, int tid,
                                          __bf16 (*sX)[lds_x<NP, KS, I8 ? 16 : 8>()], f32x16 (&acc)[RT][KH ? 4 : 2],
                                          int kt0 = 0, int kt1 = -1) {
    constexpr int KC = I8 ? 16 : 8;
    constexpr int TPS = KS / GK; // k-tiles per stage
    const int lane = tid & 63, wv = tid >> 6, half = wv & 1;
    const int rows0 = w0 + (wv >> 1) * WM, wn = KH ? 0 : half * 64;
    const int nks = (kt1 < 0 ? g.K / GK : kt1) / TPS, ks0 = kt0 / TPS, ntn = g.B / GN;
    const uint32_t *flags = g.kflags + b0 / GN;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int c = 0; c < (KH ? 4 : 2); ++c)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[rt][c][r] = 0.f;

    int wbase = ks0 - 64; // empty window
    uint64_t wbits = 0;
    int ks = next_stage<TPS>(flags, ntn, ks0, nks, lane, wbase, wbits);
    int kn = ks < nks ? next_stage<TPS>(flags, ntn, ks + 1, nks, lane, wbase, wbits) : nks;
    int buf = 0, done = 0;
    Stage<NP, KS, 2 * BM, KC> st;
    ABits<KS, KH> ab, abn;
    if (ks < nks) {
        // bits first: the planes' stores then wait for them too
        load_abits<KS, KH, I8>(g, ks, rows0, lane, half, ab);
        load_stage(g, planes, ks, b0, tid, st);
        store_stage(sX[0], tid, st);
    }
    __syncthreads();
    while (ks < nks) {
        // After the last stage the loads repeat the current one (in bounds,
        // never multiplied): unconditional loads keep the waits for them
        // after this stage's products.
        const int kl = kn < nks ? kn : ks;
        load_stage(g, planes, kl, b0, tid, st);
        load_abits<KS, KH, I8>(g, kl, rows0, lane, half, abn);
        __builtin_amdgcn_sched_barrier(0); // issued before the products, not sunk below them
        mma_stage<NP, KS, KH, I8>(sX[buf], ab, lane, wn, half, acc);
        if constexpr (stages<NP, KS, BM, KC>() == 2) {
            if (kn < nks) store_stage(sX[buf ^ 1], tid, st);
            __syncthreads();
            buf ^= 1;
        } else {
            __syncthreads(); // every wave is done with the stage
            if (kn < nks) store_stage(sX[0], tid, st);
            __syncthreads();
        }
        ab = abn;
        ks = kn;
        kn = kn < nks ? next_stage<TPS>(flags, ntn, kn + 1, nks, lane, wbase, wbits) : nks;
        ++done;
    }
    if (tid == 0 && g.ktiles) {
        // in units of one plane's 32 x 128 x 128 (k, rows, sources): 2^20 flops
        constexpr unsigned long long U = (unsigned long long)NP * (BM / 128);
        atomicAdd(&g.ktiles[0], (unsigned long long)done * TPS * U);
        atomicAdd(&g.ktiles[1], (unsigned long long)(nks - ks0) * TPS * U);
    }
    if constexpr (I8) {
        // whole vectors: a bit cast of one vector element reads element 0
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int c = 0; c < (KH ? 4 : 2); ++c)
                acc[rt][c] = __builtin_convertvector(__builtin_bit_cast(i32x16, acc[rt][c]), f32x16);
    }
}

// The two halves of a split tile meet here after their products for limb k.
// Each stores its partial sums (agent-scope stores, coherent across XCDs) to
// its own slot for limb k; the second to arrive adds the other's and returns
// true, the first returns false.  One slot per limb: a half never waits, so
// it may be several limbs ahead of the other.
template <int T>
__device__ __forceinline__ bool split_meet(const GemmArgs &g, int k, int tile, int half, int tid, int &s_last,
                                           f32x16 (&acc)[RT][2]) {
    constexpr int V = RT * 2 * 16; // sums per thread
    float *slot = g.ws + (((size_t)k * g.ntiles + tile) * 2) * V * T;
#pragma unroll
    for (int i = 0; i < RT * 2; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r)
            __hip_atomic_store(&slot[((size_t)half * V + i * 16 + r) * T + tid], acc[i / 2][i % 2][r],
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __asm__ __volatile__("s_waitcnt vmcnt(0)" ::: "memory"); // this thread's stores are done
    __syncthreads();
    if (tid == 0) {
        uint32_t *cnt = &g.arrive[(size_t)k * g.ntiles + tile];
        s_last = atomicAdd(cnt, 1u) == 1u;
        if (s_last) __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (!s_last) return false;
#pragma unroll
    for (int i = 0; i < RT * 2; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r)
            acc[i / 2][i % 2][r] += __hip_atomic_load(&slot[((size_t)(1 - half) * V + i * 16 + r) * T + tid],
                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// Forward epilogue for limb `shift / 7`; `mode` (uniform over the launch) says
// whether it is the only limb, the first, a middle one or the last.  Lane
// layout of the 32x32 output: lane l, register r holds row 8(r/4) + 4(l/32) +
// r%4 and column l%32; the two column tiles are bitmap word q.
template <typename S>
__device__ __forceinline__ void epi_fwd(const GemmArgs &g, const EpiArgs &e, int mode, int shift,
                                        const f32x16 (&acc)[RT][2], int w0, int q, int lane) {
    const int half = lane >> 5, col = lane & 31;
    const bool first = mode == EPI_FIRST, mid = mode == EPI_MID, last = mode == EPI_LAST;
    const bool final_limb = mode == EPI_ONLY || last;
    S *sigma = reinterpret_cast<S *>(e.sigma);
    bool wide = false, ovf = false;
    uint64_t mx = 0, any_rows = 0;
    uint32_t fresh_pairs = 0;
    // The wave owns word q of its 64 rows: lane l loads row w0 + l's visited
    // word once, and each row's lanes take it by a shuffle (no global round
    // trip per row; the loop's stores to visited would otherwise keep the
    // compiler from issuing these loads ahead of them).
    const uint64_t vis_lane =
        (!first && w0 + lane < g.n) ? e.visited[(size_t)(w0 + lane) * g.NW + q] : ~0ull;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int lr = rt * 32 + 8 * (r >> 2) + 4 * half + (r & 3); // row in the wave
            const int w = w0 + lr;
            const bool valid = w < g.n;
            const uint64_t vis = __shfl(vis_lane, lr, 64);
            uint64_t m[2];
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) {
                const int bit = ct * 32 + col;
                const uint64_t P = (uint64_t)acc[rt][ct][r]; // exact integer < 2^24
                const size_t idx = (size_t)w * g.B + (size_t)q * 64 + bit;
                // A limb sum that carries out of 64 bits is a count above
                // 2^64 - 1 when w is unvisited (a level-(l+1) vertex);
                // visited vertices' sums are discarded.
                const bool open = valid && !((vis >> bit) & 1);
                bool fresh = false;
                // part is carried from limb to limb, possibly by the two
                // blocks of a split tile: agent-scope accesses keep it coherent
                unsigned long long *pp = reinterpret_cast<unsigned long long *>(&e.part[idx]);
                if (first) {
                    if (valid) __hip_atomic_store(pp, (unsigned long long)P, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    const uint64_t add = P << shift;
                    uint64_t tot = add;
                    if (valid && (mid || last)) tot += __hip_atomic_load(pp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (open && shift > 0 && ((P >> (64 - shift)) != 0 || tot < add)) ovf = true;
                    if (mid) {
                        if (valid)
                            __hip_atomic_store(pp, (unsigned long long)tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    } else {
                        fresh = open && tot != 0;
                        if (fresh) {
                            store_count(&sigma[idx], tot, wide);
                            mx = tot > mx ? tot : mx;
                        }
                    }
                }
                m[ct] = __ballot(fresh);
            }
            if (final_limb) {
                // lanes 0..31 hold vertex w of half 0, lanes 32..63 vertex w + 4
                const uint64_t word = half == 0 ? ((m[0] & 0xFFFFFFFFull) | (m[1] << 32))
                                                : ((m[0] >> 32) | (m[1] & 0xFFFFFFFF00000000ull));
                if (col == 0 && valid) {
                    e.fnext[(size_t)w * g.NW + q] = word;
                    if (word) {
                        e.visited[(size_t)w * g.NW + q] = vis | word;
                        any_rows |= 1ull << lr;
                        fresh_pairs += (uint32_t)__popcll(word);
                    }
                }
            }
        }
    }
    if (final_limb) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t o = __shfl_xor(mx, off, 64);
            mx = o > mx ? o : mx;
        }
        if (lane == 0 && mx > __hip_atomic_load(e.lvmax_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(e.lvmax_next, (unsigned long long)mx);
        if (__any(wide) && lane == 0) atomicOr(&e.status[1], 1u);
        // rows with new pairs, two words of the level's vertex filter per wave
        // (w0 is a multiple of 64)
        any_rows |= __shfl_xor(any_rows, 32, 64);
        if (lane == 0 && any_rows) {
            if ((uint32_t)any_rows) atomicOr(&e.any_next[w0 >> 5], (uint32_t)any_rows);
            if (any_rows >> 32) atomicOr(&e.any_next[(w0 >> 5) + 1], (uint32_t)(any_rows >> 32));
        }
        if (e.reach) { // lanes 0 and 32 hold the counts
            fresh_pairs += __shfl_xor(fresh_pairs, 32, 64);
            if (lane == 0 && fresh_pairs) atomicAdd(&e.reach[1], (unsigned long long)fresh_pairs);
        }
    }
    if (__any(ovf) && lane == 0) atomicOr(&e.status[0], (uint32_t)BC_DEV_SIGMA_OVERFLOW);
}

// Forward level l -> l+1: one pass per 7-bit limb of level l's largest count,
// each an int8 product followed by its epilogue.  Grid: grid_blocks<BM>(npad,
// B), tiles by tile_of.  KS: k per pipeline stage.  The two waves of a row pair split each stage's
// k range (each expands only its half of the adjacency bits, for all 128
// sources) and sum the halves through LDS before the epilogue: half the bit
// expansion of waves that each take 64 sources (ER-16384: 247 -> 233 us per
// launch with 128-row blocks).
template <typename S, int KS, int BM>
__global__ __launch_bounds__(2 * BM, BM == 128 ? 2 : 1) void k_mfma_fwd(GemmArgs g, EpiArgs e) {
    constexpr bool KH = true; // the waves' k-split (the backward keeps the column split)
    constexpr int KC = FWD_KC;
    // one LDS area: the plane buffers during the products, then the halves'
    // exchange (64 sums per lane per wave)
    constexpr size_t PLANE_BYTES = (size_t)stages<1, KS, BM, KC>() * lds_x<1, KS, KC>() * sizeof(__bf16);
    constexpr size_t XCHG_BYTES = KH ? (size_t)2 * BM / 64 * 64 * RT * 2 * 16 * sizeof(float) : 0;
    __shared__ __align__(16) unsigned char smem[PLANE_BYTES > XCHG_BYTES ? PLANE_BYTES : XCHG_BYTES];
    auto sX = reinterpret_cast<__bf16 (*)[lds_x<1, KS, KC>()]>(smem);
    __shared__ int s_last;
    int half = 0, tile = 0;
    const Tile tl = g.ksplit == 2 ? tile_of_split(g.B, half, tile) : tile_of(g.B);
    if (tl.row >= g.npad / BM || (e.reach && e.reach[2] != 0)) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int w0 = tl.row * BM + (wv >> 1) * WM, b0 = tl.col * GN;
    const int q = (b0 >> 6) + (wv & 1); // bitmap word of this wave's sources
    const int L = limbs_feeding(e.lvmax_cur, e.level, e.classes);
    if (blockIdx.x == 0 && tid == 0) atomicAdd(e.planes_issued, (unsigned long long)L);
    // split K at a stage boundary (K is a multiple of 256, the stages' depth)
    constexpr int TPS = KS / GK;
    const int nst = g.K / KS, hst = nst / 2;
    const int kt0 = g.ksplit == 2 && half ? hst * TPS : 0, kt1 = g.ksplit == 2 && !half ? hst * TPS : nst * TPS;
    f32x16 acc[RT][2];
#pragma nounroll
    for (int k = 0; k < L; ++k) {
        // int8 plane k: plane_elems bytes from the planes' start
        const __bf16 *planes_k = g.planes + (size_t)k * (g.plane_elems / 2);
        if constexpr (KH) {
            f32x16 acc4[RT][4];
            gemm_tile<1, KS, BM, true, true>(g, planes_k, tl.row * BM, b0, tid, sX, acc4, kt0, kt1);
            // wave wv keeps sources 64 h .. 64 h + 63 (h = wv & 1, its bitmap
            // word) and hands the other 64 to its partner wv ^ 1; the tile
            // loop ended at a barrier, so the plane buffers are free
            // (h is uniform over the wave: constant tile indices in each
            // branch keep acc4 in registers)
            float *xb = reinterpret_cast<float *>(smem);
            float *mine = xb + (size_t)wv * RT * 2 * 16 * 64 + lane;
            const float *theirs = xb + (size_t)(wv ^ 1) * RT * 2 * 16 * 64 + lane;
            if (wv & 1) {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int c = 0; c < 2; ++c)
#pragma unroll
                        for (int r = 0; r < 16; ++r) mine[((rt * 2 + c) * 16 + r) * 64] = acc4[rt][c][r];
            } else {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int c = 0; c < 2; ++c)
#pragma unroll
                        for (int r = 0; r < 16; ++r) mine[((rt * 2 + c) * 16 + r) * 64] = acc4[rt][2 + c][r];
            }
            __syncthreads();
            if (wv & 1) {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int c = 0; c < 2; ++c)
#pragma unroll
                        for (int r = 0; r < 16; ++r)
                            acc[rt][c][r] = acc4[rt][2 + c][r] + theirs[((rt * 2 + c) * 16 + r) * 64];
            } else {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int c = 0; c < 2; ++c)
#pragma unroll
                        for (int r = 0; r < 16; ++r)
                            acc[rt][c][r] = acc4[rt][c][r] + theirs[((rt * 2 + c) * 16 + r) * 64];
            }
        } else {
            gemm_tile<1, KS, BM, false, true>(g, planes_k, tl.row * BM, b0, tid, sX, acc, kt0, kt1);
        }
        if (g.ksplit == 2 && !split_meet<2 * BM>(g, k, tile, half, tid, s_last, acc))
            continue; // the other half finishes it
        const int mode = L == 1 ? EPI_ONLY : k == 0 ? EPI_FIRST : k + 1 < L ? EPI_MID : EPI_LAST;
        // The epilogue's row addresses do not depend on k; an opaque copy of
        // the block's first row keeps the compiler from computing all of them
        // once before the loop and holding them through the products.
        int w0k = w0;
        __asm__ volatile("" : "+s"(w0k));
        epi_fwd<S>(g, e, mode, LIMB_BITS * k, acc, w0k, q, lane);
        __syncthreads(); // the next limb's pipeline reuses the LDS buffers
    }
}

// Backward level l: acc = A . (hi + mid + lo planes of C_{l+1}), then
// delta(v,b) = lambda(v,b) * acc for v at level l, c(v,b) = (1 + delta) / lambda,
// and BC(v) += delta summed over the block's sources (v != s_b).
template <typename S>
__global__ __launch_bounds__(2 * BWD_BM, BWD_BM == 128 ? 2 : 1) void k_mfma_bwd(GemmArgs g, EpiArgs e) {
    __shared__ __align__(16) __bf16 sX[stages<3, BWD_KS, BWD_BM>()][lds_x<3, BWD_KS>()];
    // one block per tile: its stages of three planes are long enough already
    // (split in two halves of K it measured slower)
    if (g.gate && *g.gate == 0) return; // level l is empty (or the batch was handed back)
    const Tile tl = tile_of(g.B);
    if (tl.row >= g.npad / BWD_BM) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int b0 = tl.col * GN;
    f32x16 acc[RT][2];
    if (g.gate && g.gate[1] == 0) {
        // the deepest level of a replayed batch: no successor, so delta = 0
        // and c = 1 / lambda, without products (their flag scan alone would
        // cost a dependent load per stage)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[rt][ct][r] = 0.f;
    } else {
        if (blockIdx.x == 0 && tid == 0) atomicAdd(e.planes_issued, 3ull);
        gemm_tile<3, BWD_KS, BWD_BM>(g, g.planes, tl.row * BWD_BM, b0, tid, sX, acc);
    }

    const int w0 = tl.row * BWD_BM + (wv >> 1) * WM;
    const int q = (b0 >> 6) + (wv & 1);
    const int half = lane >> 5, col = lane & 31;
    S *sigma = reinterpret_cast<S *>(e.sigma);
    // level-l words of the wave's 64 rows, one load per lane (as in the forward)
    const uint64_t f_lane = w0 + lane < g.n ? e.fcur[(size_t)(w0 + lane) * g.NW + q] : 0;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int lr = rt * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
            const int v = w0 + lr;
            const uint64_t F = __shfl(f_lane, lr, 64);
            double contrib = 0.0;
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) {
                const int bit = ct * 32 + col;
                if ((F >> bit) & 1) {
                    const size_t idx = (size_t)v * g.B + (size_t)q * 64 + bit;
                    const double sv = (double)sigma[idx];
                    const double dl = sv * (double)acc[rt][ct][r];
                    e.cval[idx] = (float)((1.0 + dl) / sv);
                    if (e.delta_dump) e.delta_dump[(size_t)(q * 64 + bit) * g.n + v] = dl; // [b][v], as bc_read_sssp
                    if (e.src_lane[q * 64 + bit] != v) contrib += dl;
                }
            }
            if (e.accumulate) {
#pragma unroll
                for (int off = 16; off > 0; off >>= 1) contrib += __shfl_xor(contrib, off, 64);
                if (col == 0 && contrib != 0.0) unsafeAtomicAdd(&e.bc[v], contrib);
            }
        }
    }
}

// ---- element-wise kernels -------------------------------------------------------

// A[v][(c-1) npad + w] = 1 for every arc v -> w of weight c (c = 1 without
// weights), as bits of the panel layout, word (k % 128) / 32 of row v in
// panel k / 128 for column k: in abits at bit (k % 2) 16 + (k % 32) / 2 (the
// BF16 pair order), in abits8 at bit 8 (k % 4) + 2 ((k % 16) / 4) + (k % 32)
// / 16 (the int8 order).
__global__ __launch_bounds__(PB) void k_build_adj(int32_t n, int32_t npad, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col, const uint8_t *__restrict__ wt,
                                                  uint32_t *__restrict__ abits, uint32_t *__restrict__ abits8) {
    const int32_t v = blockIdx.x;
    if (v >= n) return;
    for (int32_t e = rp[v] + threadIdx.x; e < rp[v + 1]; e += PB) {
        const int32_t c = wt ? (int32_t)wt[e] - 1 : 0;
        const size_t k = (size_t)c * npad + col[e];
        const uint32_t j = (uint32_t)(k & 31);
        const size_t word = ((k / 128) * npad + v) * 4 + (k % 128) / 32;
        atomicOr(&abits[word], 1u << ((j & 1) * 16 + (j >> 1)));
        atomicOr(&abits8[word], 1u << (8 * (j & 3) + 2 * ((j >> 2) & 3) + (j >> 4)));
    }
}

// Planes feeding level l+1: int8 planes[k][c][v/16][b][v%16] = 7-bit limb k
// of lambda(s_b, v) for v at level l-c (class c+1, weight c+1), else 0, for
// the limbs of the largest count among the feeding levels (plane k starts
// k plane_elems bytes in); kflags[(c npad + v) / GK][b / GN] = (some limb
// non-zero).  Block (c, t, sb) covers k-tile t of class c (GK = 32 rows) for
// source block sb (GN sources) and writes its flag; thread (h, j) takes the
// 16 rows from 32 t + 16 h for source GN sb + j.  Levels are `words` words
// apart, and levels below 0 contribute nothing.
template <typename S>
__global__ __launch_bounds__(PB) void k_limb_split(int32_t n, int32_t npad, int32_t B, int32_t NW, int32_t M,
                                                   int32_t l, const unsigned long long *__restrict__ lvmax_l,
                                                   const uint64_t *__restrict__ fl, size_t words,
                                                   const S *__restrict__ sigma, __bf16 *__restrict__ planes,
                                                   size_t plane_elems, uint32_t *__restrict__ kflags,
                                                   unsigned long long *__restrict__ reach) {
    static_assert(PB == 2 * GN && GK == 32, "one block per k-tile and source block");
    const bool over = search_over(reach);
    if (reach && blockIdx.x == 0 && threadIdx.x == 0) reach[2] = over ? 1ull : 0ull; // for this level's products
    if (over) return; // the whole grid: the level's products are skipped and read no flag
    const int32_t nsb = B / GN, tiles = npad / GK;
    const int32_t c = (int32_t)(blockIdx.x / ((size_t)tiles * nsb));
    const int32_t rem = (int32_t)(blockIdx.x - (size_t)c * tiles * nsb), t = rem / nsb, sb = rem - t * nsb;
    const int32_t vg = t * 2 + (int32_t)(threadIdx.x / GN), b = sb * GN + (int32_t)(threadIdx.x % GN);
    const size_t id = ((size_t)c * (npad / 16) + vg) * B + b; // the thread's 16-byte cell
    const int L = limbs_feeding(lvmax_l, l, M);
    const uint64_t *f = c <= l ? fl - (size_t)c * words : nullptr;
    uint64_t s[16];
    bool nz = false;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int32_t v = vg * 16 + j;
        s[j] = 0;
        if (f && v < n && ((f[(size_t)v * NW + (b >> 6)] >> (b & 63)) & 1)) s[j] = (uint64_t)sigma[(size_t)v * B + b];
        nz |= s[j] != 0;
    }
    unsigned char *pb = reinterpret_cast<unsigned char *>(planes);
    for (int k = 0; k < L; ++k) {
        u32x4 o;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            uint32_t x = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) x |= (uint32_t)((s[4 * d + j] >> (LIMB_BITS * k)) & 0x7F) << (8 * j);
            o[d] = x;
        }
        *reinterpret_cast<u32x4 *>(pb + (size_t)k * plane_elems + id * 16) = o;
    }
    const int any = __syncthreads_or(nz);
    if (threadIdx.x == 0) kflags[((size_t)c * tiles + t) * nsb + sb] = any ? 1u : 0u;
}

// Planes for backward level l: planes[0..2][c][v/8][b][v%8] = hi, mid, lo BF16
// parts of c(v, b) for v at level l+1+c (class c+1), for the `deeper` levels
// below l that exist (the others contribute nothing), and kflags[(c npad +
// v) / GK][b / GN] = (some part non-zero).  Blocks as in k_limb_split; a
// thread's 16 rows are two 8-row cells.
__global__ __launch_bounds__(PB) void k_coef_split(int32_t n, int32_t npad, int32_t B, int32_t NW, int32_t M,
                                                   int32_t deeper, const uint64_t *__restrict__ fl, size_t words,
                                                   const float *__restrict__ cval, __bf16 *__restrict__ planes,
                                                   size_t plane_elems, uint32_t *__restrict__ kflags,
                                                   const uint32_t *__restrict__ gate) {
    static_assert(PB == 2 * GN && GK == 32, "one block per k-tile and source block");
    // gate[0]: level l (empty: the product exits too); gate[1]: level l+1
    // (empty: the product multiplies nothing and reads no plane or flag)
    if (gate && (gate[0] == 0 || gate[1] == 0)) return;
    const int32_t nsb = B / GN, tiles = npad / GK;
    const int32_t cl = (int32_t)(blockIdx.x / ((size_t)tiles * nsb));
    const int32_t rem = (int32_t)(blockIdx.x - (size_t)cl * tiles * nsb), t = rem / nsb, sb = rem - t * nsb;
    const int32_t b = sb * GN + (int32_t)(threadIdx.x % GN);
    const uint64_t *f = cl < deeper ? fl + (size_t)cl * words : nullptr;
    bool nz = false;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int32_t vg = t * 4 + (int32_t)(threadIdx.x / GN) * 2 + h; // 8-row cell
        const size_t id = ((size_t)cl * (npad / 8) + vg) * B + b;
        bf16x8 hi, mid, lo;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int32_t v = vg * 8 + j;
            float c = 0.f;
            if (f && v < n && ((f[(size_t)v * NW + (b >> 6)] >> (b & 63)) & 1)) c = cval[(size_t)v * B + b];
            const __bf16 hb = (__bf16)c;
            const float r1 = c - (float)hb;
            const __bf16 m = (__bf16)r1;
            const float r2 = r1 - (float)m;
            hi[j] = hb;
            mid[j] = m;
            lo[j] = (__bf16)r2;
            nz |= c != 0.f;
        }
        *reinterpret_cast<bf16x8 *>(planes + id * 8) = hi;
        *reinterpret_cast<bf16x8 *>(planes + plane_elems + id * 8) = mid;
        *reinterpret_cast<bf16x8 *>(planes + 2 * plane_elems + id * 8) = lo;
    }
    const int any = __syncthreads_or(nz);
    if (threadIdx.x == 0) kflags[((size_t)cl * tiles + t) * nsb + sb] = any ? 1u : 0u;
}

// One block of the plane kernels per k-flag word: (class, k-tile, source block).
inline size_t kflag_words(bc_ctx *ctx) {
    return (size_t)ctx->al.classes * (ctx->al.npad / GK) * (ctx->sp.batch / GN);
}

GemmArgs gemm_args(bc_ctx *ctx, const __bf16 *planes, bool forward) {
    AlgebraicState &a = ctx->al;
    GemmArgs g;
    g.abits = a.abits;
    g.abits8 = a.abits8;
    g.planes = planes;
    g.kflags = a.kflags;
    g.npad = a.npad;
    g.n = ctx->n;
    g.B = ctx->sp.batch;
    g.NW = ctx->sp.words;
    g.K = a.classes * a.npad;
    g.plane_elems = (size_t)g.K * ctx->sp.batch;
    g.ksplit = a.ksplit;
    g.ntiles = (int32_t)(!forward           ? grid_blocks<BWD_BM>(a.npad, ctx->sp.batch)
                         : a.fwd_rows == 256 ? grid_blocks<256>(a.npad, ctx->sp.batch)
                                             : grid_blocks<128>(a.npad, ctx->sp.batch));
    g.ws = a.ws;
    g.gate = nullptr;
    g.arrive = a.arrive;
    // counters: [0] planes, [1..2] forward k-tiles, [3..4] backward k-tiles
    g.ktiles = a.planes_issued ? a.planes_issued + (forward ? 1 : 3) : nullptr;
    return g;
}

} // namespace

bc_status algebraic_prepare(bc_ctx *ctx) {
    AlgebraicState &a = ctx->al;
    const int32_t B = ctx->sp.batch;
    if (ctx->weighted && ctx->max_weight > BC_ALGEBRAIC_MAX_WEIGHT)
        return bc_fail(ctx, BC_ERR_UNSUPPORTED, "algebraic form: weights above 8 (one product class per weight)");
    if (B % GN != 0) return bc_fail(ctx, BC_ERR_UNSUPPORTED, "algebraic form: batch must be 256 or 512");
    if (ctx->max_degree > BC_ALGEBRAIC_MAX_DEGREE)
        return bc_fail(ctx, BC_ERR_UNSUPPORTED,
                       "algebraic form: degrees above 65792 are not taken (exact FP32 copies of the products' sums)");
    a.npad = std::max(NPAD, (ctx->n + NPAD - 1) / NPAD * NPAD);
    a.classes = ctx->weighted ? (int32_t)ctx->max_weight : 1;
    const size_t K = (size_t)a.classes * a.npad;
    const size_t adj_bytes = (size_t)a.npad * K / 8;
    const size_t plane_elems = K * B;
    if (2 * adj_bytes + 8 * plane_elems * sizeof(__bf16) > (size_t(96) << 30))
        return bc_fail(ctx, BC_ERR_UNSUPPORTED, "algebraic form: the adjacency bits and planes would exceed 96 GiB");
    a.abits = (uint32_t *)bc_dalloc(ctx, adj_bytes);
    a.abits8 = (uint32_t *)bc_dalloc(ctx, adj_bytes);
    // up to ten int8 limb planes (10 plane_elems bytes), or 3 BF16 coefficient planes
    a.planes = (__bf16 *)bc_dalloc(ctx, 8 * plane_elems * sizeof(__bf16));
    a.part = (uint64_t *)bc_dalloc(ctx, (size_t)a.npad * B * sizeof(uint64_t));
    a.kflags = (uint32_t *)bc_dalloc(ctx, (K / GK) * (B / GN) * sizeof(uint32_t));
    a.planes_issued = (unsigned long long *)bc_dalloc(ctx, 256);
    // Unweighted forward products over a long K (one npad per limb) with
    // fewer tiles than the compute units hold blocks at once (256 units, LDS
    // for 256 / BM blocks each): two blocks per output tile, each over half
    // of K, so that the grid fills the chip.  With a full chip of tiles the
    // split measured slower (ER-16384, B = 512: 124 against 116 ms per step),
    // and with weight classes too (K is M npad; 0.43 of BF16 against 0.50).
    // The decision is the same for 128- and 256-row blocks (tiles halve as
    // the blocks per unit do); the workspace takes the larger of the two
    // (grids are rounded up to whole rounds of the eight XCDs).
    a.fwd_rows = 128;
    const size_t ntiles = grid_blocks<128>(a.npad, B), ntiles256 = grid_blocks<256>(a.npad, B);
    const size_t ws_elems = std::max(ntiles * 2 * (RT * 2 * 16) * (2 * 128), ntiles256 * 2 * (RT * 2 * 16) * (2 * 256));
    const size_t ntiles_max = std::max(ntiles, ntiles256);
    a.ksplit = a.classes == 1 && K / GK >= 256 && ntiles < (size_t)256 * (256 / 128) ? 2 : 1;
    if (a.ksplit == 2) {
        a.ws = (float *)bc_dalloc(ctx, (size_t)8 * ws_elems * sizeof(float));
        a.arrive = (uint32_t *)bc_dalloc(ctx, (size_t)8 * ntiles_max * sizeof(uint32_t));
    }
    if (!a.abits || !a.abits8 || !a.planes || !a.part || !a.kflags || !a.planes_issued ||
        (a.ksplit == 2 && (!a.ws || !a.arrive)))
        return bc_fail(ctx, BC_ERR_NOMEM, "algebraic form: allocation failed");
    if (a.ksplit == 2) BC_HIP(ctx, hipMemsetAsync(a.arrive, 0, (size_t)8 * ntiles_max * sizeof(uint32_t), ctx->stream));
    BC_HIP(ctx, hipMemsetAsync(a.abits, 0, adj_bytes, ctx->stream));
    BC_HIP(ctx, hipMemsetAsync(a.abits8, 0, adj_bytes, ctx->stream));
    BC_HIP(ctx, hipMemsetAsync(a.planes_issued, 0, 5 * sizeof(unsigned long long), ctx->stream));
    if (ctx->n > 0)
        hipLaunchKernelGGL(k_build_adj, dim3(ctx->n), dim3(PB), 0, ctx->stream, ctx->n, a.npad,
                           ctx->row_ptr, ctx->col, ctx->weighted ? (const uint8_t *)ctx->weight : nullptr, a.abits,
                           a.abits8);
    BC_HIP(ctx, hipGetLastError());
    return BC_OK;
}

bc_status algebraic_release(bc_ctx *ctx) {
    AlgebraicState &a = ctx->al;
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (void *p : {(void *)a.abits, (void *)a.abits8, (void *)a.planes, (void *)a.part, (void *)a.kflags, (void *)a.planes_issued,
                    (void *)a.ws, (void *)a.arrive})
        if (p) bc_dfree(ctx, p);
    const bool every = a.every_level;
    a = AlgebraicState{};
    a.every_level = every;
    return BC_OK;
}

// Forward level l -> l+1 as products with A.  Writes front[l+1], visited,
// counts, any[l+1] and the largest count of level l+1 exactly as the pull
// kernel does; reads the largest count of level l on the device.
template <typename S>
bc_status algebraic_forward_level_t(bc_ctx *ctx, int32_t l) {
    AlgebraicState &a = ctx->al;
    SparseState &s = ctx->sp;
    const size_t words = (size_t)ctx->n * s.words;
    const size_t aw = (size_t)(ctx->n + 31) / 32;
    const uint64_t *fcur = s.front + (size_t)l * words;
    const size_t plane_elems = (size_t)a.classes * a.npad * s.batch;
    // With every level by products the reached pairs are counted (the first
    // level by the push, the rest by the epilogue), so a level after the last
    // one skips its planes and products.
    unsigned long long *reach = a.every_level ? s.reach : nullptr;
    {
        // writes every k-flag word (no clearing pass)
        LaunchTimer tm(ctx, "limb_split");
        hipLaunchKernelGGL(k_limb_split<S>, dim3((unsigned)kflag_words(ctx)), dim3(PB), 0, ctx->stream, ctx->n,
                           a.npad, s.batch, s.words, a.classes, l, s.lvmax + l, fcur, words, (const S *)s.sigma,
                           a.planes, plane_elems, a.kflags, reach);
        tm.done();
    }
    EpiArgs e{};
    e.reach = reach;
    e.part = a.part;
    e.fnext = s.front + (size_t)(l + 1) * words;
    e.visited = s.visited;
    e.sigma = s.sigma;
    e.any_next = s.any + (size_t)(l + 1) * aw;
    e.status = ctx->status;
    e.lvmax_cur = s.lvmax + l;
    e.lvmax_next = s.lvmax + l + 1;
    e.classes = a.classes;
    e.level = l;
    e.planes_issued = a.planes_issued;
    const GemmArgs g = gemm_args(ctx, a.planes, true);
    LaunchTimer tm(ctx, "mfma_fwd");
    if (a.fwd_rows == 256)
        hipLaunchKernelGGL((k_mfma_fwd<S, FWD_KS, 256>), dim3(grid_blocks<256>(a.npad, s.batch) * a.ksplit),
                           dim3(2 * 256), 0, ctx->stream, g, e);
    else
        hipLaunchKernelGGL((k_mfma_fwd<S, FWD_KS, 128>), dim3(grid_blocks<128>(a.npad, s.batch) * a.ksplit),
                           dim3(2 * 128), 0, ctx->stream, g, e);
    tm.done();
    BC_HIP(ctx, hipGetLastError());
    return BC_OK;
}

// Backward level l as a product with A: acc = sum_c A_c . C_{l+c}, masked to
// level l; `deeper` of the levels l+1 .. l+M exist (front[l+1] at fnext, the
// next ones `words` apart).
template <typename S>
bc_status algebraic_backward_level_t(bc_ctx *ctx, const uint64_t *fcur, const uint64_t *fnext, int32_t deeper,
                                     double *delta_dump, bool accumulate, const uint32_t *gate) {
    AlgebraicState &a = ctx->al;
    SparseState &s = ctx->sp;
    const size_t words = (size_t)ctx->n * s.words;
    const size_t plane_elems = (size_t)a.classes * a.npad * s.batch;
    {
        // writes every k-flag word (no clearing pass)
        LaunchTimer tm(ctx, "coef_split");
        hipLaunchKernelGGL(k_coef_split, dim3((unsigned)kflag_words(ctx)), dim3(PB), 0, ctx->stream, ctx->n,
                           a.npad, s.batch, s.words, a.classes, fnext ? deeper : 0, fnext, words, s.cval, a.planes,
                           plane_elems, a.kflags, gate);
        tm.done();
    }
    EpiArgs e{};
    e.fcur = fcur;
    e.sigma = s.sigma;
    e.cval = s.cval;
    e.src_lane = s.src;
    e.bc = ctx->bc;
    e.delta_dump = delta_dump;
    e.accumulate = accumulate ? 1 : 0;
    e.planes_issued = a.planes_issued;
    GemmArgs g = gemm_args(ctx, a.planes, false);
    g.gate = gate;
    LaunchTimer tm(ctx, "mfma_bwd");
    hipLaunchKernelGGL(k_mfma_bwd<S>, dim3(grid_blocks<BWD_BM>(a.npad, s.batch)), dim3(2 * BWD_BM), 0, ctx->stream,
                       g, e);
    tm.done();
    BC_HIP(ctx, hipGetLastError());
    return BC_OK;
}

bc_status algebraic_forward_level(bc_ctx *ctx, bool wide, int32_t l) {
    return wide ? algebraic_forward_level_t<uint64_t>(ctx, l) : algebraic_forward_level_t<uint32_t>(ctx, l);
}

bc_status algebraic_backward_level(bc_ctx *ctx, bool wide, const uint64_t *fcur, const uint64_t *fnext,
                                   int32_t deeper, double *delta_dump, bool accumulate, const uint32_t *gate) {
    return wide ? algebraic_backward_level_t<uint64_t>(ctx, fcur, fnext, deeper, delta_dump, accumulate, gate)
                : algebraic_backward_level_t<uint32_t>(ctx, fcur, fnext, deeper, delta_dump, accumulate, gate);
}

int64_t algebraic_planes_issued(bc_ctx *ctx) {
    AlgebraicState &a = ctx->al;
    if (!a.planes_issued) return 0;
    unsigned long long v = 0;
    if (hipMemcpyAsync(&v, a.planes_issued, sizeof v, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        return -1;
    return (int64_t)v;
}

bool algebraic_ktiles(bc_ctx *ctx, int64_t *run, int64_t *dense, int64_t *run_fwd, int64_t *dense_fwd) {
    AlgebraicState &a = ctx->al;
    *run = *dense = *run_fwd = *dense_fwd = 0;
    if (!a.planes_issued) return true;
    unsigned long long v[4] = {0, 0, 0, 0};
    if (hipMemcpyAsync(v, a.planes_issued + 1, sizeof v, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        return false;
    *run_fwd = (int64_t)v[0];
    *dense_fwd = (int64_t)v[1];
    *run = (int64_t)(v[0] + v[2]);
    *dense = (int64_t)(v[1] + v[3]);
    return true;
}

void algebraic_reset_counters(bc_ctx *ctx) {
    if (ctx->al.planes_issued)
        (void)hipMemsetAsync(ctx->al.planes_issued, 0, 5 * sizeof(unsigned long long), ctx->stream);
}
