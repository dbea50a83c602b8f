// Workgroup-level helpers shared by the per-source forms (plain.hip,
// weighted.hip): barriers with device-scope ordering, prefix sums, and the
// LDS-staged, per-arc balanced expansion of a vertex list's adjacency.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wg {

constexpr int PB = 256; // threads per workgroup

// Workgroup barrier with device-scope ordering: per-source arrays are updated
// by device atomics (performed in L2), so every phase change must make them
// visible across the workgroup's waves.
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

// LDS staging for one chunk of up to PB vertices.
struct Chunk {
    int32_t v[PB];
    int32_t rp[PB];
    int32_t off[PB + 1];
    int32_t wsum[PB / 64];
};

// Calls f(k, v, arc) for every arc of the vertices list[lb..le), PB vertices
// at a time, one arc per thread: hubs are spread over the whole workgroup.
// k is the vertex's slot in the chunk (for per-vertex values a caller staged).
// pre(k, v) runs once per staged vertex before its arcs.  Ends with bar().
template <typename Pre, typename F>
__device__ __forceinline__ void for_arcs(const int32_t *list, int32_t lb, int32_t le, const int32_t *__restrict__ rp,
                                         Chunk &c, Pre pre, F f) {
    const int tid = threadIdx.x;
    for (int32_t cb = lb; cb < le; cb += PB) {
        const int32_t i = cb + tid;
        int32_t v = -1, r = 0, d = 0;
        if (i < le) {
            v = list[i];
            r = rp[v];
            d = rp[v + 1] - r;
        }
        int tot;
        const int off = block_excl_scan(d, c.wsum, &tot);
        c.v[tid] = v;
        c.rp[tid] = r;
        c.off[tid] = off;
        if (tid == 0) c.off[PB] = tot;
        if (v >= 0) pre(tid, v);
        __syncthreads();
        for (int e = tid; e < tot; e += PB) {
            const int k = owner(c.off, e);
            f(k, c.v[k], c.rp[k] + (e - c.off[k]));
        }
        bar();
    }
}

// Stages the vertices list[cb .. min(cb + PB, le)) in c (vertex, row offset,
// exclusive degree prefix; c.off[PB] = total) and returns their total degree.
// Every thread of the workgroup calls; ends with __syncthreads().
__device__ __forceinline__ int stage_chunk(const int32_t *list, int32_t cb, int32_t le,
                                           const int32_t *__restrict__ rp, Chunk &c) {
    const int tid = threadIdx.x;
    const int32_t i = cb + tid;
    int32_t v = -1, r = 0, d = 0;
    if (i < le) {
        v = list[i];
        r = rp[v];
        d = rp[v + 1] - r;
    }
    int tot;
    const int off = block_excl_scan(d, c.wsum, &tot);
    c.v[tid] = v;
    c.rp[tid] = r;
    c.off[tid] = off;
    if (tid == 0) c.off[PB] = tot;
    __syncthreads();
    return tot;
}

// Arc positions e0 + j * PB (j < U) of a staged chunk with `tot` arcs: slot
// k[j] of the owning vertex and arc index a[j] (-1 past the end).  The U
// owner searches are independent, so they overlap.
template <int U>
__device__ __forceinline__ void arc_burst(const Chunk &c, int e0, int tot, int (&k)[U], int32_t (&a)[U]) {
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const int e = e0 + j * PB;
        k[j] = 0;
        a[j] = -1;
        if (e < tot) {
            k[j] = owner(c.off, e);
            a[j] = c.rp[k[j]] + (e - c.off[k[j]]);
        }
    }
}

} // namespace wg
