// Small device kernels shared by every form: translating vertex ids between
// the caller's numbering and the internal one, and per-vertex readouts.
#include "bc_internal.h"

namespace {

constexpr int CB = 256;

__global__ __launch_bounds__(CB) void k_map_ids(int32_t *__restrict__ ids, int64_t count,
                                                const int32_t *__restrict__ table) {
    const int64_t i = (int64_t)blockIdx.x * CB + threadIdx.x;
    if (i < count) ids[i] = table[ids[i]];
}

__global__ __launch_bounds__(CB) void k_iota(int32_t *__restrict__ ids, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * CB + threadIdx.x;
    if (i < count) ids[i] = (int32_t)i;
}

// out[r][v] = in[r][table[v]] for rows r < rows, v < n.
template <typename T>
__global__ __launch_bounds__(CB) void k_gather_rows(T *__restrict__ out, const T *__restrict__ in, int64_t rows,
                                                    int32_t n, const int32_t *__restrict__ table) {
    const int64_t i = (int64_t)blockIdx.x * CB + threadIdx.x;
    if (i >= rows * n) return;
    const int64_t r = i / n;
    const int32_t v = (int32_t)(i - r * n);
    out[i] = in[r * n + table[v]];
}

inline unsigned blocks_for(int64_t count) { return (unsigned)((count + CB - 1) / CB); }

} // namespace

__global__ __launch_bounds__(CB) void k_edge_gather(double *__restrict__ out, const double *__restrict__ eb,
                                                    const int32_t *__restrict__ fwd, const int32_t *__restrict__ rev,
                                                    int64_t nnz) {
    const int64_t e = (int64_t)blockIdx.x * CB + threadIdx.x;
    if (e < nnz) out[e] = eb[fwd[e]] + eb[rev[e]];
}

bc_status edges_to_caller_order(bc_ctx *ctx, double *out) {
    if (ctx->nnz <= 0) return BC_OK;
    hipLaunchKernelGGL(k_edge_gather, dim3(blocks_for(ctx->nnz)), dim3(CB), 0, ctx->stream, out, ctx->eb,
                       ctx->arc_fwd, ctx->arc_rev, (int64_t)ctx->nnz);
    BC_HIP(ctx, hipGetLastError());
    return BC_OK;
}

bc_status fill_all_sources(bc_ctx *ctx, int32_t *ids, int64_t count) {
    if (count <= 0) return BC_OK;
    hipLaunchKernelGGL(k_iota, dim3(blocks_for(count)), dim3(CB), 0, ctx->stream, ids, count);
    BC_HIP(ctx, hipGetLastError());
    return BC_OK;
}

bc_status map_ids_to_internal(bc_ctx *ctx, int32_t *ids, int64_t count) {
    if (count <= 0 || !ctx->new_of_old) return BC_OK;
    hipLaunchKernelGGL(k_map_ids, dim3(blocks_for(count)), dim3(CB), 0, ctx->stream, ids, count, ctx->new_of_old);
    BC_HIP(ctx, hipGetLastError());
    return BC_OK;
}

template <typename T>
static bc_status gather_rows(bc_ctx *ctx, T *out, const T *in, int64_t rows) {
    const int64_t cells = rows * ctx->n;
    if (cells <= 0) return BC_OK;
    if (!ctx->new_of_old) {
        BC_HIP(ctx, hipMemcpyAsync(out, in, sizeof(T) * (size_t)cells, hipMemcpyDeviceToDevice, ctx->stream));
        return BC_OK;
    }
    hipLaunchKernelGGL(k_gather_rows<T>, dim3(blocks_for(cells)), dim3(CB), 0, ctx->stream, out, in, rows, ctx->n,
                       ctx->new_of_old);
    BC_HIP(ctx, hipGetLastError());
    return BC_OK;
}

bc_status rows_to_caller_order_f64(bc_ctx *ctx, double *out, const double *in, int64_t rows) {
    return gather_rows(ctx, out, in, rows);
}
bc_status rows_to_caller_order_i32(bc_ctx *ctx, int32_t *out, const int32_t *in, int64_t rows) {
    return gather_rows(ctx, out, in, rows);
}
bc_status rows_to_caller_order_u64(bc_ctx *ctx, uint64_t *out, const uint64_t *in, int64_t rows) {
    return gather_rows(ctx, out, in, rows);
}
