// bc_read_sssp_noalloc: the per-source readout of bc_read_sssp for callers
// that cannot allocate device memory.  Its staging lives in one fixed device
// array per GPU (`scratch`), whose address on each device is looked up once,
// when the first context is created there, and kept.
#include "bc_internal.h"

#include <map>
#include <mutex>

namespace {

// Fixed staging of bc_read_sssp_noalloc, held on every GPU the library runs
// on until the process ends.  Host code never passes the array's name to a
// kernel or a copy: only the per-device address noalloc_scratch returns.
__device__ __align__(256) unsigned char scratch[BC_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
std::map<int, unsigned char *> g_addr;  // device -> address of `scratch` on it
std::map<int, hipError_t> g_fail;       // device -> why the lookup failed

constexpr size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

} // namespace

void noalloc_init_device(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_addr.count(device) || g_fail.count(device)) return;
    unsigned char *p = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess && p) g_addr[device] = p;
    else g_fail[device] = e == hipSuccess ? hipErrorInvalidSymbol : e;
}

unsigned char *noalloc_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_addr.find(device);
    return it == g_addr.end() ? nullptr : it->second;
}

// Sets ctx->no_alloc for the duration of a call: bc_dalloc then returns NULL,
// so any path that would allocate fails with BC_ERR_NOMEM instead.
struct NoAllocScope {
    bc_ctx *ctx;
    explicit NoAllocScope(bc_ctx *c) : ctx(c) { ctx->no_alloc = true; }
    ~NoAllocScope() { ctx->no_alloc = false; }
};

extern "C" bc_status bc_read_sssp_noalloc(bc_ctx *ctx, const int32_t *sources, int32_t count, int32_t *dist,
                                          uint64_t *sigma, double *delta) {
    if (!ctx) return BC_ERR_INVALID_ARG;
    NoAllocScope scope(ctx);
    bc_status s = bc_check_usable(ctx);
    if (s != BC_OK) return s;
    const int32_t maxc = ctx->many ? 64 : ctx->form == BC_FORM_PLAIN_FP64 ? 4096 : ctx->sp.batch;
    if (!sources || count < 1 || count > maxc) return bc_fail(ctx, BC_ERR_INVALID_ARG, "count must be in [1, batch]");
    for (int32_t i = 0; i < count; ++i)
        if (sources[i] < 0 || sources[i] >= ctx->n) return bc_fail(ctx, BC_ERR_INVALID_ARG, "source id out of range");
    // staging: internal source ids, many-graph units, then the internal-order
    // rows of distances, counts and dependencies
    const size_t cells = (size_t)count * (size_t)std::max(ctx->n, 1);
    const size_t o_units = up256((size_t)count * sizeof(int32_t));
    const size_t o_dd = o_units + (ctx->many ? up256((size_t)count * 3 * sizeof(int32_t)) : 0);
    const size_t o_ds = o_dd + up256(cells * sizeof(int32_t));
    const size_t o_dl = o_ds + up256(cells * sizeof(uint64_t));
    const size_t need = o_dl + up256(cells * sizeof(double));
    if (need > BC_NOALLOC_SCRATCH_BYTES)
        return bc_fail(ctx, BC_ERR_UNSUPPORTED,
                       "bc_read_sssp_noalloc: count * n too large for BC_NOALLOC_SCRATCH_BYTES of staging");
    unsigned char *base = noalloc_scratch(ctx->device);
    if (!base) return bc_fail(ctx, BC_ERR_DEVICE, "bc_read_sssp_noalloc: the staging array has no address on this device");
    int32_t *dsrc = reinterpret_cast<int32_t *>(base);
    int32_t *units = reinterpret_cast<int32_t *>(base + o_units);
    int32_t *dd = reinterpret_cast<int32_t *>(base + o_dd);
    uint64_t *ds = reinterpret_cast<uint64_t *>(base + o_ds);
    double *dl = reinterpret_cast<double *>(base + o_dl);
    BC_HIP(ctx, hipMemcpyAsync(dsrc, sources, (size_t)count * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream)); // the caller's host array may go away
    if ((s = map_ids_to_internal(ctx, dsrc, count)) != BC_OK) return s;
    uint32_t before = 0, now = 0;
    if ((s = bc_status_save(ctx, &before)) != BC_OK) return s;
    bc_status run;
    if (ctx->many) run = multigraph_dump(ctx, sources, count, dd, ds, dl, units);
    else if (ctx->form == BC_FORM_PLAIN_FP64) run = plain_run(ctx, dsrc, count, false, dl, dd, ds);
    else run = sparse_dump(ctx, dsrc, count, dd, ds, dl);
    if (run != BC_ERR_DEVICE) s = bc_status_restore(ctx, before, &now);
    if (run != BC_OK) return run;
    if (s != BC_OK) return s;
    if (now & BC_DEV_SIGMA_OVERFLOW) return bc_fail(ctx, BC_ERR_OVERFLOW, "a shortest-path count exceeded 2^64 - 1");
    if (ctx->n > 0) {
        if ((dist && (s = rows_to_caller_order_i32(ctx, dist, dd, count)) != BC_OK) ||
            (sigma && (s = rows_to_caller_order_u64(ctx, sigma, ds, count)) != BC_OK) ||
            (delta && (s = rows_to_caller_order_f64(ctx, delta, dl, count)) != BC_OK))
            return s;
    }
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return BC_OK;
}
