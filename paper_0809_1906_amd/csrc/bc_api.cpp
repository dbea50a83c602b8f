// The C ABI of include/bc.h: host-side validation, device memory, streams,
// and dispatch to the forms.  Every device step runs in the HIP kernels of
// plain.hip and sparse.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "bc_internal.h"

namespace {

thread_local std::string g_create_error;

bc_status fail_create(bc_status s, const std::string &msg) {
    g_create_error = msg;
    return s;
}

// Host validation of the graph model (Sec. 1.1, undirected simple graph with
// positive integer weights) on host copies of the arrays.
bc_status validate_graph(int32_t n, int32_t nnz, const int32_t *rp, const int32_t *col,
                         const uint32_t *w, std::string &msg, int32_t &max_deg, uint32_t &max_w) {
    char buf[256];
    if (rp[0] != 0) { msg = "row_ptr[0] must be 0"; return BC_ERR_INVALID_GRAPH; }
    if (rp[n] != nnz) {
        snprintf(buf, sizeof buf, "row_ptr[n] = %d but nnz = %d", rp[n], nnz);
        msg = buf;
        return BC_ERR_INVALID_GRAPH;
    }
    max_deg = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (rp[v + 1] < rp[v]) {
            snprintf(buf, sizeof buf, "row_ptr decreases at vertex %d", v);
            msg = buf;
            return BC_ERR_INVALID_GRAPH;
        }
        max_deg = std::max(max_deg, rp[v + 1] - rp[v]);
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
            int32_t x = col[e];
            if (x < 0 || x >= n) {
                snprintf(buf, sizeof buf, "arc %d of vertex %d points to %d, outside [0,%d)", e, v, x, n);
                msg = buf;
                return BC_ERR_INVALID_GRAPH;
            }
            if (x == v) {
                snprintf(buf, sizeof buf, "self-loop at vertex %d", v);
                msg = buf;
                return BC_ERR_INVALID_GRAPH;
            }
            if (e > rp[v] && col[e - 1] >= x) {
                snprintf(buf, sizeof buf, "row %d is not strictly increasing (duplicate or unsorted arc)", v);
                msg = buf;
                return BC_ERR_INVALID_GRAPH;
            }
        }
    }
    max_w = 1;
    if (w) {
        for (int32_t e = 0; e < nnz; ++e) {
            if (w[e] == 0) { msg = "edge weight 0 (weights must be >= 1)"; return BC_ERR_INVALID_GRAPH; }
            max_w = std::max(max_w, w[e]);
        }
        if ((int64_t)max_w * (int64_t)(n > 0 ? n - 1 : 0) >= (int64_t(1) << 31)) {
            msg = "max weight * (n-1) must stay below 2^31";
            return BC_ERR_INVALID_GRAPH;
        }
    }
    // symmetry: (v,x) present => (x,v) present with the same weight
    for (int32_t v = 0; v < n; ++v) {
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
            int32_t x = col[e];
            const int32_t *b = col + rp[x], *en = col + rp[x + 1];
            const int32_t *it = std::lower_bound(b, en, v);
            if (it == en || *it != v) {
                snprintf(buf, sizeof buf, "arc (%d,%d) has no reverse arc (graph must be undirected)", v, x);
                msg = buf;
                return BC_ERR_INVALID_GRAPH;
            }
            if (w && w[it - col] != w[e]) {
                snprintf(buf, sizeof buf, "arcs (%d,%d) and (%d,%d) carry different weights", v, x, x, v);
                msg = buf;
                return BC_ERR_INVALID_GRAPH;
            }
        }
    }
    return BC_OK;
}

void release_all(bc_ctx *ctx) {
    if (!ctx) return;
    if (ctx->device >= 0) hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->stream);
    if (ctx->mg.stream) hipStreamSynchronize(ctx->mg.stream);
    if (ctx->mg.exec) hipGraphExecDestroy(ctx->mg.exec);
    if (ctx->mg.ev) hipEventDestroy(ctx->mg.ev);
    if (ctx->mg.stream) hipStreamDestroy(ctx->mg.stream);
    ctx->mg.exec = nullptr;
    ctx->mg.ev = nullptr;
    ctx->mg.stream = nullptr;
    sparse_graphs_release(ctx);
    bc_timers_clear(ctx);
    for (hipEvent_t e : ctx->event_pool) hipEventDestroy(e);
    ctx->event_pool.clear();
    auto owned = ctx->owned;
    for (auto &pr : owned) bc_dfree(ctx, pr.first);
    ctx->owned.clear();
    if (ctx->status_host) hipHostFree(ctx->status_host);
    if (ctx->sp.any_host) hipHostFree(ctx->sp.any_host);
    if (ctx->wt.host) hipHostFree(ctx->wt.host);
    ctx->wt.host = nullptr;
    ctx->status_host = nullptr;
    ctx->sp.any_host = nullptr;
}

} // namespace

// ---------------------------------------------------------------------------
// helpers shared with the forms
// ---------------------------------------------------------------------------

bc_status bc_fail(bc_ctx *ctx, bc_status s, const std::string &msg) {
    if (ctx) ctx->err = msg;
    else g_create_error = msg;
    return s;
}

bc_status bc_hip(bc_ctx *ctx, hipError_t e, const char *what) {
    std::string msg = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return bc_fail(ctx, BC_ERR_NOMEM, msg);
    if (ctx) ctx->poisoned = true;
    return bc_fail(ctx, BC_ERR_DEVICE, msg);
}

void *bc_dalloc(bc_ctx *ctx, size_t bytes) {
    if (ctx->no_alloc) return nullptr; // bc_read_sssp_noalloc: BC_ERR_NOMEM, never an allocation
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~size_t(255);
    void *p = nullptr;
    if (ctx->alloc.alloc) {
        p = ctx->alloc.alloc(bytes, (void *)ctx->stream, ctx->alloc.user);
    } else {
        if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    }
    if (p) {
        ctx->owned.emplace_back(p, bytes);
        ctx->device_bytes += (int64_t)bytes;
    }
    return p;
}

void bc_dfree(bc_ctx *ctx, void *p) {
    if (!p) return;
    for (size_t i = 0; i < ctx->owned.size(); ++i) {
        if (ctx->owned[i].first == p) {
            ctx->device_bytes -= (int64_t)ctx->owned[i].second;
            ctx->owned.erase(ctx->owned.begin() + (long)i);
            break;
        }
    }
    if (ctx->alloc.free) ctx->alloc.free(p, (void *)ctx->stream, ctx->alloc.user);
    else hipFree(p);
}

hipEvent_t bc_event_get(bc_ctx *ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

void bc_event_put(bc_ctx *ctx, hipEvent_t e) {
    if (e) ctx->event_pool.push_back(e);
}

void bc_timers_clear(bc_ctx *ctx) {
    for (auto &kv : ctx->timers)
        for (auto &pr : kv.second.pending) {
            bc_event_put(ctx, pr.first);
            bc_event_put(ctx, pr.second);
        }
    ctx->timers.clear();
    ctx->timing_batches = 0;
    ctx->eager_batches = 0;
    ctx->timing_sel = true;
}

void bc_timing_batch(bc_ctx *ctx) {
    if (ctx->timing > 1) ctx->timing_sel = ctx->timing_batches % ctx->timing == 0;
    ++ctx->timing_batches;
}

void bc_timing_eager(bc_ctx *ctx) { ++ctx->eager_batches; }

LaunchTimer::LaunchTimer(bc_ctx *c, const char *nm) : ctx(c), name(nm) {
    if (ctx->recording || !ctx->timing || !ctx->timing_sel) return;
    a = bc_event_get(ctx);
    b = bc_event_get(ctx);
    if (a && b) {
        hipEventRecord(a, ctx->stream);
    } else {
        bc_event_put(ctx, a);
        bc_event_put(ctx, b);
        a = b = nullptr;
    }
}

void LaunchTimer::done() {
    if (ctx->recording || !ctx->timing) return;
    auto &t = ctx->timers[name];
    t.launches += 1;
    if (!a) return;
    hipEventRecord(b, ctx->stream);
    t.pending.emplace_back(a, b);
    t.timed += 1;
    a = b = nullptr;
}

// ---------------------------------------------------------------------------
// public entry points
// ---------------------------------------------------------------------------

extern "C" {

void bc_options_init(bc_options *opt) {
    if (!opt) return;
    memset(opt, 0, sizeof(*opt));
    opt->struct_size = sizeof(bc_options);
    opt->form = BC_FORM_AUTO;
    opt->batch = 0;
    opt->device = -1;
}

const char *bc_status_string(bc_status s) {
    switch (s) {
    case BC_OK: return "BC_OK: success";
    case BC_ERR_INVALID_ARG: return "BC_ERR_INVALID_ARG: invalid argument";
    case BC_ERR_INVALID_GRAPH: return "BC_ERR_INVALID_GRAPH: graph violates the input model";
    case BC_ERR_NOMEM: return "BC_ERR_NOMEM: out of memory";
    case BC_ERR_DEVICE: return "BC_ERR_DEVICE: HIP runtime error";
    case BC_ERR_OVERFLOW: return "BC_ERR_OVERFLOW: a shortest-path count exceeded 2^64-1";
    case BC_ERR_STATE: return "BC_ERR_STATE: call not allowed in the current state";
    case BC_ERR_UNSUPPORTED: return "BC_ERR_UNSUPPORTED: request not supported by this form";
    }
    return "unknown bc_status";
}

const char *bc_last_error(const bc_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

bc_status bc_create(const bc_graph *g, const bc_options *opt_in, bc_ctx **out) {
    if (!out) return fail_create(BC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!g) return fail_create(BC_ERR_INVALID_ARG, "graph is NULL");
    bc_options opt;
    bc_options_init(&opt);
    if (opt_in) {
        if (opt_in->struct_size != sizeof(bc_options))
            return fail_create(BC_ERR_INVALID_ARG, "bc_options.struct_size mismatch (call bc_options_init)");
        opt = *opt_in;
    }
    if (g->n < 0 || g->nnz < 0) return fail_create(BC_ERR_INVALID_ARG, "negative n or nnz");
    if (!g->row_ptr) return fail_create(BC_ERR_INVALID_ARG, "row_ptr is NULL");
    if (g->nnz > 0 && !g->col) return fail_create(BC_ERR_INVALID_ARG, "col is NULL");
    if (g->mem != BC_MEM_HOST && g->mem != BC_MEM_DEVICE)
        return fail_create(BC_ERR_INVALID_ARG, "graph mem must be BC_MEM_HOST or BC_MEM_DEVICE");
    if (opt.form < BC_FORM_AUTO || opt.form > BC_FORM_HYBRID)
        return fail_create(BC_ERR_INVALID_ARG, "unknown form");
    if (opt.batch < 0 || opt.batch % 64 != 0 || opt.batch > 4096)
        return fail_create(BC_ERR_INVALID_ARG, "batch must be 0 or a multiple of 64 up to 4096");
    if (opt.vertex_order != BC_ORDER_DEGREE && opt.vertex_order != BC_ORDER_INPUT)
        return fail_create(BC_ERR_INVALID_ARG, "unknown vertex_order");
    if (opt.arena_log2 < 0 || opt.arena_log2 > 30)
        return fail_create(BC_ERR_INVALID_ARG, "arena_log2 must be in [0, 30]");
    if (opt.grid < 0 || opt.grid > 65536)
        return fail_create(BC_ERR_INVALID_ARG, "grid must be in [0, 65536]");
    if (opt.timing < 0) return fail_create(BC_ERR_INVALID_ARG, "timing must be 0 (off) or k >= 1 (one launch in k)");
    if (opt.split_degree != 0 && opt.split_degree < 64)
        return fail_create(BC_ERR_INVALID_ARG, "split_degree must be 0 (default) or at least 64");
    if ((opt.allocator.alloc == nullptr) != (opt.allocator.free == nullptr))
        return fail_create(BC_ERR_INVALID_ARG, "allocator needs both alloc and free, or neither");

    const int32_t n = g->n, nnz = g->nnz;
    // Host copies (device inputs are copied down for validation).
    std::vector<int32_t> rp, col;
    std::vector<uint32_t> w;
    const int32_t *hrp = g->row_ptr, *hcol = g->col;
    const uint32_t *hw = g->weight;
    if (g->mem == BC_MEM_DEVICE) {
        rp.resize((size_t)n + 1);
        col.resize((size_t)std::max(nnz, 1));
        if (hipMemcpy(rp.data(), g->row_ptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost) != hipSuccess ||
            (nnz > 0 && hipMemcpy(col.data(), g->col, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToHost) != hipSuccess))
            return fail_create(BC_ERR_DEVICE, "copying the device graph to the host for validation failed");
        if (g->weight) {
            w.resize((size_t)std::max(nnz, 1));
            if (nnz > 0 && hipMemcpy(w.data(), g->weight, sizeof(uint32_t) * (size_t)nnz, hipMemcpyDeviceToHost) != hipSuccess)
                return fail_create(BC_ERR_DEVICE, "copying device weights failed");
            hw = w.data();
        }
        hrp = rp.data();
        hcol = col.data();
    }
    std::string msg;
    int32_t max_deg = 0;
    uint32_t max_w = 1;
    bc_status vs = validate_graph(n, nnz, hrp, hcol, hw, msg, max_deg, max_w);
    if (vs != BC_OK) return fail_create(vs, msg);

    bc_form form = opt.form;
    if (form == BC_FORM_AUTO) form = hw ? BC_FORM_PLAIN_FP64 : BC_FORM_SPARSE;
    if (opt.edges && form == BC_FORM_ALGEBRAIC)
        return fail_create(BC_ERR_UNSUPPORTED,
                           "edge betweenness needs per-arc terms; the algebraic form's products give row sums only");
    if (hw && (form == BC_FORM_SPARSE || form == BC_FORM_HYBRID))
        return fail_create(BC_ERR_UNSUPPORTED,
                           "weighted graphs are served by the per-source and algebraic forms only");
    if (hw && form == BC_FORM_ALGEBRAIC && max_w > BC_ALGEBRAIC_MAX_WEIGHT)
        return fail_create(BC_ERR_UNSUPPORTED,
                           "the algebraic form takes weights up to BC_ALGEBRAIC_MAX_WEIGHT (one product class each)");
    // An output of a forward product sums at most deg(w) limb terms of at
    // most 127 in int32; its FP32 copy for the epilogue is exact below 2^24,
    // which deg <= 65792 keeps with a factor of two to spare.  The hybrid form
    // runs such graphs by pulls.
    if (form == BC_FORM_ALGEBRAIC && max_deg > BC_ALGEBRAIC_MAX_DEGREE)
        return fail_create(BC_ERR_UNSUPPORTED,
                           "the algebraic form takes degrees up to BC_ALGEBRAIC_MAX_DEGREE (exact FP32 copies of "
                           "the products' sums)");

    // ---- device side ----
    bc_ctx *ctx = new (std::nothrow) bc_ctx();
    if (!ctx) return fail_create(BC_ERR_NOMEM, "host allocation of the context failed");
    ctx->n = n;
    ctx->nnz = nnz;
    ctx->max_degree = max_deg;
    ctx->max_weight = max_w;
    ctx->weighted = hw != nullptr;
    ctx->stream = (hipStream_t)opt.stream;
    ctx->alloc = opt.allocator;
    ctx->timing = opt.timing;
    ctx->host_driven = opt.host_driven != 0;
    ctx->form = form;

    auto bail = [&](bc_status s, const std::string &m) {
        const std::string msg = m; // m may be ctx->err, which delete frees
        release_all(ctx);
        delete ctx;
        return fail_create(s, msg);
    };
    int dev = opt.device;
    if (dev < 0) {
        if (hipGetDevice(&dev) != hipSuccess) return bail(BC_ERR_DEVICE, "hipGetDevice failed");
    }
    if (hipSetDevice(dev) != hipSuccess) return bail(BC_ERR_DEVICE, "hipSetDevice failed");
    ctx->device = dev;
    noalloc_init_device(dev);

    // Internal numbering: vertices by nonincreasing degree (stable), or as given.
    const bool relabel = opt.vertex_order == BC_ORDER_DEGREE && n > 1;
    std::vector<int32_t> new_of_old, irp, icol;
    std::vector<uint32_t> iw;
    const int32_t *urp = hrp, *ucol = hcol;
    const uint32_t *uw = hw;
    if (relabel) {
        std::vector<int32_t> old_of_new((size_t)n);
        for (int32_t v = 0; v < n; ++v) old_of_new[(size_t)v] = v;
        std::stable_sort(old_of_new.begin(), old_of_new.end(), [&](int32_t a, int32_t b) {
            return hrp[a + 1] - hrp[a] > hrp[b + 1] - hrp[b];
        });
        new_of_old.resize((size_t)n);
        for (int32_t u = 0; u < n; ++u) new_of_old[(size_t)old_of_new[(size_t)u]] = u;
        irp.resize((size_t)n + 1);
        icol.resize((size_t)std::max(nnz, 1));
        if (hw) iw.resize((size_t)std::max(nnz, 1));
        irp[0] = 0;
        std::vector<std::pair<int32_t, uint32_t>> row;
        for (int32_t u = 0; u < n; ++u) {
            const int32_t o = old_of_new[(size_t)u];
            const int32_t b = hrp[o], e = hrp[o + 1];
            irp[(size_t)u + 1] = irp[(size_t)u] + (e - b);
            row.clear();
            for (int32_t k = b; k < e; ++k) row.emplace_back(new_of_old[(size_t)hcol[k]], hw ? hw[k] : 1u);
            std::sort(row.begin(), row.end());
            for (size_t k = 0; k < row.size(); ++k) {
                icol[(size_t)irp[(size_t)u] + k] = row[k].first;
                if (hw) iw[(size_t)irp[(size_t)u] + k] = row[k].second;
            }
        }
        urp = irp.data();
        ucol = icol.data();
        uw = hw ? iw.data() : nullptr;
    }
    ctx->h_row_ptr.assign(urp, urp + (size_t)n + 1);
    ctx->wt.arena_log2 = opt.arena_log2;
    ctx->wt.grid = opt.grid;
    ctx->pl.grid = opt.grid;

    ctx->row_ptr = (int32_t *)bc_dalloc(ctx, sizeof(int32_t) * ((size_t)n + 1));
    ctx->col = (int32_t *)bc_dalloc(ctx, sizeof(int32_t) * (size_t)std::max(nnz, 1));
    ctx->bc = (double *)bc_dalloc(ctx, sizeof(double) * (size_t)std::max(n, 1));
    ctx->bc_scratch = (double *)bc_dalloc(ctx, sizeof(double) * (size_t)std::max(n, 1));
    ctx->status = (uint32_t *)bc_dalloc(ctx, 256);
    if (!ctx->row_ptr || !ctx->col || !ctx->bc || !ctx->bc_scratch || !ctx->status)
        return bail(BC_ERR_NOMEM, "device allocation failed");
    // Weights go to the device as bytes (the weighted sweep takes weights up
    // to 255 and refuses larger ones when it is prepared).
    std::vector<uint8_t> w8;
    if (hw && max_w <= 255) {
        w8.resize((size_t)std::max(nnz, 1));
        for (int32_t e = 0; e < nnz; ++e) w8[(size_t)e] = (uint8_t)uw[e];
        ctx->weight = (uint8_t *)bc_dalloc(ctx, (size_t)std::max(nnz, 1));
        if (!ctx->weight) return bail(BC_ERR_NOMEM, "device allocation failed");
    }
    if (relabel) {
        ctx->new_of_old = (int32_t *)bc_dalloc(ctx, sizeof(int32_t) * (size_t)n);
        if (!ctx->new_of_old) return bail(BC_ERR_NOMEM, "device allocation failed");
    }
    if (hipHostMalloc((void **)&ctx->status_host, 256) != hipSuccess) return bail(BC_ERR_NOMEM, "pinned allocation failed");
    // Connected components (internal numbering): a source reaches exactly the
    // vertices of its own, which lets a batch know when its search is over.
    std::vector<int32_t> csize((size_t)std::max(n, 1), 0);
    {
        std::vector<int32_t> comp((size_t)n, -1), queue((size_t)n), sizes;
        for (int32_t r = 0; r < n; ++r) {
            if (comp[(size_t)r] >= 0) continue;
            const int32_t id = (int32_t)sizes.size();
            size_t head = 0, tail = 0;
            queue[tail++] = r;
            comp[(size_t)r] = id;
            while (head < tail) {
                const int32_t v = queue[head++];
                for (int32_t e = urp[v]; e < urp[v + 1]; ++e)
                    if (comp[(size_t)ucol[e]] < 0) {
                        comp[(size_t)ucol[e]] = id;
                        queue[tail++] = ucol[e];
                    }
            }
            sizes.push_back((int32_t)tail);
        }
        for (int32_t v = 0; v < n; ++v) csize[(size_t)v] = sizes[(size_t)comp[(size_t)v]];
    }
    ctx->comp_size = (int32_t *)bc_dalloc(ctx, sizeof(int32_t) * (size_t)std::max(n, 1));
    if (!ctx->comp_size) return bail(BC_ERR_NOMEM, "device allocation failed");
    // Host arrays (the caller's or the relabelled copies) go up synchronously.
    const bool direct_device = !relabel && g->mem == BC_MEM_DEVICE;
    hipMemcpyKind kind = direct_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (hipMemcpy(ctx->row_ptr, urp, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice) != hipSuccess ||
        (nnz > 0 && hipMemcpy(ctx->col, direct_device ? g->col : ucol, sizeof(int32_t) * (size_t)nnz, kind) != hipSuccess) ||
        (ctx->weight && nnz > 0 && hipMemcpy(ctx->weight, w8.data(), (size_t)nnz, hipMemcpyHostToDevice) != hipSuccess) ||
        (relabel && hipMemcpy(ctx->new_of_old, new_of_old.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice) != hipSuccess) ||
        hipMemcpy(ctx->comp_size, csize.data(), sizeof(int32_t) * (size_t)std::max(n, 1), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemsetAsync(ctx->bc, 0, sizeof(double) * (size_t)std::max(n, 1), ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->status, 0, 256, ctx->stream) != hipSuccess)
        return bail(BC_ERR_DEVICE, "uploading the graph failed");

    if (opt.edges) {
        // caller arc e = (u, x) -> internal arcs (u', x') and (x', u'), found
        // in the sorted internal rows
        ctx->edges = true;
        std::vector<int32_t> fwd((size_t)std::max(nnz, 1)), rev((size_t)std::max(nnz, 1));
        auto find = [&](int32_t row, int32_t x) {
            const int32_t *b = ucol + urp[row], *e = ucol + urp[row + 1];
            return (int32_t)(std::lower_bound(b, e, x) - ucol);
        };
        for (int32_t u = 0; u < n; ++u)
            for (int32_t e = hrp[u]; e < hrp[u + 1]; ++e) {
                const int32_t x = hcol[e];
                const int32_t iu = relabel ? new_of_old[(size_t)u] : u, ix = relabel ? new_of_old[(size_t)x] : x;
                fwd[(size_t)e] = find(iu, ix);
                rev[(size_t)e] = find(ix, iu);
            }
        ctx->eb = (double *)bc_dalloc(ctx, sizeof(double) * (size_t)std::max(nnz, 1));
        ctx->eb_scratch = (double *)bc_dalloc(ctx, sizeof(double) * (size_t)std::max(nnz, 1));
        ctx->arc_fwd = (int32_t *)bc_dalloc(ctx, sizeof(int32_t) * (size_t)std::max(nnz, 1));
        ctx->arc_rev = (int32_t *)bc_dalloc(ctx, sizeof(int32_t) * (size_t)std::max(nnz, 1));
        if (!ctx->eb || !ctx->eb_scratch || !ctx->arc_fwd || !ctx->arc_rev)
            return bail(BC_ERR_NOMEM, "device allocation failed");
        if (hipMemsetAsync(ctx->eb, 0, sizeof(double) * (size_t)std::max(nnz, 1), ctx->stream) != hipSuccess ||
            (nnz > 0 && (hipMemcpy(ctx->arc_fwd, fwd.data(), sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice) != hipSuccess ||
                         hipMemcpy(ctx->arc_rev, rev.data(), sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice) != hipSuccess)))
            return bail(BC_ERR_DEVICE, "uploading the arc maps failed");
    }

    bc_status ps = BC_OK;
    if (form == BC_FORM_PLAIN_FP64) ps = plain_prepare(ctx);
    else if (form == BC_FORM_SPARSE || form == BC_FORM_HYBRID || form == BC_FORM_ALGEBRAIC)
        ps = tune_prepare(ctx, opt, form);
    if (ps != BC_OK) return bail(ps, ctx->err);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return bail(BC_ERR_DEVICE, "stream synchronisation failed");
    *out = ctx;
    return BC_OK;
}


bc_status bc_create_many(const bc_graph *gs, int32_t count, const bc_options *opt_in, bc_ctx **out) {
    if (!out) return fail_create(BC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (count < 0 || (count > 0 && !gs)) return fail_create(BC_ERR_INVALID_ARG, "bad graph list");
    bc_options opt;
    bc_options_init(&opt);
    if (opt_in) {
        if (opt_in->struct_size != sizeof(bc_options))
            return fail_create(BC_ERR_INVALID_ARG, "bc_options.struct_size mismatch (call bc_options_init)");
        opt = *opt_in;
    }
    if (opt.batch < 0) return fail_create(BC_ERR_INVALID_ARG, "batch must be >= 0");
    if (opt.edges) return fail_create(BC_ERR_UNSUPPORTED, "bc_create_many computes vertex betweenness only");
    if (opt.timing < 0) return fail_create(BC_ERR_INVALID_ARG, "timing must be 0 (off) or k >= 1 (one launch in k)");
    if ((opt.allocator.alloc == nullptr) != (opt.allocator.free == nullptr))
        return fail_create(BC_ERR_INVALID_ARG, "allocator needs both alloc and free, or neither");
    // host validation of every graph, then the concatenated layout
    std::vector<int32_t> voff(1, 0), rpoff, rp, col;
    int64_t total_n = 0, total_arcs = 0;
    int32_t max_deg = 0;
    for (int32_t g = 0; g < count; ++g) {
        const bc_graph &G = gs[g];
        char buf[160];
        if (G.mem != BC_MEM_HOST) return fail_create(BC_ERR_INVALID_ARG, "bc_create_many takes host graphs");
        if (G.n < 0 || G.nnz < 0 || !G.row_ptr || (G.nnz > 0 && !G.col)) {
            snprintf(buf, sizeof buf, "graph %d: bad arrays", g);
            return fail_create(BC_ERR_INVALID_ARG, buf);
        }
        if (G.weight) return fail_create(BC_ERR_UNSUPPORTED, "bc_create_many takes unweighted graphs");
        if (G.n > MG_MAX_N) {
            snprintf(buf, sizeof buf, "graph %d has %d vertices; at most %d are supported", g, G.n, MG_MAX_N);
            return fail_create(BC_ERR_UNSUPPORTED, buf);
        }
        std::string msg;
        int32_t md = 0;
        uint32_t mw = 1;
        bc_status vs = validate_graph(G.n, G.nnz, G.row_ptr, G.col, nullptr, msg, md, mw);
        if (vs != BC_OK) {
            snprintf(buf, sizeof buf, "graph %d: ", g);
            return fail_create(vs, buf + msg);
        }
        max_deg = std::max(max_deg, md);
        if (total_n + G.n >= (int64_t(1) << 31) || total_arcs + G.nnz >= (int64_t(1) << 31))
            return fail_create(BC_ERR_INVALID_GRAPH, "the graphs together exceed 2^31 vertices or arcs");
        rpoff.push_back((int32_t)rp.size());
        for (int32_t v = 0; v <= G.n; ++v) rp.push_back((int32_t)total_arcs + G.row_ptr[v]);
        col.insert(col.end(), G.col, G.col + G.nnz);
        total_n += G.n;
        total_arcs += G.nnz;
        voff.push_back((int32_t)total_n);
    }
    bc_ctx *ctx = new (std::nothrow) bc_ctx();
    if (!ctx) return fail_create(BC_ERR_NOMEM, "host allocation of the context failed");
    ctx->n = (int32_t)total_n;
    ctx->nnz = (int32_t)total_arcs;
    ctx->max_degree = max_deg;
    ctx->stream = (hipStream_t)opt.stream;
    ctx->alloc = opt.allocator;
    ctx->timing = opt.timing;
    ctx->form = BC_FORM_MANY;
    ctx->many = true;
    auto bail = [&](bc_status s, const std::string &m) {
        const std::string msg = m; // m may be ctx->err, which delete frees
        release_all(ctx);
        delete ctx;
        return fail_create(s, msg);
    };
    int dev = opt.device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return bail(BC_ERR_DEVICE, "hipGetDevice failed");
    if (hipSetDevice(dev) != hipSuccess) return bail(BC_ERR_DEVICE, "hipSetDevice failed");
    ctx->device = dev;
    noalloc_init_device(dev);
    if (hipStreamCreateWithFlags(&ctx->mg.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->mg.ev, hipEventDisableTiming) != hipSuccess)
        return bail(BC_ERR_DEVICE, "stream creation failed");
    const size_t nn = (size_t)std::max<int64_t>(total_n, 1);
    ctx->col = (int32_t *)bc_dalloc(ctx, sizeof(int32_t) * (size_t)std::max<int64_t>(total_arcs, 1));
    ctx->bc = (double *)bc_dalloc(ctx, sizeof(double) * nn);
    ctx->bc_scratch = (double *)bc_dalloc(ctx, sizeof(double) * nn);
    ctx->status = (uint32_t *)bc_dalloc(ctx, 256);
    if (!ctx->col || !ctx->bc || !ctx->bc_scratch || !ctx->status ||
        hipHostMalloc((void **)&ctx->status_host, 256) != hipSuccess)
        return bail(BC_ERR_NOMEM, "device allocation failed");
    if ((total_arcs > 0 &&
         hipMemcpy(ctx->col, col.data(), sizeof(int32_t) * (size_t)total_arcs, hipMemcpyHostToDevice) != hipSuccess) ||
        hipMemsetAsync(ctx->bc, 0, sizeof(double) * nn, ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->status, 0, 256, ctx->stream) != hipSuccess)
        return bail(BC_ERR_DEVICE, "uploading the graphs failed");
    bc_status ps = tune_many(ctx, opt, voff, rpoff, rp);
    if (ps != BC_OK) return bail(ps, ctx->err);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return bail(BC_ERR_DEVICE, "stream synchronisation failed");
    *out = ctx;
    return BC_OK;
}

static bc_status stage_sources(bc_ctx *ctx, const int32_t *sources, int64_t count, bc_mem mem,
                               const int32_t **d_out, int64_t *count_out) {
    if (count == -1 && sources == nullptr) count = ctx->n;
    else if (count < 0 || (count > 0 && !sources)) return bc_fail(ctx, BC_ERR_INVALID_ARG, "bad sources/count");
    if (mem != BC_MEM_HOST && mem != BC_MEM_DEVICE) return bc_fail(ctx, BC_ERR_INVALID_ARG, "bad mem");
    if (count > ctx->sources_cap) {
        if (ctx->sources) bc_dfree(ctx, ctx->sources);
        ctx->sources = (int32_t *)bc_dalloc(ctx, sizeof(int32_t) * (size_t)count);
        if (!ctx->sources) { ctx->sources_cap = 0; return bc_fail(ctx, BC_ERR_NOMEM, "source staging allocation failed"); }
        ctx->sources_cap = count;
    }
    if (sources == nullptr) { // "every vertex", generated on the device in internal ids
        bc_status fs = fill_all_sources(ctx, ctx->sources, count);
        if (fs != BC_OK) return fs;
        *d_out = ctx->sources;
        *count_out = count;
        return BC_OK;
    }
    // Explicit sources: validated on the host (a device list is read back first).
    std::vector<int32_t> host;
    const int32_t *hs = sources;
    if (mem == BC_MEM_DEVICE) {
        host.resize((size_t)count);
        BC_HIP(ctx, hipMemcpy(host.data(), sources, sizeof(int32_t) * (size_t)count, hipMemcpyDeviceToHost));
        hs = host.data();
    }
    for (int64_t i = 0; i < count; ++i)
        if (hs[i] < 0 || hs[i] >= ctx->n) {
            char buf[128];
            snprintf(buf, sizeof buf, "source %d at position %lld is outside [0,%d)", hs[i], (long long)i, ctx->n);
            return bc_fail(ctx, BC_ERR_INVALID_ARG, buf);
        }
    if (count > 0)
        BC_HIP(ctx, hipMemcpyAsync(ctx->sources, hs, sizeof(int32_t) * (size_t)count, hipMemcpyHostToDevice, ctx->stream));
    // the caller's (or our) host array must stay alive until the copy is done
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    bc_status ms = map_ids_to_internal(ctx, ctx->sources, count);
    if (ms != BC_OK) return ms;
    *d_out = ctx->sources;
    *count_out = count;
    return BC_OK;
}

} // extern "C"

bc_status bc_check_usable(bc_ctx *ctx) {
    if (ctx->poisoned) return bc_fail(ctx, BC_ERR_STATE, "context poisoned by an earlier device error");
    if (hipSetDevice(ctx->device) != hipSuccess) return bc_hip(ctx, hipErrorInvalidDevice, "hipSetDevice");
    // Every call may synchronise the stream or read results back, which a
    // stream under graph capture does not allow; nothing is recorded.
    if (ctx->stream) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(ctx->stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
            return bc_fail(ctx, BC_ERR_STATE, "the context's stream is being captured into a HIP graph");
    }
    // batches replayed by an earlier bc_run: read their checks, re-run what
    // they handed back
    return sparse_settle(ctx);
}

extern "C" {

static bc_status check_overflow(bc_ctx *ctx) {
    BC_HIP(ctx, hipMemcpyAsync(ctx->status_host, ctx->status, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream));
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (*ctx->status_host & BC_DEV_SIGMA_OVERFLOW) {
        ctx->overflow_seen = true;
        return bc_fail(ctx, BC_ERR_OVERFLOW, "a shortest-path count exceeded 2^64 - 1");
    }
    return BC_OK;
}

bc_status bc_run(bc_ctx *ctx, const int32_t *sources, int64_t count, bc_mem mem) {
    if (!ctx) return BC_ERR_INVALID_ARG;
    bc_status s = bc_check_usable(ctx);
    if (s != BC_OK) return s;
    if (ctx->overflow_seen) return bc_fail(ctx, BC_ERR_OVERFLOW, "an earlier run overflowed a path count; call bc_reset");
    if (ctx->many) {
        if (sources != nullptr || count != -1)
            return bc_fail(ctx, BC_ERR_UNSUPPORTED, "a many-graph context runs every source: pass NULL, -1");
        s = multigraph_run(ctx);
        if (s == BC_OK) ctx->sources_run += ctx->n;
        return s;
    }
    const int32_t *d_src = nullptr;
    int64_t cnt = 0;
    s = stage_sources(ctx, sources, count, mem, &d_src, &cnt);
    if (s != BC_OK) return s;
    if (cnt == 0 || ctx->n == 0) return BC_OK;
    if (ctx->form == BC_FORM_PLAIN_FP64) s = plain_run(ctx, d_src, cnt, true, nullptr, nullptr, nullptr);
    else if (ctx->form == BC_FORM_SPARSE || ctx->form == BC_FORM_ALGEBRAIC || ctx->form == BC_FORM_HYBRID)
        s = sparse_run(ctx, d_src, cnt);
    else s = bc_fail(ctx, BC_ERR_UNSUPPORTED, "form not available");
    if (s == BC_OK) ctx->sources_run += cnt;
    return s;
}

bc_status bc_read(bc_ctx *ctx, double *bc_out, bc_mem mem) {
    if (!ctx) return BC_ERR_INVALID_ARG;
    if (!bc_out && ctx->n > 0) return bc_fail(ctx, BC_ERR_INVALID_ARG, "bc_out is NULL");
    bc_status s = bc_check_usable(ctx);
    if (s != BC_OK) return s;
    s = check_overflow(ctx);
    if (s != BC_OK) return s;
    if (ctx->n == 0) return BC_OK;
    s = rows_to_caller_order_f64(ctx, ctx->bc_scratch, ctx->bc, 1);
    if (s != BC_OK) return s;
    BC_HIP(ctx, hipMemcpyAsync(bc_out, ctx->bc_scratch, sizeof(double) * (size_t)ctx->n,
                               mem == BC_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, ctx->stream));
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return BC_OK;
}

bc_status bc_read_edges(bc_ctx *ctx, double *eb_out, bc_mem mem) {
    if (!ctx) return BC_ERR_INVALID_ARG;
    if (!ctx->edges) return bc_fail(ctx, BC_ERR_UNSUPPORTED, "the context was created without edges");
    if (!eb_out && ctx->nnz > 0) return bc_fail(ctx, BC_ERR_INVALID_ARG, "eb_out is NULL");
    bc_status s = bc_check_usable(ctx);
    if (s != BC_OK) return s;
    s = check_overflow(ctx);
    if (s != BC_OK) return s;
    if (ctx->nnz == 0) return BC_OK;
    s = edges_to_caller_order(ctx, ctx->eb_scratch);
    if (s != BC_OK) return s;
    BC_HIP(ctx, hipMemcpyAsync(eb_out, ctx->eb_scratch, sizeof(double) * (size_t)ctx->nnz,
                               mem == BC_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, ctx->stream));
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return BC_OK;
}

bc_status bc_reset(bc_ctx *ctx) {
    if (!ctx) return BC_ERR_INVALID_ARG;
    bc_status s = bc_check_usable(ctx);
    if (s != BC_OK) return s;
    BC_HIP(ctx, hipMemsetAsync(ctx->bc, 0, sizeof(double) * (size_t)std::max(ctx->n, 1), ctx->stream));
    if (ctx->eb) BC_HIP(ctx, hipMemsetAsync(ctx->eb, 0, sizeof(double) * (size_t)std::max(ctx->nnz, 1), ctx->stream));
    BC_HIP(ctx, hipMemsetAsync(ctx->status, 0, 256, ctx->stream));
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    bc_timers_clear(ctx);
    algebraic_reset_counters(ctx);
    ctx->overflow_seen = false;
    ctx->sources_run = 0;
    return BC_OK;
}

// Calls that run sources without adding to BC (per-source dumps, all pairs)
// share the device overflow flag with bc_run: they save it and clear it first,
// then read what they raised and put the saved value back.
} // extern "C"

bc_status bc_status_save(bc_ctx *ctx, uint32_t *before) {
    BC_HIP(ctx, hipMemcpyAsync(ctx->status_host, ctx->status, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream));
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *before = *ctx->status_host;
    BC_HIP(ctx, hipMemsetAsync(ctx->status, 0, sizeof(uint32_t), ctx->stream));
    return BC_OK;
}

bc_status bc_status_restore(bc_ctx *ctx, uint32_t before, uint32_t *now) {
    BC_HIP(ctx, hipMemcpyAsync(ctx->status_host, ctx->status, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream));
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *now = *ctx->status_host;
    *ctx->status_host = before;
    BC_HIP(ctx, hipMemcpyAsync(ctx->status, ctx->status_host, sizeof(uint32_t), hipMemcpyHostToDevice, ctx->stream));
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return BC_OK;
}

extern "C" {

bc_status bc_read_sssp(bc_ctx *ctx, const int32_t *sources, int32_t count,
                       int32_t *dist, uint64_t *sigma, double *delta) {
    if (!ctx) return BC_ERR_INVALID_ARG;
    bc_status s = bc_check_usable(ctx);
    if (s != BC_OK) return s;
    int32_t maxc = ctx->many ? 64 : ctx->form == BC_FORM_PLAIN_FP64 ? 4096 : ctx->sp.batch;
    if (!sources || count < 1 || count > maxc) return bc_fail(ctx, BC_ERR_INVALID_ARG, "count must be in [1, batch]");
    const int32_t *d_src = nullptr;
    int64_t cnt = 0;
    s = stage_sources(ctx, sources, count, BC_MEM_HOST, &d_src, &cnt);
    if (s != BC_OK) return s;
    size_t cells = (size_t)count * (size_t)std::max(ctx->n, 1);
    int32_t *dd = (int32_t *)bc_dalloc(ctx, cells * sizeof(int32_t));
    uint64_t *ds = (uint64_t *)bc_dalloc(ctx, cells * sizeof(uint64_t));
    double *dl = (double *)bc_dalloc(ctx, cells * sizeof(double));
    int32_t *od = (int32_t *)bc_dalloc(ctx, cells * sizeof(int32_t));
    uint64_t *os = (uint64_t *)bc_dalloc(ctx, cells * sizeof(uint64_t));
    double *ol = (double *)bc_dalloc(ctx, cells * sizeof(double));
    auto cleanup = [&]() {
        bc_dfree(ctx, dd); bc_dfree(ctx, ds); bc_dfree(ctx, dl);
        bc_dfree(ctx, od); bc_dfree(ctx, os); bc_dfree(ctx, ol);
    };
    if (!dd || !ds || !dl || !od || !os || !ol) { cleanup(); return bc_fail(ctx, BC_ERR_NOMEM, "dump allocation failed"); }
    uint32_t before = 0, now = 0;
    if ((s = bc_status_save(ctx, &before)) != BC_OK) { cleanup(); return s; }
    bc_status run;
    if (ctx->many) run = multigraph_dump(ctx, sources, count, dd, ds, dl);
    else if (ctx->form == BC_FORM_PLAIN_FP64) run = plain_run(ctx, d_src, count, false, dl, dd, ds);
    else run = sparse_dump(ctx, d_src, count, dd, ds, dl);
    if (run != BC_ERR_DEVICE) s = bc_status_restore(ctx, before, &now);
    if (run != BC_OK || s != BC_OK) { cleanup(); return run != BC_OK ? run : s; }
    if (now & BC_DEV_SIGMA_OVERFLOW) { cleanup(); return bc_fail(ctx, BC_ERR_OVERFLOW, "a shortest-path count exceeded 2^64 - 1"); }
    if (ctx->n > 0) {
        if ((s = rows_to_caller_order_i32(ctx, od, dd, count)) != BC_OK ||
            (s = rows_to_caller_order_u64(ctx, os, ds, count)) != BC_OK ||
            (s = rows_to_caller_order_f64(ctx, ol, dl, count)) != BC_OK) { cleanup(); return s; }
        BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (dist) BC_HIP(ctx, hipMemcpy(dist, od, cells * sizeof(int32_t), hipMemcpyDeviceToHost));
        if (sigma) BC_HIP(ctx, hipMemcpy(sigma, os, cells * sizeof(uint64_t), hipMemcpyDeviceToHost));
        if (delta) BC_HIP(ctx, hipMemcpy(delta, ol, cells * sizeof(double), hipMemcpyDeviceToHost));
    }
    cleanup();
    return BC_OK;
}

bc_status bc_all_pairs(bc_ctx *ctx, double *bc_out, bc_mem mem) {
    if (!ctx) return BC_ERR_INVALID_ARG;
    if (!bc_out && ctx->n > 0) return bc_fail(ctx, BC_ERR_INVALID_ARG, "bc_out is NULL");
    bc_status s = bc_check_usable(ctx);
    if (s != BC_OK) return s;
    if (ctx->many) return bc_fail(ctx, BC_ERR_UNSUPPORTED, "all pairs: not for a context of many graphs");
    if (ctx->n > BC_ALL_PAIRS_MAX_N)
        return bc_fail(ctx, BC_ERR_UNSUPPORTED, "all pairs: n above BC_ALL_PAIRS_MAX_N");
    if (ctx->n == 0) return BC_OK;
    double *res = (double *)bc_dalloc(ctx, sizeof(double) * (size_t)ctx->n);
    if (!res) return bc_fail(ctx, BC_ERR_NOMEM, "all pairs: result allocation failed");
    uint32_t before = 0, now = 0;
    if ((s = bc_status_save(ctx, &before)) != BC_OK) {
        bc_dfree(ctx, res);
        return s;
    }
    const bc_status run = allpairs_bc(ctx, res);
    if (run != BC_ERR_DEVICE) s = bc_status_restore(ctx, before, &now);
    if (run != BC_OK || s != BC_OK) {
        bc_dfree(ctx, res);
        return run != BC_OK ? run : s;
    }
    if (now & BC_DEV_SIGMA_OVERFLOW) {
        bc_dfree(ctx, res);
        return bc_fail(ctx, BC_ERR_OVERFLOW, "a shortest-path count exceeded 2^64 - 1");
    }
    s = rows_to_caller_order_f64(ctx, ctx->bc_scratch, res, 1);
    if (s == BC_OK) {
        hipError_t e = hipMemcpyAsync(bc_out, ctx->bc_scratch, sizeof(double) * (size_t)ctx->n,
                                      mem == BC_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                      ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) s = bc_hip(ctx, e, "all pairs: copy out");
    }
    bc_dfree(ctx, res);
    return s;
}

bc_status bc_sampled_distances(bc_ctx *ctx, const int32_t *sources, int32_t count, const int32_t *sample,
                               int32_t nsample, int32_t limit, int32_t *dist_out, bc_mem mem) {
    if (!ctx) return BC_ERR_INVALID_ARG;
    bc_status s = bc_check_usable(ctx);
    if (s != BC_OK) return s;
    if (ctx->many) return bc_fail(ctx, BC_ERR_UNSUPPORTED, "sampled forward: not for a context of many graphs");
    if (ctx->weighted) return bc_fail(ctx, BC_ERR_UNSUPPORTED, "sampled forward: unweighted graphs only");
    if (count < 0 || nsample < 0 || limit < 0 || (count > 0 && (!sources || !dist_out)) || (nsample > 0 && !sample) ||
        (mem != BC_MEM_HOST && mem != BC_MEM_DEVICE))
        return bc_fail(ctx, BC_ERR_INVALID_ARG, "sampled forward: bad arguments");
    for (int32_t i = 0; i < count; ++i)
        if (sources[i] < 0 || sources[i] >= ctx->n) return bc_fail(ctx, BC_ERR_INVALID_ARG, "source id out of range");
    for (int32_t i = 0; i < nsample; ++i)
        if (sample[i] < 0 || sample[i] >= ctx->n) return bc_fail(ctx, BC_ERR_INVALID_ARG, "sample id out of range");
    if (count == 0 || ctx->n == 0) return BC_OK;
    return sampled_distances(ctx, sources, count, sample, nsample, limit, dist_out, mem == BC_MEM_DEVICE);
}

bc_status bc_get_info(const bc_ctx *ctx, bc_info *out) {
    if (!ctx || !out) return BC_ERR_INVALID_ARG;
    if (!ctx->poisoned) (void)sparse_settle(const_cast<bc_ctx *>(ctx)); // replays' depth and sources
    memset(out, 0, sizeof(*out));
    out->n = ctx->n;
    out->m = ctx->nnz / 2;
    out->max_degree = ctx->max_degree;
    out->weighted = ctx->weighted ? 1 : 0;
    out->form = ctx->form;
    out->batch = ctx->many ? ctx->mg.chunk : ctx->form == BC_FORM_PLAIN_FP64 ? 1 : ctx->sp.batch;
    out->max_levels = ctx->max_levels;
    out->sources_run = ctx->sources_run;
    out->device_bytes = ctx->device_bytes;
    const bool every = ctx->form == BC_FORM_ALGEBRAIC;
    const bool hybrid = ctx->form == BC_FORM_HYBRID && ctx->hy.products;
    out->mfma_density_fwd = every ? 0.0 : hybrid ? ctx->hy.theta_fwd : 2.0;
    out->mfma_density_bwd = every ? 0.0 : hybrid ? ctx->hy.theta_bwd : 2.0;
    out->tune_source = ctx->hy.tune_source;
    out->mfma_fwd_rows = every || hybrid ? ctx->al.fwd_rows : 0;
    out->mfma_planes = ctx->poisoned ? 0 : algebraic_planes_issued(const_cast<bc_ctx *>(ctx));
    out->mfma_ktiles_run = out->mfma_ktiles_dense = out->mfma_ktiles_run_fwd = out->mfma_ktiles_dense_fwd = 0;
    if (!ctx->poisoned && !algebraic_ktiles(const_cast<bc_ctx *>(ctx), &out->mfma_ktiles_run, &out->mfma_ktiles_dense,
                                            &out->mfma_ktiles_run_fwd, &out->mfma_ktiles_dense_fwd))
        out->mfma_ktiles_run = out->mfma_ktiles_dense = out->mfma_ktiles_run_fwd = out->mfma_ktiles_dense_fwd = -1;
    return BC_OK;
}

bc_status bc_get_timing(bc_ctx *ctx, const char *kernel, double *total_ms, int64_t *launches) {
    if (!ctx || !kernel || !total_ms || !launches) return BC_ERR_INVALID_ARG;
    *total_ms = 0.0;
    *launches = 0;
    if (!ctx->poisoned) (void)sparse_settle(ctx); // replays' handed-back batches are counted too
    auto it = ctx->timers.find(kernel);
    if (it == ctx->timers.end()) return BC_OK;
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (auto &pr : it->second.pending) {
        float ms = 0.f;
        BC_HIP(ctx, hipEventElapsedTime(&ms, pr.first, pr.second));
        it->second.total_ms += ms;
        bc_event_put(ctx, pr.first);
        bc_event_put(ctx, pr.second);
    }
    it->second.pending.clear();
    const KernelTimer &t = it->second;
    // host-driven batches count their launches; replayed ones are alike and
    // carry no events: scale by batches
    const double f = ctx->eager_batches > 0 && ctx->timing_batches > ctx->eager_batches
                         ? (double)ctx->timing_batches / (double)ctx->eager_batches
                         : 1.0;
    *total_ms = t.timed ? t.total_ms * (double)t.launches / (double)t.timed * f : 0.0;
    *launches = (int64_t)std::llround((double)t.launches * f);
    return BC_OK;
}

void bc_destroy(bc_ctx *ctx) {
    if (!ctx) return;
    release_all(ctx);
    delete ctx;
}

} // extern "C"
