// Autotuning of the batched forms and of the many-graph queue.
//
// The paper analyses one method at a time; choosing between them per level is
// this library's own addition.  Before any timed work, the tuner fixes
//   * the batch width B of the sparse and hybrid forms;
//   * the hybrid form's two density thresholds: forward level l -> l+1 (and
//     backward level l) is computed by products with the adjacency matrix
//     (Sec. 3.1) when the level's union-frontier density reaches the
//     threshold, and by CSR pulls (the level sweep of Sec. 4) otherwise;
//   * for the hybrid form, also whole batches with every level by products
//     (the algebraic form's mode, whose products count the pairs they reach
//     and so skip the empty level that ends a search), kept when faster;
//   * the rows of the adjacency one workgroup of the forward products takes
//     (128 or 256), for the algebraic form and a hybrid form with forward
//     products;
//   * the sources per work unit of bc_create_many's queue.
// It measures calibration batches of sources drawn from the graph itself,
// each width once with every level by pulls and once with every level >= 1 by
// products, records every level's GPU time and density, and picks for each
// direction the threshold that minimises the summed time of the recorded
// levels; block rows and unit sizes are timed over whole batches or
// launches.  Results are cached per process and, optionally, in a text file.
#include "bc_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

namespace {

constexpr int32_t kTinyN = 2048;                    // smaller graphs take the defaults
constexpr size_t kStateBudget = size_t(24) << 30;   // batch state allowed for a candidate width
// padded vertex count up to which the hybrid form considers products: one
// product costs 2 B npad^2 flops whatever the level's size
constexpr size_t kHybridMaxNpad = 92672;
constexpr int kReps = 2;                            // timed calibration batches per width and mode
constexpr double kSyncMs = 0.02;                    // host round trip per level of a stepwise forward
constexpr double kNever = 2.0;                      // a threshold no density reaches
// thresholds of the hybrid form's every-level mode in the cache file: every
// level l >= 1 by products, with the end of search the algebraic form has
constexpr double kEvery = -1.0;
constexpr double kAccept = 0.97;                    // a mix must beat pulls by 3% to be kept
constexpr int kConfirm = 3;                         // alternating whole-batch comparisons of a mix
constexpr double kManySampleWork = 3e9;             // many graphs: sum of n_g (n_g + arcs_g) one timed launch takes
const int32_t kUnitSizes[] = {16, 32, 64, 128, 256}; // many graphs: sources per work unit tried

struct TuneResult {
    int32_t batch; // sources per batch, or per work unit for many graphs
    double theta_fwd, theta_bwd;
    int32_t fwd_rows; // forward product block rows; 0 = not recorded (128)
};

std::mutex g_mu;
std::map<std::string, TuneResult> g_cache;

uint64_t fnv1a(const void *p, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    return h;
}

// Values in log2 buckets, each bucket's share quantised to 1/64, hashed.
uint64_t log2_histogram_hash(const std::vector<uint32_t> &vals) {
    int64_t hist[33] = {0};
    for (uint32_t x : vals) ++hist[31 - __builtin_clz(x + 1u)];
    uint8_t q[33];
    for (int k = 0; k < 33; ++k)
        q[k] = (uint8_t)std::lround(64.0 * (double)hist[k] / (double)std::max<size_t>(vals.size(), 1));
    return fnv1a(q, sizeof q);
}

std::string device_key(int device) {
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) std::strcpy(prop.gcnArchName, "unknown");
    char buf[160];
    std::snprintf(buf, sizeof buf, " arch=%s cu=%d", prop.gcnArchName, prop.multiProcessorCount);
    return buf;
}

std::string clean_key(std::string k) {
    for (char &c : k)
        if (c == '\t' || c == '\n') c = ' ';
    return k;
}

// Graph shape key: n, m, the largest weight (0 unweighted), the degree
// histogram, the form, the requested width, the row split and the device.
std::string make_key(const bc_ctx *ctx, bc_form form, int32_t req_batch, int32_t split) {
    std::vector<uint32_t> deg((size_t)ctx->n);
    const std::vector<int32_t> &rp = ctx->h_row_ptr;
    for (int32_t v = 0; v < ctx->n; ++v) deg[(size_t)v] = (uint32_t)(rp[(size_t)v + 1] - rp[(size_t)v]);
    char buf[256];
    std::snprintf(buf, sizeof buf, "n=%d m=%lld w=%u dh=%016llx form=%d batch=%d split=%d", ctx->n,
                  (long long)ctx->nnz / 2, ctx->weighted ? ctx->max_weight : 0u,
                  (unsigned long long)log2_histogram_hash(deg), (int)form, req_batch, split);
    return clean_key(buf + device_key(ctx->device));
}

// Many graphs: their number, total vertices and arcs, and the histograms of
// their vertex and arc counts.
std::string make_many_key(const bc_ctx *ctx) {
    const MultiState &m = ctx->mg;
    std::vector<uint32_t> ns((size_t)m.ngraphs), arcs((size_t)m.ngraphs);
    for (int32_t g = 0; g < m.ngraphs; ++g) {
        ns[(size_t)g] = (uint32_t)(m.h_voff[(size_t)g + 1] - m.h_voff[(size_t)g]);
        arcs[(size_t)g] = (uint32_t)m.h_arcs[(size_t)g];
    }
    char buf[256];
    std::snprintf(buf, sizeof buf, "many graphs=%d n=%d arcs=%lld nh=%016llx ah=%016llx form=%d batch=0", m.ngraphs,
                  ctx->n, (long long)ctx->nnz, (unsigned long long)log2_histogram_hash(ns),
                  (unsigned long long)log2_histogram_hash(arcs), (int)BC_FORM_MANY);
    return clean_key(buf + device_key(ctx->device));
}

// File format: one entry per line,
// "<key>\t<batch> <theta_fwd> <theta_bwd> [<fwd_rows>]"; the last entry for a
// key wins; lines starting with '#' are ignored.
bool file_lookup(const char *path, const std::string &key, TuneResult &out) {
    std::ifstream f(path);
    if (!f) return false;
    bool found = false;
    std::string line;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        const size_t tab = line.find('\t');
        if (tab == std::string::npos || line.compare(0, tab, key) != 0 || tab != key.size()) continue;
        std::istringstream v(line.substr(tab + 1));
        TuneResult r{};
        if (v >> r.batch >> r.theta_fwd >> r.theta_bwd) {
            if (!(v >> r.fwd_rows)) r.fwd_rows = 0;
            out = r;
            found = true;
        }
    }
    return found;
}

void file_store(const char *path, const std::string &key, const TuneResult &r) {
    FILE *f = std::fopen(path, "a");
    if (!f) return; // an unwritable cache only costs a later calibration
    std::fprintf(f, "%s\t%d %.17g %.17g %d\n", key.c_str(), r.batch, r.theta_fwd, r.theta_bwd, r.fwd_rows);
    std::fclose(f);
}

// The caller's file comes first, then what this process measured before (a
// result measured here and missing from the file is appended to it).
bool cache_lookup(const bc_options &opt, const std::string &key, TuneResult &out) {
    if (opt.tune_cache && file_lookup(opt.tune_cache, key, out)) return true;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(key);
        if (it == g_cache.end()) return false;
        out = it->second;
    }
    if (opt.tune_cache) file_store(opt.tune_cache, key, out);
    return true;
}

void cache_store(const bc_options &opt, const std::string &key, const TuneResult &r, bool measured) {
    if (measured) {
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[key] = r;
    }
    if (opt.tune_cache) file_store(opt.tune_cache, key, r);
}

uint64_t fmix64(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    return x ^ (x >> 33);
}

size_t state_bytes(int32_t n, int32_t batch) {
    // counts (8 B) and coefficients (4 B) per (vertex, source), plus 16
    // levels of frontier bits
    return (size_t)n * batch * 12 + (size_t)16 * n * (batch / 8);
}

bool products_possible(const bc_ctx *ctx) {
    if (ctx->weighted || ctx->max_degree > BC_ALGEBRAIC_MAX_DEGREE) return false;
    const size_t npad = (size_t)std::max(256, (ctx->n + 255) / 256 * 256);
    return npad <= kHybridMaxNpad;
}

// The hybrid form in its every-level mode: every level l >= 1 by products and
// the end of search (thresholds read 0: every density reaches them).  Edge
// betweenness needs the per-arc pulls in the backward, so a context with
// edges keeps pulls at every level instead.
void set_every_level(bc_ctx *ctx) {
    if (ctx->edges) {
        ctx->hy.theta_fwd = ctx->hy.theta_bwd = kNever;
        return;
    }
    ctx->hy.theta_fwd = ctx->hy.theta_bwd = 0.0;
    ctx->al.every_level = true;
}

bc_status prepare_width(bc_ctx *ctx, int32_t batch, int32_t split, bool products) {
    bc_status st = sparse_prepare(ctx, batch, split);
    if (st == BC_OK && products) st = algebraic_prepare(ctx);
    return st;
}

bc_status release_width(bc_ctx *ctx, bool products) {
    bc_status st = sparse_release(ctx);
    if (st == BC_OK && products) st = algebraic_release(ctx);
    return st;
}

struct Sample {
    double density = 0.0, t_pull = 0.0, t_prod = 0.0;
    bool has_pull = false, has_prod = false;
};
using SampleKey = std::pair<int, std::pair<int, int>>; // (batch index, (forward, level))

struct Calibration {
    std::map<SampleKey, Sample> samples;
};

// Modes of a calibration run: per-level probes with every level by pulls or
// by products, or whole batches without probes, with the current thresholds
// or with pulls only.
enum { kProbePulls = 1, kProbeProducts = 2, kPlainMixed = 3, kPlainPulls = 4 };

// Runs batches [0, kReps] (batch 0 warms up) of the calibration sources;
// per-level times go into cal.samples and the device time per source of the
// timed batches into *ms_per_source.
bc_status run_mode(bc_ctx *ctx, const int32_t *d_src, int32_t B, int mode, Calibration &cal,
                   double *ms_per_source) {
    LevelProbe probe;
    probe.mode = mode == kProbeProducts ? 2 : 1;
    const bool products = ctx->hy.products;
    if (mode == kProbePulls || mode == kProbeProducts) ctx->hy.probe = &probe;
    if (mode == kPlainPulls) ctx->hy.products = false;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    bc_status st = BC_OK;
    std::vector<size_t> batch_end;
    if (!(t0 = bc_event_get(ctx)) || !(t1 = bc_event_get(ctx))) st = bc_fail(ctx, BC_ERR_DEVICE, "hipEventCreate failed");
    for (int j = 0; j <= kReps && st == BC_OK; ++j) {
        if (j == 1 && hipEventRecord(t0, ctx->stream) != hipSuccess) st = bc_fail(ctx, BC_ERR_DEVICE, "hipEventRecord failed");
        if (st == BC_OK) st = sparse_batch(ctx, d_src + (size_t)j * B, B, true);
        batch_end.push_back(probe.recs.size());
    }
    if (st == BC_OK && hipEventRecord(t1, ctx->stream) != hipSuccess) st = bc_fail(ctx, BC_ERR_DEVICE, "hipEventRecord failed");
    if (st == BC_OK && hipEventSynchronize(t1) != hipSuccess) st = bc_fail(ctx, BC_ERR_DEVICE, "calibration failed");
    if (st == BC_OK) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, t0, t1);
        *ms_per_source = (double)ms / ((double)kReps * B);
    }
    size_t j = 0;
    for (size_t i = 0; i < probe.recs.size(); ++i) {
        while (j < batch_end.size() && i >= batch_end[j]) ++j;
        const LevelProbe::Rec &r = probe.recs[i];
        if (st == BC_OK && j >= 1) { // batch 0 warms up
            float ms = 0.f;
            hipEventElapsedTime(&ms, r.a, r.b);
            Sample &smp = cal.samples[{(int)j, {r.forward ? 1 : 0, r.level}}];
            smp.density = r.density;
            if (mode == kProbePulls) {
                smp.t_pull = ms;
                smp.has_pull = true;
            } else {
                smp.t_prod = ms;
                smp.has_prod = true;
            }
        }
        bc_event_put(ctx, r.a);
        bc_event_put(ctx, r.b);
    }
    bc_event_put(ctx, t0);
    bc_event_put(ctx, t1);
    ctx->hy.probe = nullptr;
    ctx->hy.products = products;
    return st;
}

// Threshold for one direction minimising the summed level time of the
// samples; *saved_ms is the time it saves over all-pulls.  Ties keep pulls.
// A threshold strictly inside the range of one level's densities over the
// calibration batches is not a candidate: some batches would take that level
// by products and others by pulls, and a replayed batch, which keeps the plan
// of the batch it was recorded from, would run whichever that one took.
double fit_threshold(const Calibration &cal, bool forward, double *saved_ms) {
    std::vector<const Sample *> v;
    std::map<int, std::pair<double, double>> range; // level -> lowest, highest density
    for (const auto &kv : cal.samples)
        if ((kv.first.second.first == 1) == forward && kv.second.has_pull && kv.second.has_prod) {
            v.push_back(&kv.second);
            const double d = kv.second.density;
            auto it = range.find(kv.first.second.second);
            if (it == range.end()) range[kv.first.second.second] = {d, d};
            else it->second = {std::min(it->second.first, d), std::max(it->second.second, d)};
        }
    auto splits_a_level = [&](double theta) {
        for (const auto &kv : range)
            if (kv.second.first < theta && theta <= kv.second.second) return true;
        return false;
    };
    double all_pull = 0.0;
    for (const Sample *s : v) all_pull += s->t_pull;
    double best_theta = kNever, best = all_pull;
    for (const Sample *c : v) {
        const double theta = c->density;
        if (splits_a_level(theta)) continue;
        double cost = forward ? kSyncMs * (double)v.size() : 0.0;
        for (const Sample *s : v) cost += s->density >= theta ? s->t_prod : s->t_pull;
        if (cost < best || (cost == best && theta > best_theta && best_theta <= 1.0)) {
            best = cost;
            best_theta = theta;
        }
    }
    *saved_ms = all_pull - best;
    // The best candidate is the lowest density of some level's range; any
    // threshold between it and the next lower sampled density splits the
    // samples alike.  Take the middle of that gap (or half the density when
    // nothing lies below): batches outside the calibration sample spread
    // around the sampled densities, and one just below the candidate would
    // send the level to pulls, in a replayed run for every batch.
    if (best_theta <= 1.0) {
        double below = -1.0;
        for (const Sample *s : v)
            if (s->density < best_theta) below = std::max(below, s->density);
        best_theta = below >= 0.0 ? 0.5 * (below + best_theta) : 0.5 * best_theta;
    }
    return best_theta;
}

// Forward product block rows: whole batches, every level as the form runs it
// (the algebraic form: all by products; the hybrid form: by its thresholds),
// with 128- and 256-row blocks, timed alternately so that both see the same
// cache and clock state.  256 rows are kept only if they beat 128 by kAccept.
bc_status pick_fwd_rows(bc_ctx *ctx, const int32_t *d_src, int32_t B, int32_t *rows) {
    Calibration cal;
    double t128 = 0.0, t256 = 0.0;
    bc_status st = BC_OK;
    for (int rep = 0; rep < kConfirm && st == BC_OK; ++rep) {
        double a = 0.0, b = 0.0;
        ctx->al.fwd_rows = 128;
        st = run_mode(ctx, d_src, B, kPlainMixed, cal, &a);
        ctx->al.fwd_rows = 256;
        if (st == BC_OK) st = run_mode(ctx, d_src, B, kPlainMixed, cal, &b);
        t128 += a;
        t256 += b;
    }
    *rows = st == BC_OK && t256 < kAccept * t128 ? 256 : 128;
    ctx->al.fwd_rows = *rows;
    return st;
}

// Calibration sources: (kReps + 1) batches of `width`, drawn from the graph
// by a fixed hash so that every context of one shape times the same ones.
bc_status calibration_sources(bc_ctx *ctx, int32_t width, int32_t **out) {
    const size_t nsrc = (size_t)(kReps + 1) * width;
    std::vector<int32_t> h_src(nsrc);
    for (size_t i = 0; i < nsrc; ++i) h_src[i] = (int32_t)(fmix64(0x0809190600ull + i) % (uint64_t)ctx->n);
    int32_t *d_src = (int32_t *)bc_dalloc(ctx, nsrc * sizeof(int32_t));
    if (!d_src) return bc_fail(ctx, BC_ERR_NOMEM, "tuning: source buffer allocation failed");
    if (hipMemcpy(d_src, h_src.data(), nsrc * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
        bc_dfree(ctx, d_src);
        return bc_fail(ctx, BC_ERR_DEVICE, "tuning: source upload failed");
    }
    *out = d_src;
    return BC_OK;
}

// Calibration added to BC (and, with edges on, to the per-arc terms) and may
// have flagged an overflow: start clean.
bc_status clear_after_calibration(bc_ctx *ctx) {
    BC_HIP(ctx, hipMemsetAsync(ctx->bc, 0, sizeof(double) * (size_t)std::max(ctx->n, 1), ctx->stream));
    if (ctx->eb) BC_HIP(ctx, hipMemsetAsync(ctx->eb, 0, sizeof(double) * (size_t)std::max(ctx->nnz, 1), ctx->stream));
    BC_HIP(ctx, hipMemsetAsync(ctx->status, 0, 256, ctx->stream));
    BC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    bc_timers_clear(ctx);
    algebraic_reset_counters(ctx); // products and k-tiles count from create
    ctx->max_levels = 0;
    return BC_OK;
}

// The algebraic form: batch width from opt (default 256); the forward block
// rows from the cache or timed batches.
bc_status tune_algebraic(bc_ctx *ctx, const bc_options &opt) {
    const int32_t w = opt.batch ? opt.batch : 256;
    bc_status st = sparse_prepare(ctx, w, opt.split_degree);
    if (st == BC_OK) st = algebraic_prepare(ctx);
    ctx->al.every_level = true;
    if (st != BC_OK) return st;
    const std::string key = make_key(ctx, BC_FORM_ALGEBRAIC, opt.batch, opt.split_degree);
    TuneResult r{};
    if (cache_lookup(opt, key, r)) {
        if (r.batch != w || (r.fwd_rows != 0 && r.fwd_rows != 128 && r.fwd_rows != 256))
            return bc_fail(ctx, BC_ERR_INVALID_ARG, "tuning cache: entry for this graph names an unusable batch width or block rows");
        ctx->al.fwd_rows = r.fwd_rows ? r.fwd_rows : 128;
        ctx->hy.tune_source = BC_TUNE_CACHED;
        return BC_OK;
    }
    r = TuneResult{w, kNever, kNever, 128};
    if (ctx->n < kTinyN) { // calibration would time launch latency only
        ctx->hy.tune_source = BC_TUNE_DEFAULT;
        cache_store(opt, key, r, false);
        return BC_OK;
    }
    int32_t *d_src = nullptr;
    st = calibration_sources(ctx, w, &d_src);
    if (st != BC_OK) return st;
    st = pick_fwd_rows(ctx, d_src, w, &r.fwd_rows);
    bc_dfree(ctx, d_src);
    if (st == BC_OK) st = clear_after_calibration(ctx);
    if (st != BC_OK) return st;
    ctx->hy.tune_source = BC_TUNE_MEASURED;
    cache_store(opt, key, r, true);
    return BC_OK;
}

} // namespace

bc_status tune_prepare(bc_ctx *ctx, const bc_options &opt, bc_form form) {
    ctx->hy = HybridState{};
    if (form == BC_FORM_ALGEBRAIC) return tune_algebraic(ctx, opt);
    const bool hybrid = form == BC_FORM_HYBRID;
    const int32_t split = opt.split_degree;
    if (hybrid && opt.batch != 0 && opt.batch != 256 && opt.batch != 512)
        return bc_fail(ctx, BC_ERR_INVALID_ARG, "hybrid form: batch must be 0 (tuned), 256 or 512");
    const bool products = hybrid && products_possible(ctx);
    ctx->hy.products = products;
    if (!hybrid && opt.batch != 0) return sparse_prepare(ctx, opt.batch, split); // nothing to tune

    const std::string key = make_key(ctx, form, opt.batch, split);
    TuneResult r{};
    if (cache_lookup(opt, key, r)) {
        const bool ok_width = r.batch == 128 || r.batch == 256 || r.batch == 512 || (!hybrid && r.batch == 64);
        if (!ok_width || (hybrid && r.batch % 256 != 0) || (opt.batch != 0 && r.batch != opt.batch) ||
            (r.fwd_rows != 0 && r.fwd_rows != 128 && r.fwd_rows != 256))
            return bc_fail(ctx, BC_ERR_INVALID_ARG,
                           "tuning cache: entry for this graph names an unusable batch width or block rows");
        bc_status st = prepare_width(ctx, r.batch, split, products);
        if (st != BC_OK) return st;
        ctx->hy.theta_fwd = products ? r.theta_fwd : kNever;
        ctx->hy.theta_bwd = products ? r.theta_bwd : kNever;
        if (products && r.theta_fwd < 0.0) set_every_level(ctx);
        if (products) ctx->al.fwd_rows = r.fwd_rows ? r.fwd_rows : 128;
        ctx->hy.tune_source = BC_TUNE_CACHED;
        return BC_OK;
    }
    if (ctx->n < kTinyN) { // calibration would time launch latency only
        const int32_t w = opt.batch ? opt.batch : 256;
        bc_status st = prepare_width(ctx, w, split, products);
        ctx->hy.tune_source = BC_TUNE_DEFAULT;
        if (st == BC_OK) cache_store(opt, key, TuneResult{w, kNever, kNever, 128}, false);
        return st;
    }

    std::vector<int32_t> widths;
    if (opt.batch) widths.push_back(opt.batch);
    else if (hybrid) widths = {256, 512};
    else widths = {128, 256, 512};
    while (widths.size() > 1 && state_bytes(ctx->n, widths.back()) > kStateBudget) widths.pop_back();

    int32_t *d_src = nullptr;
    bc_status st = calibration_sources(ctx, widths.back(), &d_src);
    if (st != BC_OK) return st;

    double best_ms = 0.0;
    int32_t best_w = 0, prepared = 0, rows = 128;
    double best_tf = kNever, best_tb = kNever;
    for (int32_t w : widths) {
        if (prepared) st = release_width(ctx, products);
        if (st == BC_OK) st = prepare_width(ctx, w, split, products);
        if (st != BC_OK) break;
        prepared = w;
        Calibration cal;
        double ms = 0.0, unused = 0.0;
        st = run_mode(ctx, d_src, w, kPlainPulls, cal, &ms);
        if (st == BC_OK && products) st = run_mode(ctx, d_src, w, kProbePulls, cal, &unused);
        if (st == BC_OK && products) st = run_mode(ctx, d_src, w, kProbeProducts, cal, &unused);
        if (st != BC_OK) break;
        double tf = kNever, tb = kNever, saved = 0.0;
        if (products) {
            tf = fit_threshold(cal, true, &saved);
            tb = fit_threshold(cal, false, &saved);
        }
        if (tf <= 1.0 || tb <= 1.0) {
            // The per-level fit leaves out host round trips and launch gaps:
            // keep the mix only if whole batches with it beat pulls, timed
            // alternately so that both see the same cache and clock state.
            ctx->hy.theta_fwd = tf;
            ctx->hy.theta_bwd = tb;
            double mixed = 0.0, pulls = 0.0;
            for (int rep = 0; rep < kConfirm && st == BC_OK; ++rep) {
                double a = 0.0, b = 0.0;
                st = run_mode(ctx, d_src, w, kPlainMixed, cal, &a);
                if (st == BC_OK) st = run_mode(ctx, d_src, w, kPlainPulls, cal, &b);
                mixed += a;
                pulls += b;
            }
            if (st != BC_OK) break;
            if (mixed < kAccept * pulls) ms = mixed / kConfirm;
            else {
                tf = tb = kNever;
                ms = pulls / kConfirm;
            }
        }
        if (products && !ctx->edges) {
            // every level by products against the choice above, alternately
            double every = 0.0, chosen = 0.0;
            for (int rep = 0; rep < kConfirm && st == BC_OK; ++rep) {
                double a = 0.0, b = 0.0;
                ctx->al.every_level = true;
                st = run_mode(ctx, d_src, w, kPlainMixed, cal, &a);
                ctx->al.every_level = false;
                ctx->hy.theta_fwd = tf;
                ctx->hy.theta_bwd = tb;
                if (st == BC_OK) st = run_mode(ctx, d_src, w, tf <= 1.0 || tb <= 1.0 ? kPlainMixed : kPlainPulls, cal, &b);
                every += a;
                chosen += b;
            }
            if (st != BC_OK) break;
            if (every < kAccept * chosen) {
                tf = tb = kEvery;
                ms = every / kConfirm;
            }
        }
        if (best_w == 0 || ms < best_ms) {
            best_ms = ms;
            best_w = w;
            best_tf = tf;
            best_tb = tb;
        }
    }
    if (st == BC_OK && prepared != best_w) {
        st = release_width(ctx, products);
        if (st == BC_OK) st = prepare_width(ctx, best_w, split, products);
    }
    ctx->hy.theta_fwd = best_tf;
    ctx->hy.theta_bwd = best_tb;
    if (best_tf < 0.0) set_every_level(ctx);
    // forward products in use: their block rows too
    if (st == BC_OK && products && best_tf <= 1.0) st = pick_fwd_rows(ctx, d_src, best_w, &rows);
    bc_dfree(ctx, d_src);
    if (st == BC_OK) st = clear_after_calibration(ctx);
    if (st != BC_OK) return st;
    ctx->hy.tune_source = BC_TUNE_MEASURED;
    cache_store(opt, key, TuneResult{best_w, best_tf, best_tb, rows}, true);
    return BC_OK;
}

// bc_create_many's queue: sources per work unit from opt, the cache, or timed
// launches.  The calibration runs a sample of the graphs (every k-th by size,
// k chosen so that one launch takes about kManySampleWork of n_g (n_g +
// arcs_g)) once per unit size to warm up and record the launch, then kReps
// times timed; the fastest mean wins.  The compact sweep's workgroups per
// compute unit are fixed at two by its LDS (each takes just under half).
bc_status tune_many(bc_ctx *ctx, const bc_options &opt, const std::vector<int32_t> &voff,
                    const std::vector<int32_t> &rpoff, const std::vector<int32_t> &rp) {
    ctx->hy = HybridState{};
    bc_status st = multigraph_prepare(ctx, voff, rpoff, rp, opt.batch > 0 ? opt.batch : 64);
    if (st != BC_OK || opt.batch > 0) return st;
    MultiState &m = ctx->mg;
    const std::string key = make_many_key(ctx);
    TuneResult r{};
    if (cache_lookup(opt, key, r)) {
        if (r.batch < 1 || r.batch > 4096)
            return bc_fail(ctx, BC_ERR_INVALID_ARG, "tuning cache: entry for these graphs names an unusable unit size");
        ctx->hy.tune_source = BC_TUNE_CACHED;
        return r.batch == m.chunk ? BC_OK : multigraph_set_queue(ctx, nullptr, r.batch);
    }
    if (ctx->n < kTinyN) {
        ctx->hy.tune_source = BC_TUNE_DEFAULT;
        cache_store(opt, key, TuneResult{m.chunk, kNever, kNever, 0}, false);
        return BC_OK;
    }
    double total = 0.0;
    for (int32_t g = 0; g < m.ngraphs; ++g) {
        const double n = (double)(m.h_voff[(size_t)g + 1] - m.h_voff[(size_t)g]);
        total += n * (n + (double)m.h_arcs[(size_t)g]);
    }
    const size_t stride = (size_t)std::max(1.0, std::ceil(total / kManySampleWork));
    std::vector<int32_t> sample;
    for (size_t i = 0; i < m.h_order.size(); i += stride) sample.push_back(m.h_order[i]);

    hipEvent_t t0 = bc_event_get(ctx), t1 = bc_event_get(ctx);
    if (!t0 || !t1) st = bc_fail(ctx, BC_ERR_DEVICE, "hipEventCreate failed");
    int32_t best = m.chunk;
    double best_ms = 0.0;
    for (int32_t c : kUnitSizes) {
        if (st == BC_OK) st = multigraph_set_queue(ctx, &sample, c);
        if (st == BC_OK) st = multigraph_run(ctx); // records the launch
        if (st == BC_OK && hipEventRecord(t0, ctx->stream) != hipSuccess) st = bc_fail(ctx, BC_ERR_DEVICE, "hipEventRecord failed");
        for (int j = 0; j < kReps && st == BC_OK; ++j) st = multigraph_run(ctx);
        if (st == BC_OK && hipEventRecord(t1, ctx->stream) != hipSuccess) st = bc_fail(ctx, BC_ERR_DEVICE, "hipEventRecord failed");
        if (st == BC_OK && hipEventSynchronize(t1) != hipSuccess) st = bc_fail(ctx, BC_ERR_DEVICE, "calibration failed");
        if (st != BC_OK) break;
        float ms = 0.f;
        hipEventElapsedTime(&ms, t0, t1);
        if (best_ms == 0.0 || ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    bc_event_put(ctx, t0);
    bc_event_put(ctx, t1);
    if (st == BC_OK) st = multigraph_set_queue(ctx, nullptr, best);
    if (st == BC_OK) st = clear_after_calibration(ctx);
    if (st != BC_OK) return st;
    ctx->hy.tune_source = BC_TUNE_MEASURED;
    cache_store(opt, key, TuneResult{best, kNever, kNever, 0}, true);
    return BC_OK;
}
