// dms_batch.hip -- batched form: many scalar fields of uneven shapes
// (ensemble members or time steps) through order -> gradient -> critical
// simplices with one graph launch.
//
// All fields are concatenated.  The order is one radix sort on a composite
// key (field index above the float32 value key), so each field's ranks are
// its global positions minus the field's offset.  The gradient is one
// launch over the (field, tile) list, a block per tile; the extraction one
// pass over the records the gradient flagged in its critical mask.  The first run records these launches into a hipGraph on a
// private capture stream; later runs with the same arguments replay it on the
// caller's stream.  An autotuner picks the gradient tile shape per batch
// (timed on the first run, remembered in an optional cache file).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "dms_internal.hpp"

struct dms_batch {
    int nfields = 0;
    int dtype = 0;
    int tune = 0;
    int variant = 0;
    bool tuned = false;
    std::string cache;
    uint64_t signature = 0;
    std::vector<int64_t> dims;  // 3 per field
    std::vector<int64_t> off;   // nfields + 1
    int64_t total = 0;
    dms::BatchField *d_fields = nullptr;
    int64_t *d_off = nullptr;
    int64_t *d_tiles[dms::kGradVariants] = {nullptr, nullptr, nullptr};
    uint16_t *d_tile_field[dms::kGradVariants] = {nullptr, nullptr, nullptr};  // field of each tile
    int64_t tiles[dms::kGradVariants] = {0, 0, 0};
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const void *> args;  // pointer/capacity signature of the captured graph
};

namespace {

uint64_t fnv1a(const int64_t *v, size_t n)
{
    uint64_t h = 1469598103934665603ull;
    const unsigned char *p = (const unsigned char *)v;
    for (size_t i = 0; i < n * sizeof(int64_t); ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

int cache_lookup(const std::string &path, uint64_t sig)
{
    if (path.empty()) return -1;
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return -1;
    char arch[64];
    unsigned long long s;
    int v, found = -1;
    while (std::fscanf(f, "%63s %llx %d", arch, &s, &v) == 3)
        if (std::strcmp(arch, "gfx950") == 0 && s == sig && v >= 0 && v < dms::kGradVariants) found = v;
    std::fclose(f);
    return found;
}

void cache_store(const std::string &path, uint64_t sig, int variant)
{
    if (path.empty()) return;
    FILE *f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "gfx950 %llx %d\n", (unsigned long long)sig, variant);
    std::fclose(f);
}

struct Ws {
    char *order, *crit, *grad;
    uint32_t *mask;  // the critical mask: a bit per record
};

size_t mask_bytes(int64_t total) { return dms::align_up((size_t)((total + 31) / 32) * 4, 256); }

Ws carve(const dms_batch *b, void *ws)
{
    Ws w;
    w.order = (char *)ws;
    w.crit = w.order + dms::align_up(dms::order_batch_workspace_size(b->total), 256);
    w.mask = (uint32_t *)(w.crit + dms::align_up(dms::critical_batch_workspace_size(b->total, b->nfields), 256));
    w.grad = (char *)w.mask + mask_bytes(b->total);
    return w;
}

void destroy_graph(dms_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

int enqueue_all(dms_batch *b, const void *values, int32_t *order, uint32_t *rec, int64_t *const crit[4],
                const int64_t cap[4], int64_t *counts, int64_t *offsets, void *ws, uint32_t *flags,
                hipStream_t s)
{
    const Ws w = carve(b, ws);
    int st = dms::launch_order_batch((const float *)values, b->total, b->d_off, b->nfields, order,
                                     w.order, flags, s);
    if (st) return st;
    st = dms::launch_gradient_batch(b->variant, order, b->d_fields, b->nfields, b->d_tiles[b->variant],
                                    b->d_tile_field[b->variant], b->tiles[b->variant], b->total, rec,
                                    w.mask, w.grad, s);
    if (st) return st;
    return dms::launch_critical_batch(rec, w.mask, b->total, b->d_off, b->nfields, b->d_fields, crit, cap,
                                      counts, offsets, w.crit, flags, s);
}

// Times each tile shape on the caller's data (the order must be ready).
int autotune(dms_batch *b, const int32_t *order, uint32_t *rec, const Ws &w, hipStream_t s)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return DMS_E_HIP;
    float best = 1e30f;
    int best_v = 0;
    for (int v = 0; v < dms::kGradVariants; ++v) {
        float t = 0.f;
        for (int rep = 0; rep < 2; ++rep) {
            (void)hipEventRecord(e0, s);
            int st = dms::launch_gradient_batch(v, order, b->d_fields, b->nfields, b->d_tiles[v],
                                                b->d_tile_field[v], b->tiles[v],
                                                b->total, rec, w.mask, w.grad, s);
            (void)hipEventRecord(e1, s);
            if (st) return st;
            if (hipEventSynchronize(e1) != hipSuccess) return DMS_E_HIP;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            t = rep == 0 ? ms : (ms < t ? ms : t);
        }
        if (t < best) { best = t; best_v = v; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->variant = best_v;
    cache_store(b->cache, b->signature, best_v);
    return DMS_OK;
}

}  // namespace

extern "C" int dms_batch_create(const int64_t *dims, int nfields, int dtype, int tune,
                                const char *tune_cache, dms_batch **out)
{
    if (!out) return DMS_E_ARG;
    *out = nullptr;
    if (!dims || nfields < 1) return DMS_E_ARG;
    if (nfields > dms::kMaxBatchFields) return DMS_E_SIZE;
    if (dtype != DMS_F32) return DMS_E_UNSUPPORTED;
    dms_batch *b = new dms_batch();
    b->nfields = nfields;
    b->dtype = dtype;
    b->tune = tune;
    b->cache = tune_cache ? tune_cache : "";
    b->dims.assign(dims, dims + 3 * nfields);
    b->off.assign(nfields + 1, 0);
    std::vector<dms::BatchField> hf(nfields);
    for (int f = 0; f < nfields; ++f) {
        const int64_t *d = dims + 3 * f;
        if (d[0] < 1 || d[1] < 1 || d[2] < 1 || !dms::grid_size_ok(d)) {
            delete b;
            return d[0] < 1 || d[1] < 1 || d[2] < 1 ? DMS_E_ARG : DMS_E_SIZE;
        }
        b->off[f + 1] = b->off[f] + d[0] * d[1] * d[2];
        hf[f] = {{d[0], d[1], d[2]}, b->off[f]};
    }
    b->total = b->off[nfields];
    if (b->total > 2147483647LL) {
        delete b;
        return DMS_E_SIZE;
    }
    if (const int dc = dms::device_check()) {
        delete b;
        return dc;
    }
    b->signature = fnv1a(dims, 3 * (size_t)nfields);
    std::vector<int64_t> ts(nfields + 1);
    bool ok = hipMalloc(&b->d_fields, sizeof(dms::BatchField) * nfields) == hipSuccess &&
              hipMalloc(&b->d_off, sizeof(int64_t) * (nfields + 1)) == hipSuccess &&
              hipMemcpy(b->d_fields, hf.data(), sizeof(dms::BatchField) * nfields, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(b->d_off, b->off.data(), sizeof(int64_t) * (nfields + 1), hipMemcpyHostToDevice) == hipSuccess;
    for (int v = 0; ok && v < dms::kGradVariants; ++v) {
        const int gx = dms::kTileX[v], gy = dms::kTileVertsPerBlock / gx;
        ts[0] = 0;
        for (int f = 0; f < nfields; ++f) {
            const int64_t *d = dims + 3 * f;
            ts[f + 1] = ts[f] + ((d[0] + gx - 1) / gx) * ((d[1] + gy - 1) / gy) * d[2];
        }
        b->tiles[v] = ts[nfields];
        std::vector<uint16_t> tf((size_t)(ts[nfields] > 0 ? ts[nfields] : 1));
        for (int f = 0; f < nfields; ++f)
            for (int64_t t = ts[f]; t < ts[f + 1]; ++t) tf[(size_t)t] = (uint16_t)f;
        ok = hipMalloc(&b->d_tiles[v], sizeof(int64_t) * (nfields + 1)) == hipSuccess &&
             hipMemcpy(b->d_tiles[v], ts.data(), sizeof(int64_t) * (nfields + 1), hipMemcpyHostToDevice) == hipSuccess &&
             hipMalloc(&b->d_tile_field[v], sizeof(uint16_t) * tf.size()) == hipSuccess &&
             hipMemcpy(b->d_tile_field[v], tf.data(), sizeof(uint16_t) * tf.size(), hipMemcpyHostToDevice) == hipSuccess;
    }
    ok = ok && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) == hipSuccess &&
         dms::init_tables(b->cap_stream) == DMS_OK;
    if (!ok) {
        dms_batch_destroy(b);
        return DMS_E_HIP;
    }
    const int cached = cache_lookup(b->cache, b->signature);
    if (cached >= 0) {
        b->variant = cached;
        b->tuned = true;
    } else if (!tune) {
        b->tuned = true;  // fixed default shape
    }
    *out = b;
    return DMS_OK;
}

extern "C" size_t dms_batch_workspace_size(const dms_batch *b)
{
    if (!b) return 0;
    return dms::align_up(dms::order_batch_workspace_size(b->total), 256) +
           dms::align_up(dms::critical_batch_workspace_size(b->total, b->nfields), 256) + mask_bytes(b->total) +
           dms::gradient_workspace_size(b->total);
}

extern "C" int64_t dms_batch_total(const dms_batch *b) { return b ? b->total : -1; }

extern "C" int dms_batch_variant(const dms_batch *b) { return b ? b->variant : -1; }

extern "C" int dms_batch_run(dms_batch *b, const void *values, int32_t *order, uint32_t *rec,
                             int64_t *crit0, int64_t *crit1, int64_t *crit2, int64_t *crit3,
                             const int64_t cap[4], int64_t *counts, int64_t *offsets, void *ws,
                             size_t ws_bytes, uint32_t *dev_flags, void *stream)
{
    if (!b || !values || !order || !rec || !cap || !counts || !offsets || !dev_flags) return DMS_E_ARG;
    int64_t *crit[4] = {crit0, crit1, crit2, crit3};
    for (int d = 0; d < 4; ++d)
        if (cap[d] < 0 || (cap[d] > 0 && !crit[d])) return DMS_E_ARG;
    if (!ws || ws_bytes < dms_batch_workspace_size(b)) return DMS_E_WORKSPACE;
    if (const int dc = dms::device_check()) return dc;
    hipStream_t s = (hipStream_t)stream;
    if (!b->tuned) {
        // tuning pass, outside the graph: order once, then time every tile shape
        const Ws w = carve(b, ws);
        int st = dms::launch_order_batch((const float *)values, b->total, b->d_off, b->nfields, order,
                                         w.order, dev_flags, s);
        if (st) return st;
        st = autotune(b, order, rec, w, s);
        if (st) return st;
        b->tuned = true;
        destroy_graph(b);
    }
    std::vector<const void *> sig = {values, order, rec, crit0, crit1, crit2, crit3, counts, offsets,
                                     ws, dev_flags};
    for (int d = 0; d < 4; ++d) sig.push_back((const void *)(intptr_t)cap[d]);
    if (!b->exec || sig != b->args) {
        destroy_graph(b);
        if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) return DMS_E_HIP;
        const int st = enqueue_all(b, values, order, rec, crit, cap, counts, offsets, ws, dev_flags,
                                   b->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
        if (st || e != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return st ? st : DMS_E_HIP;
        }
        b->graph = g;
        if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
            destroy_graph(b);
            return DMS_E_HIP;
        }
        b->args = sig;
    }
    return hipGraphLaunch(b->exec, s) == hipSuccess ? DMS_OK : DMS_E_HIP;
}

extern "C" void dms_batch_destroy(dms_batch *b)
{
    if (!b) return;
    destroy_graph(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    (void)hipFree(b->d_fields);
    (void)hipFree(b->d_off);
    for (int v = 0; v < dms::kGradVariants; ++v) {
        (void)hipFree(b->d_tiles[v]);
        (void)hipFree(b->d_tile_field[v]);
    }
    delete b;
}
