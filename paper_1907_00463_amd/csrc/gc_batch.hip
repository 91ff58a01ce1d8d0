// gc_batch.hip -- batches of receivers behind the C ABI: one persistent
// launch over every (receiver, tile) work item, captured into a HIP graph,
// with the block shape and grid picked by timing the candidates on the
// bound batch.
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "gc_internal.h"
#include "gc_device.h"

using gc::DeviceGuard;
using gc::from_hip;

struct gc_batch {
    gc_ctx* ctx;
    int n_rx, n_chan, max_taps;
    uint32_t max_dumps;
    std::vector<gc_rx_desc> rx;
    std::vector<int32_t> chan_begin, chan_end;
    gc::DevChan* d_chans;
    gc::DevMeta* d_meta;
    gc::DevRx* d_rx;
    gc_chan_state* state;
    void* out;
    uint32_t* dump_n;
    uint32_t* n_dumps;
    int32_t* status;
    int shape, grid;           // current configuration of the chip-by-chip kernel
    uint32_t n_items;
    int pchunk;                // tiles per item of the periodic kernel (0: kernel off)
    gc::PbinItem* d_pitems;
    uint32_t n_pitems, max_pitems;
    uint32_t* d_order;         // chip-by-chip items with work (written on the device)
    uint32_t* d_count;         // their number, then the periodic kernel's queue counter
    int cus;
    float tuned_ms;
    hipStream_t cap;           // private stream for graph capture
    hipGraph_t graph;
    hipGraphExec_t exec;
    bool have_graph;
};

namespace {

// Receiver table for a shape: work items are the receivers' tiles, in order.
hipError_t upload_rx(gc_batch* b, int shape) {
    const uint32_t tile = gc::epl_batch_tile(shape);
    std::vector<gc::DevRx> h((size_t)b->n_rx);
    uint32_t items = 0;
    for (int r = 0; r < b->n_rx; ++r) {
        gc::DevRx& d = h[(size_t)r];
        d.samples = (const uint8_t*)b->rx[(size_t)r].samples;
        d.n = b->rx[(size_t)r].n_samples;
        d.fmt = b->rx[(size_t)r].fmt;
        d.chan_begin = b->chan_begin[(size_t)r];
        d.chan_end = b->chan_end[(size_t)r];
        d.tile_begin = items;
        items += (uint32_t)((d.n + tile - 1) / tile);
    }
    b->n_items = items;
    return hipMemcpy(b->d_rx, h.data(), sizeof(gc::DevRx) * h.size(), hipMemcpyHostToDevice);
}

constexpr int kChunkDefault = 4;
constexpr int kChunkCandidates[] = {2, 4, 8};
constexpr int kChunkMin = 2;

uint32_t tiles(uint64_t n, uint32_t tile) { return (uint32_t)((n + tile - 1) / tile); }

// Work items of the periodic kernel: per receiver, groups of at most kGroup
// channels times chunks of `chunk` tiles.
constexpr int kGroup = 16;
// the periodic kernel takes real input only (complex receivers get no items)
bool periodic_format(int fmt) { return fmt == GC_I8_REAL || fmt == GC_I2_REAL; }
uint32_t count_pitems(const gc_batch* b, int chunk) {
    const uint32_t tile = (uint32_t)gc::pbin_tile_samples();
    uint64_t k = 0;
    for (int r = 0; r < b->n_rx; ++r) {
        const int nc = b->chan_end[(size_t)r] - b->chan_begin[(size_t)r];
        if (nc <= 0 || !periodic_format(b->rx[(size_t)r].fmt)) continue;
        k += (uint64_t)((nc + kGroup - 1) / kGroup) *
             ((tiles(b->rx[(size_t)r].n_samples, tile) + chunk - 1) / chunk);
    }
    return (uint32_t)k;
}

hipError_t upload_pitems(gc_batch* b, int chunk) {
    b->n_pitems = 0;
    if (chunk <= 0) return hipSuccess;
    const uint32_t tile = (uint32_t)gc::pbin_tile_samples();
    std::vector<gc::PbinItem> h;
    h.reserve(count_pitems(b, chunk));
    for (int r = 0; r < b->n_rx; ++r) {
        if (!periodic_format(b->rx[(size_t)r].fmt)) continue;
        const int cb = b->chan_begin[(size_t)r], nc = b->chan_end[(size_t)r] - cb;
        const uint32_t nt = tiles(b->rx[(size_t)r].n_samples, tile);
        for (int first = 0; first < nc; first += kGroup)
            for (uint32_t t = 0; t < nt; t += (uint32_t)chunk)
                h.push_back(gc::PbinItem{r, cb + first, std::min(kGroup, nc - first), t,
                                         std::min(nt, t + (uint32_t)chunk)});
    }
    // the queue hands out larger items (more channels, more tiles) first, so
    // that the last items to finish are small ones
    std::stable_sort(h.begin(), h.end(), [](const gc::PbinItem& a, const gc::PbinItem& c) {
        return (uint64_t)a.n_chan * (a.tile_end - a.tile_begin) >
               (uint64_t)c.n_chan * (c.tile_end - c.tile_begin);
    });
    if (h.size() > b->max_pitems) return hipErrorInvalidValue;
    b->n_pitems = (uint32_t)h.size();
    if (h.empty()) return hipSuccess;
    return hipMemcpy(b->d_pitems, h.data(), sizeof(gc::PbinItem) * h.size(),
                     hipMemcpyHostToDevice);
}

hipError_t enqueue(gc_batch* b, hipStream_t s) {
    const int32_t allow = gc::kAllowBinned | (b->pchunk > 0 ? gc::kAllowPeriodic : 0);
    // with the periodic kernel on, the chip-by-chip kernel runs only the
    // tiles of receivers that still have work, selected on the device by one
    // more block of the set-up's row kernel (which also zeroes the periodic
    // kernel's item queue)
    const bool sel = b->pchunk > 0;
    gc::SelectArgs sa;
    sa.rx = b->d_rx;
    sa.n_rx = b->n_rx;
    sa.n_chan = b->n_chan;
    sa.n_items = b->n_items;
    sa.order = b->d_order;
    sa.count = b->d_count;
    sa.queue = b->d_count + 1;
    hipError_t e = gc::launch_setup(b->d_chans, b->d_meta, b->state, b->n_chan, 0, GC_I8_REAL,
                                    GC_CARRIER_LUT, b->max_dumps, b->out, b->max_taps, b->dump_n,
                                    b->n_dumps, b->status, allow, b->d_rx, nullptr, nullptr, s,
                                    sel ? &sa : nullptr);
    if (e == hipSuccess && b->pchunk > 0)
        e = gc::launch_pbin_batch(b->cus, b->d_rx, b->d_pitems, b->n_pitems, b->d_count + 1,
                                  b->d_chans, b->d_meta, b->state, (int32_t*)b->out,
                                  b->max_taps, b->max_dumps, b->ctx->d_tables, s);
    if (e == hipSuccess)
        e = gc::launch_epl_batch(b->shape, b->grid > 0 ? b->grid : b->cus, b->d_rx, b->n_rx,
                                 sel ? b->d_order : nullptr, b->n_items,
                                 sel ? b->d_count : nullptr, b->d_chans, b->d_meta, b->state,
                                 (int32_t*)b->out, b->max_taps, b->max_dumps, b->ctx->d_tables,
                                 s);
    return e;
}

void drop_graph(gc_batch* b) {
    if (b->have_graph) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->have_graph = false;
    }
}

}  // namespace

extern "C" {

gc_status gc_batch_create(gc_ctx* ctx, const gc_rx_desc* rx, int32_t n_rx,
                          const gc_chan_cfg* cfg, const int32_t* chan_rx, int32_t n_chan,
                          gc_chan_state* state, void* out, uint32_t* dump_n,
                          uint32_t* n_dumps, int32_t* status, uint32_t max_dumps,
                          gc_batch** out_batch) {
    if (!ctx || !rx || !cfg || !chan_rx || !state || !out || !dump_n || !n_dumps || !status ||
        !out_batch)
        return GC_EINVAL;
    *out_batch = nullptr;
    if (n_rx < 1 || n_rx > 65536 || n_chan < 1 || n_chan > GC_MAX_CHANNELS || max_dumps == 0)
        return GC_EINVAL;
    for (int r = 0; r < n_rx; ++r) {
        const gc_rx_desc& d = rx[r];
        if ((d.fmt != GC_I8_REAL && d.fmt != GC_I8_IQ && d.fmt != GC_I2_REAL && d.fmt != GC_I2_IQ) ||
            d.reserved != 0 ||
            d.n_samples >= (1ull << 31) || (d.n_samples > 0 && !d.samples))
            return GC_EINVAL;
    }
    std::vector<gc::DevChan> h((size_t)n_chan);
    std::vector<int32_t> cb((size_t)n_rx, 0), ce((size_t)n_rx, 0);
    int max_taps = 0;
    for (int i = 0; i < n_chan; ++i) {
        const gc_status st = gc::fill_devchan(cfg[i], h[(size_t)i]);
        if (st != GC_OK) return st;
        if (cfg[i].n_taps > 4) return GC_EINVAL;
        const int r = chan_rx[i];
        if (r < 0 || r >= n_rx || (i > 0 && r < chan_rx[i - 1])) return GC_EINVAL;
        h[(size_t)i].rx = r;
        if (i == 0 || r != chan_rx[i - 1]) cb[(size_t)r] = i;
        ce[(size_t)r] = i + 1;
        if (cfg[i].n_taps > max_taps) max_taps = cfg[i].n_taps;
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return GC_EDEVICE;
    gc_batch* b = new (std::nothrow) gc_batch();
    if (!b) return GC_ENOMEM;
    b->ctx = ctx;
    b->n_rx = n_rx;
    b->n_chan = n_chan;
    b->max_taps = max_taps;
    b->max_dumps = max_dumps;
    b->rx.assign(rx, rx + n_rx);
    b->chan_begin = cb;
    b->chan_end = ce;
    b->d_chans = nullptr;
    b->d_meta = nullptr;
    b->d_rx = nullptr;
    b->state = state;
    b->out = out;
    b->dump_n = dump_n;
    b->n_dumps = n_dumps;
    b->status = status;
    b->shape = 0;
    b->grid = 0;
    b->cus = gc::epl_blocks_per_device(ctx->device);
    b->tuned_ms = 0.0f;
    b->cap = nullptr;
    b->have_graph = false;
    b->pchunk = kChunkDefault;
    b->d_pitems = nullptr;
    b->n_pitems = 0;
    b->max_pitems = count_pitems(b, kChunkMin);
    b->d_order = nullptr;
    b->d_count = nullptr;
    uint64_t max_items = 1;   // chip-by-chip items of the shape with the smallest tile
    for (int sh = 0; sh < gc::epl_batch_shapes(); ++sh) {
        uint64_t k = 0;
        for (int r = 0; r < n_rx; ++r) k += tiles(rx[r].n_samples, gc::epl_batch_tile(sh));
        max_items = std::max(max_items, k);
    }
    hipError_t e = hipMalloc(&b->d_chans, sizeof(gc::DevChan) * (size_t)n_chan);
    if (e == hipSuccess) e = hipMalloc(&b->d_meta, sizeof(gc::DevMeta) * (size_t)n_chan);
    if (e == hipSuccess) e = hipMalloc(&b->d_rx, sizeof(gc::DevRx) * (size_t)n_rx);
    if (e == hipSuccess)
        e = hipMalloc(&b->d_pitems, sizeof(gc::PbinItem) * (size_t)std::max(1u, b->max_pitems));
    if (e == hipSuccess) e = hipMalloc(&b->d_order, sizeof(uint32_t) * (size_t)max_items);
    if (e == hipSuccess) e = hipMalloc(&b->d_count, 2 * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMemcpy(b->d_chans, h.data(), sizeof(gc::DevChan) * (size_t)n_chan,
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) e = upload_rx(b, 0);
    if (e == hipSuccess) e = upload_pitems(b, b->pchunk);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        if (b->d_chans) (void)hipFree(b->d_chans);
        if (b->d_meta) (void)hipFree(b->d_meta);
        if (b->d_rx) (void)hipFree(b->d_rx);
        if (b->d_pitems) (void)hipFree(b->d_pitems);
        if (b->d_order) (void)hipFree(b->d_order);
        if (b->d_count) (void)hipFree(b->d_count);
        if (b->cap) (void)hipStreamDestroy(b->cap);
        delete b;
        return from_hip(e);
    }
    *out_batch = b;
    return GC_OK;
}

gc_status gc_batch_configure(gc_batch* b, int32_t shape, int32_t grid, int32_t periodic_chunk) {
    if (!b || shape < 0 || shape >= gc::epl_batch_shapes() || grid < 0 || grid > 65536 ||
        periodic_chunk < -1 || periodic_chunk > 65536)
        return GC_EINVAL;
    DeviceGuard g(b->ctx->device);
    if (!g.ok) return GC_EDEVICE;
    (void)hipDeviceSynchronize();
    drop_graph(b);
    b->shape = shape;
    b->grid = grid;
    const int chunk = periodic_chunk == 0 ? kChunkDefault
                                          : (periodic_chunk < 0 ? 0 : std::max(kChunkMin, (int)periodic_chunk));
    b->pchunk = chunk;
    hipError_t e = upload_rx(b, shape);
    if (e == hipSuccess) e = upload_pitems(b, chunk);
    return from_hip(e);
}

gc_status gc_batch_tune(gc_batch* b, int32_t reps) {
    if (!b || reps < 1 || reps > 100) return GC_EINVAL;
    DeviceGuard g(b->ctx->device);
    if (!g.ok) return GC_EDEVICE;
    (void)hipDeviceSynchronize();
    drop_graph(b);
    const size_t sbytes = sizeof(gc_chan_state) * (size_t)b->n_chan;
    gc_chan_state* snap = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&snap, sbytes);
    if (e == hipSuccess) e = hipMemcpyAsync(snap, b->state, sbytes, hipMemcpyDeviceToDevice, b->cap);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&e0, hipEventDisableSystemFence);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&e1, hipEventDisableSystemFence);
    // mean time of `reps` launches of the current configuration (after one
    // warm-up), the bound states restored before each
    auto time_config = [&](float* mean) {
        float total = 0.0f;
        for (int r = 0; e == hipSuccess && r <= reps; ++r) {
            e = hipMemcpyAsync(b->state, snap, sbytes, hipMemcpyDeviceToDevice, b->cap);
            if (e == hipSuccess) e = hipEventRecord(e0, b->cap);
            if (e == hipSuccess) e = enqueue(b, b->cap);
            if (e == hipSuccess) e = hipEventRecord(e1, b->cap);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (r > 0) total += ms;
        }
        *mean = total / (float)reps;
    };
    // the two kernels run one after the other: tune the chip-by-chip
    // kernel's shape and grid first, then the periodic kernel's chunk
    const int keep_chunk = b->pchunk;
    int best_shape = b->shape, best_grid = b->grid, best_chunk = keep_chunk;
    float best = -1.0f;
    for (int sh = 0; e == hipSuccess && sh < gc::epl_batch_shapes(); ++sh) {
        e = upload_rx(b, sh);
        for (int gm = 1; e == hipSuccess && gm <= 2; ++gm) {
            b->shape = sh;
            b->grid = gm * b->cus;
            float mean = 0.0f;
            time_config(&mean);
            if (e == hipSuccess && (best < 0.0f || mean < best)) {
                best = mean;
                best_shape = sh;
                best_grid = b->grid;
            }
        }
    }
    b->shape = best_shape;
    b->grid = best_grid;
    if (e == hipSuccess) e = upload_rx(b, best_shape);
    if (keep_chunk > 0) {
        for (int chunk : kChunkCandidates) {
            if (e != hipSuccess) break;
            b->pchunk = chunk;
            e = upload_pitems(b, chunk);
            float mean = 0.0f;
            time_config(&mean);
            if (e == hipSuccess && mean < best) {
                best = mean;
                best_chunk = chunk;
            }
        }
    }
    if (snap) {
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->state, snap, sbytes, hipMemcpyDeviceToDevice, b->cap);
        (void)hipStreamSynchronize(b->cap);
        (void)hipFree(snap);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    b->shape = best_shape;
    b->grid = best_grid;
    b->pchunk = best_chunk;
    hipError_t e2 = upload_rx(b, best_shape);
    if (e2 == hipSuccess) e2 = upload_pitems(b, best_chunk);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) b->tuned_ms = best;
    return from_hip(e);
}

gc_status gc_batch_launch(gc_batch* b, void* stream) {
    if (!b) return GC_EINVAL;
    DeviceGuard g(b->ctx->device);
    if (!g.ok) return GC_EDEVICE;
    hipError_t e = hipSuccess;
    if (!b->have_graph) {
        // capture on the private stream (the caller's may be the null
        // stream), then replay on the caller's
        e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t el = enqueue(b, b->cap);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(b->cap, &graph);
            if (el != hipSuccess) e = el;
            if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
            if (e == hipSuccess) {
                b->graph = graph;
                b->have_graph = true;
            } else if (graph) {
                (void)hipGraphDestroy(graph);
            }
        }
    }
    if (e == hipSuccess) e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    return from_hip(e);
}

gc_status gc_batch_info(const gc_batch* b, int32_t* shape, int32_t* grid, int32_t* n_items,
                        int32_t* n_shapes, float* tuned_ms, int32_t* periodic_chunk,
                        int32_t* periodic_items) {
    if (!b) return GC_EINVAL;
    if (periodic_chunk) *periodic_chunk = b->pchunk > 0 ? b->pchunk : -1;
    if (periodic_items) *periodic_items = (int32_t)b->n_pitems;
    if (shape) *shape = b->shape;
    if (grid) *grid = b->grid > 0 ? b->grid : b->cus;
    if (n_items) *n_items = (int32_t)b->n_items;
    if (n_shapes) *n_shapes = gc::epl_batch_shapes();
    if (tuned_ms) *tuned_ms = b->tuned_ms;
    return GC_OK;
}

gc_status gc_batch_destroy(gc_batch* b) {
    if (!b) return GC_EINVAL;
    DeviceGuard g(b->ctx->device);
    (void)hipDeviceSynchronize();
    drop_graph(b);
    (void)hipFree(b->d_pitems);
    (void)hipFree(b->d_order);
    (void)hipFree(b->d_count);
    (void)hipFree(b->d_chans);
    (void)hipFree(b->d_meta);
    (void)hipFree(b->d_rx);
    (void)hipStreamDestroy(b->cap);
    delete b;
    return GC_OK;
}

}  // extern "C"
