// gc_server.hip -- serving loop behind the C ABI.
//
// Receivers are registered once; their channels live in server-wide device
// arrays (configuration, resident NCO state, output rows).  A request is one
// block of samples for one receiver: gc_server_submit admits it when its
// samples fit the device arena (the HBM budget) and the pinned host arena,
// copies the samples to pinned memory and starts their upload.  A
// dispatcher thread keeps up to n_streams launches in flight: each takes
// the oldest request of every idle receiver (a receiver's requests run in
// order, since each continues the NCO state of the one before) and runs
// them together -- set-up over their channels, one persistent launch of the
// batched chip-by-chip kernel, and the copies of the results to pinned host
// memory -- so requests that arrive while others are on the GPU join the
// next launch as streams and memory free up.  With GC_SERVER_PLAIN every
// request runs alone, one direct-kernel launch per channel (the baseline).
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gc_internal.h"
#include "gc_device.h"

using gc::DeviceGuard;
using gc::from_hip;

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kTapStride = 4;

// First-fit allocator over [0, size) in 256-byte units.
struct Arena {
    uint64_t size = 0;
    std::map<uint64_t, uint64_t> free_;  // offset -> length
    void init(uint64_t n) {
        size = n;
        free_.clear();
        if (n) free_[0] = n;
    }
    static uint64_t round(uint64_t n) { return (n + 255) & ~uint64_t(255); }
    bool alloc(uint64_t n, uint64_t* off) {
        n = round(n ? n : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const uint64_t rest = it->second - n, at = it->first + n;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t n) {
        n = round(n ? n : 1);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t in_use() const {
        uint64_t f = 0;
        for (auto& kv : free_) f += kv.second;
        return size - f;
    }
};

struct SrvRx {
    int fmt;
    int n_chan;
    int cb;                        // first channel in the server arrays
    std::deque<uint64_t> pending;  // request ids in submission order
    bool busy = false;             // its oldest request is on the device
};

struct SrvReq {
    int rx;
    uint64_t n;
    uint64_t dev_off, dev_bytes;   // samples in the device arena
    uint64_t host_off, host_bytes; // staging + results in the pinned arena
    hipEvent_t uploaded;
    int state;                     // 0 uploading/queued, 1 on the device, 2 done
    Clock::time_point t_submit, t_done;
};

// Where one request's results go: its channels in the server arrays and
// its result area in the pinned host arena (device-visible pointers).
struct ExportDesc {
    int32_t cb, n_chan;
    int32_t* out;
    uint32_t* dump_n;
    uint32_t* n_dumps;
    int32_t* status;
};

// A launch's tables, laid out the same in pinned host memory (written by
// the dispatcher) and in device memory (copied there by a kernel at the
// start of the launch): the compact receiver table, the channel list, each
// listed channel's receiver index, the export descriptors.
struct LaunchLayout {
    size_t off_rx, off_list, off_lrx, off_exp, bytes;
    void init(int max_rx, int cap_chan) {
        auto up16 = [](size_t v) { return (v + 15) & ~size_t(15); };
        off_rx = 0;
        off_list = up16(off_rx + sizeof(gc::DevRx) * (size_t)max_rx);
        off_lrx = up16(off_list + sizeof(int32_t) * (size_t)cap_chan);
        off_exp = up16(off_lrx + sizeof(int32_t) * (size_t)cap_chan);
        bytes = up16(off_exp + sizeof(ExportDesc) * (size_t)max_rx);
    }
};

struct SrvSlot {
    hipStream_t s = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<uint64_t> reqs;
    uint8_t* h_tab = nullptr;      // pinned launch tables (host view)
    uint8_t* h_tab_dev = nullptr;  // the same memory, device view
    uint8_t* d_tab = nullptr;      // device copy
    Clock::time_point t_enq;       // end of the current launch's enqueue
};

// n bytes from src to dst (16-byte aligned starts; either side may be
// pinned host memory seen from the device): 16-byte moves, then the tail.
__global__ __launch_bounds__(256) void k_copy(uint8_t* __restrict__ dst,
                                              const uint8_t* __restrict__ src, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t n16 = n / 16;
    for (uint64_t i = t; i < n16; i += stride)
        reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(src)[i];
    for (uint64_t i = n16 * 16 + t; i < n; i += stride) dst[i] = src[i];
}

// The used parts of a launch's tables: range blockIdx.y of (offset,
// length) pairs, both multiples of 16 bytes, from pinned host memory to the
// device copy.
struct Ranges {
    uint32_t off[4], len[4];
};
__global__ __launch_bounds__(256) void k_copy_ranges(uint8_t* __restrict__ dst,
                                                     const uint8_t* __restrict__ src, Ranges r) {
    const uint32_t o = r.off[blockIdx.y], n16 = r.len[blockIdx.y] / 16;
    const uint4* sp = reinterpret_cast<const uint4*>(src + o);
    uint4* dp = reinterpret_cast<uint4*>(dst + o);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += gridDim.x * blockDim.x)
        dp[i] = sp[i];
}

// Results of request blockIdx.y into its pinned result area.
__global__ __launch_bounds__(256) void k_export(const ExportDesc* __restrict__ ds,
                                                const int32_t* __restrict__ d_out,
                                                const uint32_t* __restrict__ d_dump_n,
                                                const uint32_t* __restrict__ d_n_dumps,
                                                const int32_t* __restrict__ d_status,
                                                uint32_t max_dumps, int tap_stride) {
    const ExportDesc D = ds[blockIdx.y];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t rows = (uint64_t)D.n_chan * max_dumps;
    // rows of tap_stride * 2 words (tap_stride * 8 bytes, a multiple of 16)
    const uint64_t n16 = rows * (uint64_t)tap_stride / 2;
    const uint4* so = reinterpret_cast<const uint4*>(d_out + (uint64_t)D.cb * max_dumps * tap_stride * 2);
    uint4* dout = reinterpret_cast<uint4*>(D.out);
    for (uint64_t i = t; i < n16; i += stride) dout[i] = so[i];
    const uint32_t* sd = d_dump_n + (uint64_t)D.cb * max_dumps;
    for (uint64_t i = t; i < rows; i += stride) D.dump_n[i] = sd[i];
    for (uint64_t i = t; i < (uint64_t)D.n_chan; i += stride) {
        D.n_dumps[i] = d_n_dumps[D.cb + i];
        D.status[i] = d_status[D.cb + i];
    }
}

}  // namespace

struct gc_server {
    gc_ctx* ctx;
    int plain;
    int max_batch_rx;
    uint32_t max_dumps;
    int cap_chan, n_chan, cap_rx;
    gc::DevChan* d_chans;
    gc::DevMeta* d_meta;
    gc_chan_state* d_state;
    int32_t* d_out;
    uint32_t* d_dump_n;
    uint32_t* d_n_dumps;
    int32_t* d_status;
    uint8_t* d_arena;
    Arena dev;
    uint8_t* h_arena;
    uint8_t* h_arena_dev;          // the pinned arena seen from the device
    Arena host;
    LaunchLayout lay;
    hipStream_t up;
    int cus;
    std::vector<SrvRx> rx;
    std::unordered_map<uint64_t, SrvReq> reqs;
    std::deque<uint64_t> done_ids;
    std::vector<SrvSlot> slots;
    std::mutex mu;
    std::condition_variable cv;
    std::thread th;
    bool stop;
    bool hold;                     // form no new launches
    uint64_t next_id;
    size_t rr;                     // round-robin start over receivers
    uint64_t launches, launched_reqs;
    // host-side timing: enqueue of a launch, enqueue end to completion seen,
    // HIP calls of a submission (seconds)
    double enq_sum, enq_max, dev_sum, dev_max, sub_max;
    hipError_t err;                // first device error seen by the dispatcher
};

namespace {

uint64_t sample_bytes(int fmt, uint64_t n) {
    return fmt == GC_I2_REAL ? (n + 3) / 4 : fmt == GC_I2_IQ ? (n + 1) / 2
         : fmt == GC_I8_IQ ? 2 * n : n;
}

uint64_t result_bytes(int n_chan, uint32_t max_dumps) {
    return (uint64_t)n_chan * max_dumps * kTapStride * 2 * 4    // out
           + (uint64_t)n_chan * max_dumps * 4                   // dump_n
           + (uint64_t)n_chan * 4 * 2;                          // n_dumps, status
}

// Result layout in the pinned arena after the staged samples.
struct ResPtr {
    int32_t* out;
    uint32_t* dump_n;
    uint32_t* n_dumps;
    int32_t* status;
};

ResPtr res_ptr(const gc_server* s, const SrvReq& q) {
    const int nc = s->rx[(size_t)q.rx].n_chan;
    uint8_t* base =
        s->h_arena + q.host_off + Arena::round(sample_bytes(s->rx[(size_t)q.rx].fmt, q.n));
    ResPtr r;
    r.out = (int32_t*)base;
    r.dump_n = (uint32_t*)(base + (uint64_t)nc * s->max_dumps * kTapStride * 2 * 4);
    r.n_dumps = r.dump_n + (uint64_t)nc * s->max_dumps;
    r.status = (int32_t*)(r.n_dumps + nc);
    return r;
}

// What one launch needs of a request, copied under the lock so that the
// launch itself runs without it.
struct Job {
    const uint8_t* samples;
    uint64_t n;
    int fmt, cb, n_chan;
    hipEvent_t uploaded;
    ResPtr res;                    // device view of the result area
};

// Device view of a pointer into the pinned host arena.
template <class T>
T* dev_view(const gc_server* s, T* host_ptr) {
    return reinterpret_cast<T*>(s->h_arena_dev + (reinterpret_cast<uint8_t*>(host_ptr) - s->h_arena));
}

// One launch of the given requests (distinct receivers) on a slot: the
// launch tables copied to the device, the correlation, the results written
// into each request's pinned result area -- every step a kernel on the
// slot's stream.
hipError_t launch_batch(const gc_server* s, SrvSlot& sl, const std::vector<Job>& jobs) {
    const int nr = (int)jobs.size();
    const LaunchLayout& L = s->lay;
    gc::DevRx* h_rx = reinterpret_cast<gc::DevRx*>(sl.h_tab + L.off_rx);
    int32_t* h_list = reinterpret_cast<int32_t*>(sl.h_tab + L.off_list);
    int32_t* h_lrx = reinterpret_cast<int32_t*>(sl.h_tab + L.off_lrx);
    ExportDesc* h_exp = reinterpret_cast<ExportDesc*>(sl.h_tab + L.off_exp);
    const gc::DevRx* d_rx = reinterpret_cast<const gc::DevRx*>(sl.d_tab + L.off_rx);
    const int32_t* d_list = reinterpret_cast<const int32_t*>(sl.d_tab + L.off_list);
    const int32_t* d_lrx = reinterpret_cast<const int32_t*>(sl.d_tab + L.off_lrx);
    const ExportDesc* d_exp = reinterpret_cast<const ExportDesc*>(sl.d_tab + L.off_exp);
    const uint32_t tile = gc::epl_batch_tile(0);
    uint32_t items = 0;
    int nl = 0;
    for (int i = 0; i < nr; ++i) {
        const Job& j = jobs[(size_t)i];
        gc::DevRx& d = h_rx[i];
        d.samples = j.samples;
        d.n = j.n;
        d.fmt = j.fmt;
        d.chan_begin = j.cb;
        d.chan_end = j.cb + j.n_chan;
        d.tile_begin = items;
        items += (uint32_t)((j.n + tile - 1) / tile);
        for (int c = 0; c < j.n_chan; ++c) {
            h_list[nl] = j.cb + c;
            h_lrx[nl] = i;
            ++nl;
        }
        h_exp[i] = ExportDesc{j.cb, j.n_chan, j.res.out, j.res.dump_n, j.res.n_dumps,
                              j.res.status};
    }
    hipError_t e = hipSuccess;
    for (const Job& j : jobs)
        if (e == hipSuccess) e = hipStreamWaitEvent(sl.s, j.uploaded, 0);
    if (e == hipSuccess) {
        auto up16 = [](size_t v) { return (uint32_t)((v + 15) & ~size_t(15)); };
        Ranges r;
        r.off[0] = (uint32_t)L.off_rx;   r.len[0] = up16(sizeof(gc::DevRx) * (size_t)nr);
        r.off[1] = (uint32_t)L.off_list; r.len[1] = up16(sizeof(int32_t) * (size_t)nl);
        r.off[2] = (uint32_t)L.off_lrx;  r.len[2] = up16(sizeof(int32_t) * (size_t)nl);
        r.off[3] = (uint32_t)L.off_exp;  r.len[3] = up16(sizeof(ExportDesc) * (size_t)nr);
        hipLaunchKernelGGL(k_copy_ranges, dim3(2, 4), dim3(256), 0, sl.s, sl.d_tab, sl.h_tab_dev,
                           r);
        e = hipGetLastError();
    }
    if (s->plain) {
        // every channel alone: its set-up and a direct-kernel launch
        for (int i = 0; i < nr && e == hipSuccess; ++i) {
            const Job& j = jobs[(size_t)i];
            for (int c = 0; c < j.n_chan && e == hipSuccess; ++c) {
                const int ch = j.cb + c;
                int32_t* out = s->d_out + (uint64_t)ch * s->max_dumps * kTapStride * 2;
                e = gc::launch_setup(s->d_chans + ch, s->d_meta + ch, s->d_state + ch, 1, j.n,
                                     j.fmt, GC_CARRIER_LUT, s->max_dumps, out, kTapStride,
                                     s->d_dump_n + (uint64_t)ch * s->max_dumps,
                                     s->d_n_dumps + ch, s->d_status + ch, 0, nullptr, nullptr,
                                     nullptr, sl.s);
                if (e == hipSuccess)
                    e = gc::launch_generic(j.samples, j.n, j.fmt, GC_CARRIER_LUT,
                                           s->d_chans + ch, s->d_meta + ch, s->d_state + ch, 1,
                                           kTapStride, out, kTapStride, s->max_dumps,
                                           s->ctx->d_tables, 0, sl.s);
            }
        }
    } else {
        if (e == hipSuccess)
            e = gc::launch_setup(s->d_chans, s->d_meta, s->d_state, nl, 0, GC_I8_REAL,
                                 GC_CARRIER_LUT, s->max_dumps, s->d_out, kTapStride, s->d_dump_n,
                                 s->d_n_dumps, s->d_status, gc::kAllowBinned, d_rx, d_list, d_lrx,
                                 sl.s);
        if (e == hipSuccess)
            e = gc::launch_epl_batch(0, s->cus, d_rx, nr, nullptr, items, nullptr, s->d_chans,
                                     s->d_meta, s->d_state, s->d_out, kTapStride, s->max_dumps,
                                     s->ctx->d_tables, sl.s);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_export, dim3(4, nr), dim3(256), 0, sl.s, d_exp, s->d_out,
                           s->d_dump_n, s->d_n_dumps, s->d_status, s->max_dumps, kTapStride);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.s);
    return e;
}

// The dispatcher holds the lock only to read and update the queues: HIP
// calls (event queries, copies, launches) run without it, so submissions
// and polls never wait for a launch to be enqueued.  While launches are in
// flight it polls their events, yielding the core between rounds; when the
// device is idle it sleeps until a submission or hold change wakes it.
void dispatcher(gc_server* s) {
    (void)hipSetDevice(s->ctx->device);
    std::vector<Job> jobs;
    std::vector<char> finished(s->slots.size());
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        bool progress = false, in_flight = false;
        // completions (queried without the lock; only this thread touches slots)
        lk.unlock();
        for (size_t k = 0; k < s->slots.size(); ++k)
            finished[k] = s->slots[k].busy && hipEventQuery(s->slots[k].done) == hipSuccess;
        lk.lock();
        const Clock::time_point now = Clock::now();
        for (size_t k = 0; k < s->slots.size(); ++k) {
            SrvSlot& sl = s->slots[k];
            if (!finished[k]) continue;
            const double dev = std::chrono::duration<double>(now - sl.t_enq).count();
            s->dev_sum += dev;
            s->dev_max = std::max(s->dev_max, dev);
            for (uint64_t id : sl.reqs) {
                SrvReq& q = s->reqs[id];
                q.state = 2;
                q.t_done = now;
                s->dev.release(q.dev_off, q.dev_bytes);
                SrvRx& R = s->rx[(size_t)q.rx];
                R.busy = false;
                R.pending.pop_front();
                s->done_ids.push_back(id);
            }
            sl.busy = false;
            sl.reqs.clear();
            progress = true;
        }
        // new launches on free slots
        for (SrvSlot& sl : s->slots) {
            if (sl.busy || s->hold) continue;
            const size_t nrx = s->rx.size();
            jobs.clear();
            for (size_t k = 0; k < nrx && (int)sl.reqs.size() < s->max_batch_rx; ++k) {
                SrvRx& R = s->rx[(s->rr + k) % nrx];
                if (R.busy || R.pending.empty()) continue;
                R.busy = true;
                const uint64_t id = R.pending.front();
                SrvReq& q = s->reqs[id];
                q.state = 1;
                sl.reqs.push_back(id);
                ResPtr rp = res_ptr(s, q);
                rp.out = dev_view(s, rp.out);
                rp.dump_n = dev_view(s, rp.dump_n);
                rp.n_dumps = dev_view(s, rp.n_dumps);
                rp.status = dev_view(s, rp.status);
                jobs.push_back(Job{s->d_arena + q.dev_off, q.n, R.fmt, R.cb, R.n_chan,
                                   q.uploaded, rp});
            }
            if (sl.reqs.empty()) break;
            s->rr = (s->rr + 1) % (nrx ? nrx : 1);
            sl.busy = true;
            s->launches += 1;
            s->launched_reqs += sl.reqs.size();
            lk.unlock();
            const Clock::time_point t0 = Clock::now();
            const hipError_t e = launch_batch(s, sl, jobs);
            sl.t_enq = Clock::now();
            lk.lock();
            const double enq = std::chrono::duration<double>(sl.t_enq - t0).count();
            s->enq_sum += enq;
            s->enq_max = std::max(s->enq_max, enq);
            if (e != hipSuccess && s->err == hipSuccess) s->err = e;
            progress = true;
        }
        for (const SrvSlot& sl : s->slots) in_flight |= sl.busy;
        if (progress) continue;
        if (in_flight) {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else {
            s->cv.wait(lk);
        }
    }
}

}  // namespace

extern "C" {

gc_status gc_server_create(gc_ctx* ctx, uint64_t hbm_budget_bytes, uint64_t host_budget_bytes,
                           int32_t max_channels, int32_t max_receivers, uint32_t max_dumps,
                           int32_t n_streams, int32_t max_batch_rx, int32_t flags,
                           gc_server** out) {
    if (!ctx || !out) return GC_EINVAL;
    *out = nullptr;
    if (hbm_budget_bytes < 4096 || host_budget_bytes < 4096 || max_channels < 1 ||
        max_channels > GC_MAX_CHANNELS || max_receivers < 1 || max_receivers > 65536 ||
        max_dumps < 2 || max_dumps > 4096 || n_streams < 1 || n_streams > 16 ||
        max_batch_rx < 1 || max_batch_rx > 4096 || (flags & ~GC_SERVER_PLAIN))
        return GC_EINVAL;
    DeviceGuard g(ctx->device);
    if (!g.ok) return GC_EDEVICE;
    gc_server* s = new (std::nothrow) gc_server();
    if (!s) return GC_ENOMEM;
    s->ctx = ctx;
    s->plain = flags & GC_SERVER_PLAIN;
    s->max_batch_rx = (flags & GC_SERVER_PLAIN) ? 1 : max_batch_rx;
    s->max_dumps = max_dumps;
    s->cap_chan = max_channels;
    s->cap_rx = max_receivers;
    s->n_chan = 0;
    s->stop = false;
    s->hold = false;
    s->next_id = 1;
    s->rr = 0;
    s->launches = s->launched_reqs = 0;
    s->enq_sum = s->enq_max = s->dev_sum = s->dev_max = s->sub_max = 0.0;
    s->err = hipSuccess;
    s->cus = gc::epl_blocks_per_device(ctx->device);
    const size_t C = (size_t)max_channels;
    hipError_t e = hipMalloc(&s->d_chans, sizeof(gc::DevChan) * C);
    if (e == hipSuccess) e = hipMalloc(&s->d_meta, sizeof(gc::DevMeta) * C);
    if (e == hipSuccess) e = hipMalloc(&s->d_state, sizeof(gc_chan_state) * C);
    if (e == hipSuccess) e = hipMalloc(&s->d_out, (size_t)max_dumps * kTapStride * 2 * 4 * C);
    if (e == hipSuccess) e = hipMalloc(&s->d_dump_n, (size_t)max_dumps * 4 * C);
    if (e == hipSuccess) e = hipMalloc(&s->d_n_dumps, 4 * C);
    if (e == hipSuccess) e = hipMalloc(&s->d_status, 4 * C);
    if (e == hipSuccess) e = hipMalloc(&s->d_arena, hbm_budget_bytes);
    if (e == hipSuccess) e = hipHostMalloc(&s->h_arena, host_budget_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&s->h_arena_dev, s->h_arena, 0);
    s->lay.init(max_batch_rx, max_channels);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->up, hipStreamNonBlocking);
    s->dev.init(hbm_budget_bytes);
    s->host.init(host_budget_bytes);
    s->slots.resize((size_t)n_streams);
    for (SrvSlot& sl : s->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc(&sl.d_tab, s->lay.bytes);
        if (e == hipSuccess) e = hipHostMalloc(&sl.h_tab, s->lay.bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&sl.h_tab_dev, sl.h_tab, 0);
    }
    // touch every stream once with a device operation (clearing the status
    // words), so that no request pays for the runtime's first use of a queue
    for (SrvSlot& sl : s->slots)
        if (e == hipSuccess) e = hipMemsetAsync(s->d_status, 0, 4 * C, sl.s);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_n_dumps, 0, 4 * C, s->up);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        s->stop = true;
        gc_server_destroy(s);
        return from_hip(e);
    }
    s->th = std::thread(dispatcher, s);
    *out = s;
    return GC_OK;
}

gc_status gc_server_open_rx(gc_server* s, int32_t fmt, const gc_chan_cfg* cfg,
                            const gc_chan_state* state0, int32_t n_chan, int32_t* rx_id) {
    if (!s || !cfg || !state0 || !rx_id || n_chan < 1) return GC_EINVAL;
    if (fmt != GC_I8_REAL && fmt != GC_I8_IQ && fmt != GC_I2_REAL && fmt != GC_I2_IQ)
        return GC_EINVAL;
    std::vector<gc::DevChan> h((size_t)n_chan);
    for (int i = 0; i < n_chan; ++i) {
        const gc_status st = gc::fill_devchan(cfg[i], h[(size_t)i]);
        if (st != GC_OK) return st;
        if (cfg[i].n_taps > kTapStride) return GC_EINVAL;
    }
    DeviceGuard g(s->ctx->device);
    if (!g.ok) return GC_EDEVICE;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->n_chan + n_chan > s->cap_chan || (int)s->rx.size() >= s->cap_rx) return GC_ENOMEM;
    const int cb = s->n_chan;
    for (int i = 0; i < n_chan; ++i) h[(size_t)i].rx = (int32_t)s->rx.size();
    hipError_t e = hipMemcpy(s->d_chans + cb, h.data(), sizeof(gc::DevChan) * (size_t)n_chan,
                             hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(s->d_state + cb, state0, sizeof(gc_chan_state) * (size_t)n_chan,
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) return from_hip(e);
    SrvRx R;
    R.fmt = fmt;
    R.n_chan = n_chan;
    R.cb = cb;
    s->rx.push_back(R);
    s->n_chan += n_chan;
    *rx_id = (int32_t)s->rx.size() - 1;
    return GC_OK;
}

gc_status gc_server_submit(gc_server* s, int32_t rx_id, const void* host_samples,
                           uint64_t n_samples, uint64_t* req_id) {
    if (!s || !req_id || (n_samples > 0 && !host_samples) || n_samples >= (1ull << 31))
        return GC_EINVAL;
    DeviceGuard g(s->ctx->device);
    if (!g.ok) return GC_EDEVICE;
    std::lock_guard<std::mutex> lk(s->mu);
    if (rx_id < 0 || rx_id >= (int32_t)s->rx.size()) return GC_EINVAL;
    if (s->err != hipSuccess) return from_hip(s->err);
    const SrvRx& R = s->rx[(size_t)rx_id];
    SrvReq q;
    q.rx = rx_id;
    q.n = n_samples;
    q.dev_bytes = sample_bytes(R.fmt, n_samples);
    q.host_bytes = Arena::round(q.dev_bytes) + result_bytes(R.n_chan, s->max_dumps);
    if (!s->dev.alloc(q.dev_bytes, &q.dev_off)) return GC_EBUSY;       // HBM budget
    if (!s->host.alloc(q.host_bytes, &q.host_off)) {
        s->dev.release(q.dev_off, q.dev_bytes);
        return GC_EBUSY;
    }
    memcpy(s->h_arena + q.host_off, host_samples, q.dev_bytes);
    const Clock::time_point t0 = Clock::now();
    hipError_t e = hipEventCreateWithFlags(&q.uploaded, hipEventDisableTiming);
    if (e == hipSuccess && q.dev_bytes > 0) {
        const uint32_t blocks = (uint32_t)std::min<uint64_t>(64, (q.dev_bytes + 4095) / 4096);
        hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s->up, s->d_arena + q.dev_off,
                           s->h_arena_dev + q.host_off, q.dev_bytes);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(q.uploaded, s->up);
    s->sub_max = std::max(s->sub_max, std::chrono::duration<double>(Clock::now() - t0).count());
    if (e != hipSuccess) {
        s->dev.release(q.dev_off, q.dev_bytes);
        s->host.release(q.host_off, q.host_bytes);
        return from_hip(e);
    }
    q.state = 0;
    q.t_submit = Clock::now();
    const uint64_t id = s->next_id++;
    s->reqs[id] = q;
    s->rx[(size_t)rx_id].pending.push_back(id);
    *req_id = id;
    s->cv.notify_one();
    return GC_OK;
}

gc_status gc_server_hold(gc_server* s, int32_t hold) {
    if (!s || (hold != 0 && hold != 1)) return GC_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->hold = hold != 0;
    }
    s->cv.notify_one();
    return GC_OK;
}

gc_status gc_server_poll(gc_server* s, uint64_t* ids, int32_t max_n, int32_t* n_done) {
    if (!s || !n_done || (max_n > 0 && !ids) || max_n < 0) return GC_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    int k = 0;
    while (k < max_n && !s->done_ids.empty()) {
        const uint64_t id = s->done_ids.front();
        s->done_ids.pop_front();
        if (s->reqs.count(id)) ids[k++] = id;   // skip ids already collected
    }
    *n_done = k;
    return s->err == hipSuccess ? GC_OK : from_hip(s->err);
}

gc_status gc_server_result(gc_server* s, uint64_t req_id, int32_t* out, uint32_t* dump_n,
                           uint32_t* n_dumps, int32_t* status, double* service_s) {
    if (!s) return GC_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) return GC_EINVAL;
    SrvReq& q = it->second;
    if (q.state != 2) return GC_EAGAIN;
    const int nc = s->rx[(size_t)q.rx].n_chan;
    const ResPtr r = res_ptr(s, q);
    const uint64_t rows = (uint64_t)nc * s->max_dumps;
    if (out) memcpy(out, r.out, rows * kTapStride * 2 * 4);
    if (dump_n) memcpy(dump_n, r.dump_n, rows * 4);
    if (n_dumps) memcpy(n_dumps, r.n_dumps, (size_t)nc * 4);
    if (status) memcpy(status, r.status, (size_t)nc * 4);
    if (service_s) service_s[0] = std::chrono::duration<double>(q.t_done - q.t_submit).count();
    (void)hipEventDestroy(q.uploaded);
    s->host.release(q.host_off, q.host_bytes);
    s->reqs.erase(it);
    return GC_OK;
}

gc_status gc_server_state(gc_server* s, int32_t rx_id, gc_chan_state* host_out) {
    if (!s || !host_out) return GC_EINVAL;
    DeviceGuard g(s->ctx->device);
    if (!g.ok) return GC_EDEVICE;
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (rx_id < 0 || rx_id >= (int32_t)s->rx.size()) return GC_EINVAL;
            const SrvRx& R = s->rx[(size_t)rx_id];
            if (R.pending.empty()) {
                return from_hip(hipMemcpy(host_out, s->d_state + R.cb,
                                          sizeof(gc_chan_state) * (size_t)R.n_chan,
                                          hipMemcpyDeviceToHost));
            }
            if (s->err != hipSuccess) return from_hip(s->err);
        }
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

gc_status gc_server_info(gc_server* s, uint32_t* max_dumps, int32_t* tap_stride,
                         int32_t* in_flight, uint64_t* hbm_in_use, uint64_t* launches,
                         uint64_t* launched_requests) {
    if (!s) return GC_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (max_dumps) *max_dumps = s->max_dumps;
    if (tap_stride) *tap_stride = kTapStride;
    if (in_flight) {
        int k = 0;
        for (auto& kv : s->reqs) k += kv.second.state != 2;
        *in_flight = k;
    }
    if (hbm_in_use) *hbm_in_use = s->dev.in_use();
    if (launches) *launches = s->launches;
    if (launched_requests) *launched_requests = s->launched_reqs;
    return GC_OK;
}

gc_status gc_server_stats(gc_server* s, gc_server_timing* out) {
    if (!s || !out) return GC_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    const double n = s->launches ? (double)s->launches : 1.0;
    out->launches = s->launches;
    out->launched_requests = s->launched_reqs;
    out->enqueue_mean_ms = 1e3 * s->enq_sum / n;
    out->enqueue_max_ms = 1e3 * s->enq_max;
    out->device_mean_ms = 1e3 * s->dev_sum / n;
    out->device_max_ms = 1e3 * s->dev_max;
    out->submit_max_ms = 1e3 * s->sub_max;
    return GC_OK;
}

gc_status gc_server_destroy(gc_server* s) {
    if (!s) return GC_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    DeviceGuard g(s->ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : s->reqs)
        if (kv.second.uploaded) (void)hipEventDestroy(kv.second.uploaded);
    for (SrvSlot& sl : s->slots) {
        if (sl.s) (void)hipStreamDestroy(sl.s);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.d_tab) (void)hipFree(sl.d_tab);
        if (sl.h_tab) (void)hipHostFree(sl.h_tab);
    }
    if (s->up) (void)hipStreamDestroy(s->up);
    if (s->d_chans) (void)hipFree(s->d_chans);
    if (s->d_meta) (void)hipFree(s->d_meta);
    if (s->d_state) (void)hipFree(s->d_state);
    if (s->d_out) (void)hipFree(s->d_out);
    if (s->d_dump_n) (void)hipFree(s->d_dump_n);
    if (s->d_n_dumps) (void)hipFree(s->d_n_dumps);
    if (s->d_status) (void)hipFree(s->d_status);
    if (s->d_arena) (void)hipFree(s->d_arena);
    if (s->h_arena) (void)hipHostFree(s->h_arena);
    delete s;
    return GC_OK;
}

}  // extern "C"
