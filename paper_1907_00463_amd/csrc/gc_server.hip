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

struct SrvSlot {
    hipStream_t s = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<uint64_t> reqs;
    gc::DevRx* d_rx = nullptr;     // compact receiver table of the launch
    int32_t* d_list = nullptr;     // channels, then their receiver index
    gc::DevRx* h_rx = nullptr;     // pinned mirrors
    int32_t* h_list = nullptr;
};

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
    Arena host;
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
    hipError_t err;                // first device error seen by the dispatcher
};

namespace {

uint64_t sample_bytes(int fmt, uint64_t n) { return fmt == GC_I2_REAL ? (n + 3) / 4 : n; }

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
    ResPtr res;
};

// Copies of one request's rows, sample counts, dump counts and statuses.
hipError_t copy_results(const gc_server* s, const Job& j, hipStream_t st) {
    const uint64_t rows = (uint64_t)j.n_chan * s->max_dumps;
    hipError_t e = hipMemcpyAsync(j.res.out,
                                  s->d_out + (uint64_t)j.cb * s->max_dumps * kTapStride * 2,
                                  rows * kTapStride * 2 * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(j.res.dump_n, s->d_dump_n + (uint64_t)j.cb * s->max_dumps, rows * 4,
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(j.res.n_dumps, s->d_n_dumps + j.cb, (size_t)j.n_chan * 4,
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(j.res.status, s->d_status + j.cb, (size_t)j.n_chan * 4,
                           hipMemcpyDeviceToHost, st);
    return e;
}

// One launch of the given requests (distinct receivers) on a slot.
hipError_t launch_batch(const gc_server* s, SrvSlot& sl, const std::vector<Job>& jobs) {
    const int nr = (int)jobs.size();
    hipError_t e = hipSuccess;
    for (const Job& j : jobs)
        if (e == hipSuccess) e = hipStreamWaitEvent(sl.s, j.uploaded, 0);
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
            if (e == hipSuccess) e = copy_results(s, j, sl.s);
        }
    } else {
        const uint32_t tile = gc::epl_batch_tile(0);
        uint32_t items = 0;
        int nl = 0;
        for (int i = 0; i < nr; ++i) {
            const Job& j = jobs[(size_t)i];
            gc::DevRx& d = sl.h_rx[i];
            d.samples = j.samples;
            d.n = j.n;
            d.fmt = j.fmt;
            d.chan_begin = j.cb;
            d.chan_end = j.cb + j.n_chan;
            d.tile_begin = items;
            items += (uint32_t)((j.n + tile - 1) / tile);
            for (int c = 0; c < j.n_chan; ++c) {
                sl.h_list[nl] = j.cb + c;
                sl.h_list[s->cap_chan + nl] = i;
                ++nl;
            }
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(sl.d_rx, sl.h_rx, sizeof(gc::DevRx) * (size_t)nr,
                               hipMemcpyHostToDevice, sl.s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(sl.d_list, sl.h_list, sizeof(int32_t) * (size_t)nl,
                               hipMemcpyHostToDevice, sl.s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(sl.d_list + s->cap_chan, sl.h_list + s->cap_chan,
                               sizeof(int32_t) * (size_t)nl, hipMemcpyHostToDevice, sl.s);
        if (e == hipSuccess)
            e = gc::launch_setup(s->d_chans, s->d_meta, s->d_state, nl, 0, GC_I8_REAL,
                                 GC_CARRIER_LUT, s->max_dumps, s->d_out, kTapStride, s->d_dump_n,
                                 s->d_n_dumps, s->d_status, gc::kAllowBinned, sl.d_rx, sl.d_list,
                                 sl.d_list + s->cap_chan, sl.s);
        if (e == hipSuccess)
            e = gc::launch_epl_batch(0, s->cus, sl.d_rx, nr, nullptr, items, nullptr, s->d_chans,
                                     s->d_meta, s->d_state, s->d_out, kTapStride, s->max_dumps,
                                     s->ctx->d_tables, sl.s);
        for (int i = 0; i < nr && e == hipSuccess; ++i) e = copy_results(s, jobs[(size_t)i], sl.s);
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
                jobs.push_back(Job{s->d_arena + q.dev_off, q.n, R.fmt, R.cb, R.n_chan,
                                   q.uploaded, res_ptr(s, q)});
            }
            if (sl.reqs.empty()) break;
            s->rr = (s->rr + 1) % (nrx ? nrx : 1);
            sl.busy = true;
            s->launches += 1;
            s->launched_reqs += sl.reqs.size();
            lk.unlock();
            const hipError_t e = launch_batch(s, sl, jobs);
            lk.lock();
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
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->up, hipStreamNonBlocking);
    s->dev.init(hbm_budget_bytes);
    s->host.init(host_budget_bytes);
    s->slots.resize((size_t)n_streams);
    for (SrvSlot& sl : s->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc(&sl.d_rx, sizeof(gc::DevRx) * (size_t)max_batch_rx);
        if (e == hipSuccess) e = hipMalloc(&sl.d_list, sizeof(int32_t) * 2 * C);
        if (e == hipSuccess)
            e = hipHostMalloc(&sl.h_rx, sizeof(gc::DevRx) * (size_t)max_batch_rx,
                              hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc(&sl.h_list, sizeof(int32_t) * 2 * C, hipHostMallocDefault);
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
    if (fmt != GC_I8_REAL && fmt != GC_I2_REAL) return GC_EINVAL;
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
    hipError_t e = hipEventCreateWithFlags(&q.uploaded, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->d_arena + q.dev_off, s->h_arena + q.host_off, q.dev_bytes,
                           hipMemcpyHostToDevice, s->up);
    if (e == hipSuccess) e = hipEventRecord(q.uploaded, s->up);
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
        if (sl.d_rx) (void)hipFree(sl.d_rx);
        if (sl.d_list) (void)hipFree(sl.d_list);
        if (sl.h_rx) (void)hipHostFree(sl.h_rx);
        if (sl.h_list) (void)hipHostFree(sl.h_list);
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
