// gc_internal.h -- definitions shared by the libgnsscorr host runtime and its
// HIP kernels (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gnsscorr.h"

// A context: one device and its tables (opaque in the C ABI).
struct gc_ctx {
    int device;
    uint32_t* d_tables;  // G1, G2, carrier table, sign and code tables (gc::kTabWords words)
    hipStream_t stream;  // context-private stream for synchronous helpers
    int n_cu;            // compute units of the device (persistent grids)
    uint8_t* d_scratch;  // this device's copy of the fixed array of gc_correlate_noalloc
};

namespace gc {

// Makes `dev` current for the guard's lifetime.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

inline gc_status from_hip(hipError_t e) {
    if (e == hipSuccess) return GC_OK;
    if (e == hipErrorOutOfMemory) return GC_ENOMEM;
    return GC_EDEVICE;
}

constexpr uint64_t kTwo32 = 1ull << 32;
constexpr int kCodeLen = GC_CODE_LEN;

// Per-channel static configuration as the kernels read it (device memory,
// written once by gc_plan_create).
struct DevChan {
    int32_t prn;
    int32_t n_taps;
    int32_t int_periods;
    int32_t g2_delay;      // IS-GPS-200 Table 3-Ia G2 delay of this PRN, chips
    uint64_t window;       // W = int_periods * 1023 * 2^32
    int32_t epl;           // 1: taps are early/prompt/late at +1/2, 0, -1/2 chip
    int32_t slot_e, slot_p, slot_l;  // output tap slots of E, P, L when epl
    int32_t mt_ok;         // every tap a multiple of 2^27 (1/32 chip) spanning <= 8 chip shifts
    int32_t mt_jmin;       // smallest chip shift floor(d_min / 32), d = tap / 2^27
    int32_t mt_nj;         // number of chip shifts
    int32_t rx;            // receiver of the channel in a batch (0 in a plan)
    int64_t taps[GC_MAX_TAPS];
};

// Per-channel, per-call values fixed before the accumulation kernels run
// (device scratch owned by the plan, rewritten by every call).
struct DevMeta {
    uint64_t p0;           // code phase at sample 0 (Q32 chips, in [0, W))
    uint64_t dp;           // code step
    uint64_t window;
    uint32_t phi0;         // carrier phase word at sample 0
    uint32_t dphi;         // carrier step word
    double phf0;           // FP32 carrier: cycles at sample 0
    double ff;             // FP32 carrier: cycles per sample
    uint32_t m_close;      // windows closed by this block (dumps emitted)
    int32_t status;        // gc_status of this channel for this call
    uint32_t acc_n0;       // samples already in the open dump
    int32_t path;          // kPath* (per call, from the steps)
    uint64_t c_full0;      // first chip whose samples all lie in this block
    uint64_t c_full1;      // one past the last such chip
    uint32_t head_end;     // samples [0, head_end) precede chip c_full0
    uint32_t tail_beg;     // samples [tail_beg, n) follow chip c_full1 - 1
    int32_t bin_len;       // samples per half chip on the periodic path
    uint32_t pad2;
};

// One receiver of a batch: its sample block and the channels and work
// items (tiles) that belong to it.
struct DevRx {
    const uint8_t* samples;
    uint64_t n;            // samples in the block
    int32_t fmt;
    int32_t chan_begin;    // channels [chan_begin, chan_end)
    int32_t chan_end;
    uint32_t tile_begin;   // first work item of this receiver
};

// A work item of the batched periodic kernel: tiles [tile_begin, tile_end)
// of receiver rx for its channels [chan_begin, chan_begin + n_chan), at most
// 16 of them.
struct PbinItem {
    int32_t rx;
    int32_t chan_begin;
    int32_t n_chan;
    uint32_t tile_begin;
    uint32_t tile_end;
};

constexpr int32_t kPathDirect = 0;
constexpr int32_t kPathBinned = 1;
constexpr int32_t kPathPeriodic = 2;
constexpr int32_t kPathMtap = 3;

// Plan-level switches passed to the set-up kernel.
constexpr int32_t kAllowBinned = 1;
constexpr int32_t kAllowPeriodic = 2;
constexpr int32_t kAllowMtap = 4;

// Loop constants of gc_track, passed by value: the loop parameters and the
// CORDIC angles round(atan(2^-i) * 2^30), i = 0 .. kCordicSteps - 1.
constexpr int kCordicSteps = 31;
struct TrackConsts {
    double fs, if_hz;
    double dll_bw, dll_zeta, dll_k;
    double pll_bw, pll_zeta, pll_k;
    double fll_bw;
    int64_t tab[kCordicSteps];
};

// Validated device form of a channel configuration (host side).
gc_status fill_devchan(const gc_chan_cfg& c, DevChan& d);

// Kernel launch entry points (defined in the .hip files, called by the runtime).
hipError_t launch_make_tables(uint32_t* d_tables, hipStream_t s);
// channel records from device-resident configurations (gc_correlate_noalloc)
hipError_t launch_fill_chans(const gc_chan_cfg* cfg, int n_chan, int tap_stride, DevChan* out,
                             hipStream_t s);
hipError_t launch_code_table(const uint32_t* d_tables, int g2_delay, int8_t* d_out, hipStream_t s);
// The chip-by-chip batch kernel's item selection, run inside the set-up:
// receivers rx[0 .. n_rx) (with tile_begin, n_items tiles in all), the
// channels chans[0 .. n_chan) (with their receiver in DevChan.rx); order
// (n_items words) and *count receive the items with work, *queue (when not
// null) is zeroed.
struct SelectArgs {
    const DevRx* rx = nullptr;
    int n_rx = 0;
    int n_chan = 0;
    uint32_t n_items = 0;
    uint32_t* order = nullptr;
    uint32_t* count = nullptr;
    uint32_t* queue = nullptr;
};
hipError_t launch_setup(const DevChan* chans, DevMeta* meta, gc_chan_state* state, int n_chan,
                        uint64_t n_samples, int fmt, int carrier, uint32_t max_dumps,
                        void* out, int tap_stride, uint32_t* dump_n, uint32_t* n_dumps,
                        int32_t* status, int32_t allow, const DevRx* rx,
                        const int32_t* list, const int32_t* list_rx, hipStream_t s,
                        const SelectArgs* sel = nullptr);
// list: the channels to set up (null: 0 .. n_chan-1); rx: receiver table of a
// batch (null: one block of n_samples in fmt), indexed by list_rx[i] when
// given, else by the channel's rx field
// batched chip-by-chip kernel (shape 0 .. epl_batch_shapes()-1)
int epl_batch_shapes();
uint32_t epl_batch_tile(int shape);
// (n_items_dev: when not null, a device word holding the number of items
// of `order` to run, at most n_items)
hipError_t launch_epl_batch(int shape, int grid, const DevRx* rx, int n_rx,
                            const uint32_t* order, uint32_t n_items, const uint32_t* n_items_dev,
                            const DevChan* chans, const DevMeta* meta, gc_chan_state* state,
                            int32_t* out, int tap_stride, uint32_t max_dumps,
                            const uint32_t* tables, hipStream_t s);
hipError_t launch_pbin(const uint8_t* samples, uint64_t n_samples, int fmt, const DevChan* chans,
                       const DevMeta* meta, gc_chan_state* state, int n_chan, int32_t* out,
                       int tap_stride, uint32_t max_dumps, const uint32_t* d_tables, int grid,
                       hipStream_t s);
int pbin_tile_samples();
// counter: one device word, the items' queue, zero when the kernel starts
// (the set-up's item selection zeroes it)
hipError_t launch_pbin_batch(int grid, const DevRx* rx, const PbinItem* items, uint32_t n_items,
                             uint32_t* counter, const DevChan* chans, const DevMeta* meta,
                             gc_chan_state* state, int32_t* out, int tap_stride,
                             uint32_t max_dumps, const uint32_t* tables, hipStream_t s);
hipError_t launch_mtap(const uint8_t* samples, uint64_t n_samples, int fmt, const DevChan* chans,
                       const DevMeta* meta, gc_chan_state* state, int n_chan, int32_t* out,
                       int tap_stride, uint32_t max_dumps, const uint32_t* d_tables, int grid,
                       hipStream_t s);
// carrier: GC_CARRIER_LUT (integer dumps) or GC_CARRIER_F32 (float dumps in out)
hipError_t launch_epl(const uint8_t* samples, uint64_t n_samples, int fmt, int carrier,
                      const DevChan* chans, const DevMeta* meta, gc_chan_state* state, int n_chan,
                      int32_t* out, int tap_stride, uint32_t max_dumps, const uint32_t* d_tables,
                      int grid, hipStream_t s);
int epl_blocks_per_device(int device);
hipError_t launch_lock_metrics(const int32_t* rows, int stride, int col, const uint32_t* n_dumps,
                               int n_chan, uint32_t max_dumps, uint32_t K, double T,
                               double lock_min, const uint32_t* phase, double* cn0, double* lock,
                               uint32_t max_windows, uint32_t* n_windows, uint32_t* lock_fails,
                               uint32_t* hist, uint32_t* edge, uint8_t* bits, uint32_t max_bits,
                               uint32_t* n_bits, hipStream_t s);
hipError_t launch_track(const uint8_t* samples, uint64_t n, int fmt, const DevChan* chans,
                        gc_chan_state* state, gc_loop_state* loop, const TrackConsts& consts,
                        int n_chan, int32_t* rows, uint32_t* dump_n, uint32_t* n_dumps,
                        int32_t* status, uint32_t max_dumps, const uint32_t* tables,
                        hipStream_t s);
// largest errors of the float carrier's sin/cos over a range of fp32 phases
// (two zeroed device words in, double bit patterns out)
hipError_t launch_carrier_sweep(uint32_t first, uint32_t count, unsigned long long* out,
                                hipStream_t s);
hipError_t launch_generic(const uint8_t* samples, uint64_t n_samples, int fmt, int carrier,
                          const DevChan* chans, const DevMeta* meta, gc_chan_state* state,
                          int n_chan, int max_taps, void* out, int tap_stride,
                          uint32_t max_dumps, const uint32_t* d_tables, int grid_x,
                          hipStream_t s);  // grid_x 0: one block per tile

}  // namespace gc
