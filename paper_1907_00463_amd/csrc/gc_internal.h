// gc_internal.h -- definitions shared by the libgnsscorr host runtime and its
// HIP kernels (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gnsscorr.h"

namespace gc {

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
    uint32_t pad;
};

// Kernel launch entry points (defined in the .hip files, called by the runtime).
hipError_t launch_make_tables(uint32_t* d_tables, hipStream_t s);
hipError_t launch_code_table(const uint32_t* d_tables, int g2_delay, int8_t* d_out, hipStream_t s);
hipError_t launch_setup(const DevChan* chans, DevMeta* meta, gc_chan_state* state, int n_chan,
                        uint64_t n_samples, int fmt, int carrier, uint32_t max_dumps,
                        void* out, int tap_stride, uint32_t* dump_n, uint32_t* n_dumps,
                        int32_t* status, hipStream_t s);
hipError_t launch_generic(const uint8_t* samples, uint64_t n_samples, int fmt, int carrier,
                          const DevChan* chans, const DevMeta* meta, gc_chan_state* state,
                          int n_chan, int max_taps, void* out, int tap_stride,
                          uint32_t max_dumps, const uint32_t* d_tables, hipStream_t s);

}  // namespace gc
