// gc_runtime.hip -- host runtime of libgnsscorr: contexts, plans, argument
// validation, NCO word conversion and kernel dispatch behind the C ABI.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "gc_internal.h"
#include "gc_device.h"

using gc::DeviceGuard;
using gc::from_hip;


struct gc_plan {
    gc_ctx* ctx;
    int fmt;
    int carrier;
    int n_chan;
    int max_taps;
    gc::DevChan* d_chans;
    gc::DevMeta* d_meta;
    int use_epl;      // all channels <= 4 taps (chip-by-chip kernel, either carrier)
    int use_mtap;     // table carrier and some channel has dense 1/32-chip taps
    int kernels;      // GC_KERNEL_* mask
    int epl_grid;     // persistent blocks of the binned kernel
    // timing slots (empty: off): events before, between and after the two
    // correlation kernels of a call
    std::vector<hipEvent_t> ev_start, ev_mid, ev_stop;
    std::vector<uint8_t> ev_used;
    uint64_t calls;
};

namespace {

// The fixed device array of gc_correlate_noalloc: GC_NOALLOC_MAX_CHANNELS
// channel records (DevChan) followed by as many per-call set-up records
// (DevMeta).  Each GPU holds its own copy from the library's load to the end
// of the process; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (gc_create keeps it in
// the context), never through the array's name.
constexpr size_t kNoallocChanBytes = sizeof(gc::DevChan) * GC_NOALLOC_MAX_CHANNELS;
constexpr size_t kNoallocBytes = kNoallocChanBytes + sizeof(gc::DevMeta) * GC_NOALLOC_MAX_CHANNELS;
static_assert(kNoallocChanBytes % 256 == 0, "set-up records start 256-byte aligned");

}  // namespace

static __device__ __align__(256) uint8_t scratch[kNoallocBytes];

namespace {

// G2 delay in chips of PRN 1..32 (IS-GPS-200, Table 3-Ia).
const int32_t kG2Delay[32] = {5,   6,   7,   8,   17,  18,  139, 140, 141, 251, 252,
                              254, 255, 256, 257, 258, 469, 470, 471, 472, 473, 474,
                              509, 512, 513, 514, 515, 516, 859, 860, 861, 862};

}  // namespace

namespace gc {

gc_status fill_devchan(const gc_chan_cfg& c, DevChan& d) {
    if (c.prn < 1 || c.prn > 32 || c.n_taps < 1 || c.n_taps > GC_MAX_TAPS ||
        c.int_periods < 1 || c.int_periods > 1000 || c.reserved != 0)
        return GC_EINVAL;
    memset(&d, 0, sizeof(d));
    d.prn = c.prn;
    d.n_taps = c.n_taps;
    d.int_periods = c.int_periods;
    d.g2_delay = kG2Delay[c.prn - 1];
    d.window = (uint64_t)c.int_periods * GC_CODE_LEN * gc::kTwo32;
    for (int k = 0; k < c.n_taps; ++k) {
        const int64_t t = c.tap_q32[k];
        if (t <= -(int64_t(1) << 40) || t >= (int64_t(1) << 40)) return GC_EINVAL;
        d.taps[k] = t;
    }
    // early / prompt / late at +1/2, 0, -1/2 chip, in any order
    d.epl = 0;
    d.slot_e = d.slot_p = d.slot_l = -1;
    if (c.n_taps == 3) {
        const int64_t h = int64_t(1) << 31;
        for (int k = 0; k < 3; ++k) {
            if (c.tap_q32[k] == h) d.slot_e = k;
            else if (c.tap_q32[k] == 0) d.slot_p = k;
            else if (c.tap_q32[k] == -h) d.slot_l = k;
        }
        d.epl = d.slot_e >= 0 && d.slot_p >= 0 && d.slot_l >= 0;
    }
    // dense taps on the 1/32-chip grid: d = tap / 2^27, chip shifts
    // floor(d_min / 32) .. floor((d_max + 31) / 32), at most 8 of them
    bool grid = true;
    int64_t dmin = 0, dmax = 0;
    for (int k = 0; k < c.n_taps; ++k) {
        const int64_t t = c.tap_q32[k];
        if (t & ((int64_t(1) << 27) - 1)) grid = false;
        const int64_t dk = t >> 27;
        if (k == 0 || dk < dmin) dmin = dk;
        if (k == 0 || dk > dmax) dmax = dk;
    }
    auto fdiv = [](int64_t a, int64_t b) { return a >= 0 ? a / b : -((b - 1 - a) / b); };
    const int64_t jmin = fdiv(dmin, 32), jmax = fdiv(dmax + 31, 32);
    d.mt_ok = grid && jmax - jmin + 1 <= 8;
    d.mt_jmin = (int32_t)jmin;
    d.mt_nj = (int32_t)(jmax - jmin + 1);
    return GC_OK;
}

}  // namespace gc

namespace {

// What one correlation call launches, from a plan or from the fixed array.
struct Launches {
    int fmt, carrier, n_chan, tap_stride;
    bool periodic, binned, mtap;
    int grid;
    gc::DevChan* chans;
    gc::DevMeta* meta;
    const uint32_t* tables;
    hipEvent_t ev_start = nullptr, ev_mid = nullptr, ev_stop = nullptr;  // null: untimed
};

// Set-up, then two correlation kernels; which one does the work is decided
// on the device per channel.  Periodic plans: the periodic kernel, then the
// chip-by-chip kernel for the E/P/L channels it leaves.  Multi-tap plans:
// the MFMA kernel, then the direct kernel (one block per channel and tap
// group looping over the tiles) for channels off the 1/32-chip grid or
// above 32 samples per chip.  A kernel with no channel returns at once.
// Timing events (when given) go before, between and after the two; the
// kernel time is the longer of the two intervals.
hipError_t run_correlation(const Launches& L, const void* samples, uint64_t n_samples,
                           gc_chan_state* state, void* out, uint32_t* dump_n,
                           uint32_t* n_dumps, int32_t* status, uint32_t max_dumps,
                           hipStream_t s) {
    const int32_t allow = (L.periodic ? gc::kAllowPeriodic : 0) |
                          (L.binned ? gc::kAllowBinned : 0) | (L.mtap ? gc::kAllowMtap : 0);
    hipError_t e = gc::launch_setup(L.chans, L.meta, state, L.n_chan, n_samples, L.fmt,
                                    L.carrier, max_dumps, out, L.tap_stride, dump_n, n_dumps,
                                    status, allow, nullptr, nullptr, nullptr, s);
    const uint8_t* x = (const uint8_t*)samples;
    int32_t* o = (int32_t*)out;
    if (e == hipSuccess && L.ev_start) e = hipEventRecord(L.ev_start, s);
    if (e == hipSuccess) {
        if (L.mtap)
            e = gc::launch_mtap(x, n_samples, L.fmt, L.chans, L.meta, state, L.n_chan, o,
                                L.tap_stride, max_dumps, L.tables, L.grid, s);
        else if (L.periodic)
            e = gc::launch_pbin(x, n_samples, L.fmt, L.chans, L.meta, state, L.n_chan, o,
                                L.tap_stride, max_dumps, L.tables, L.grid, s);
        else if (L.binned)
            e = gc::launch_epl(x, n_samples, L.fmt, L.carrier, L.chans, L.meta, state, L.n_chan, o,
                               L.tap_stride, max_dumps, L.tables, L.grid, s);
        else
            e = gc::launch_generic(x, n_samples, L.fmt, L.carrier, L.chans, L.meta, state,
                                   L.n_chan, L.tap_stride, out, L.tap_stride, max_dumps,
                                   L.tables, 0, s);
    }
    if (e == hipSuccess && L.ev_mid) e = hipEventRecord(L.ev_mid, s);
    if (e == hipSuccess && L.periodic)
        e = gc::launch_epl(x, n_samples, L.fmt, L.carrier, L.chans, L.meta, state, L.n_chan, o,
                           L.tap_stride, max_dumps, L.tables, L.grid, s);
    if (e == hipSuccess && L.mtap)
        e = gc::launch_generic(x, n_samples, L.fmt, L.carrier, L.chans, L.meta, state,
                               L.n_chan, L.tap_stride, out, L.tap_stride, max_dumps,
                               L.tables, 1, s);
    if (e == hipSuccess && L.ev_stop) e = hipEventRecord(L.ev_stop, s);
    return e;
}

}  // namespace

extern "C" {

const char* gc_strerror(gc_status s) {
    switch (s) {
        case GC_OK: return "ok";
        case GC_EINVAL: return "invalid argument";
        case GC_ENOMEM: return "out of memory";
        case GC_EDEVICE: return "HIP device error";
        case GC_ERANGE: return "dump could exceed the int32 accumulator range";
        case GC_EBUSY: return "admission refused: over the HBM budget";
        case GC_EAGAIN: return "result not ready";
        case GC_ENOSPC: return "more dumps than max_dumps";
    }
    return "unknown status";
}

gc_status gc_version(int32_t* major, int32_t* minor) {
    if (!major || !minor) return GC_EINVAL;
    *major = GC_VERSION_MAJOR;
    *minor = GC_VERSION_MINOR;
    return GC_OK;
}

gc_status gc_create(gc_ctx** out, int32_t device) {
    if (!out) return GC_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return GC_EDEVICE;
    if (device < 0 || device >= n) return GC_EINVAL;
    DeviceGuard g(device);
    if (!g.ok) return GC_EDEVICE;
    gc_ctx* c = new (std::nothrow) gc_ctx();
    if (!c) return GC_ENOMEM;
    c->device = device;
    c->d_tables = nullptr;
    c->stream = nullptr;
    c->n_cu = gc::epl_blocks_per_device(device);
    c->d_scratch = nullptr;
    // this device's copy of the fixed array (the device is current here)
    hipError_t e = hipGetSymbolAddress((void**)&c->d_scratch, HIP_SYMBOL(scratch));
    if (e == hipSuccess && !c->d_scratch) e = hipErrorInvalidSymbol;
    if (e == hipSuccess) e = hipMalloc(&c->d_tables, gc::kTabWords * sizeof(uint32_t));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = gc::launch_make_tables(c->d_tables, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        if (c->d_tables) (void)hipFree(c->d_tables);
        if (c->stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return from_hip(e);
    }
    *out = c;
    return GC_OK;
}

gc_status gc_destroy(gc_ctx* ctx) {
    if (!ctx) return GC_EINVAL;
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(ctx->d_tables);
    (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return GC_OK;
}

gc_status gc_nco_init(double fs_hz, double carr_hz, double carr_phase_cyc, double code_rate_cps,
                      double code_phase_chips, int32_t int_periods, gc_chan_state* out) {
    if (!out || !(fs_hz > 0.0) || !(code_rate_cps > 0.0) || int_periods < 1) return GC_EINVAL;
    if (!isfinite(carr_hz) || !isfinite(carr_phase_cyc) || !isfinite(code_phase_chips))
        return GC_EINVAL;
    const double two32 = 4294967296.0;
    const double step_code = nearbyint(code_rate_cps / fs_hz * two32);
    if (!(step_code >= 1.0) || !(step_code < 2147483648.0)) return GC_EINVAL;
    memset(out, 0, sizeof(*out));
    const double cstep = nearbyint(carr_hz / fs_hz * two32);
    out->carr_step = (uint32_t)(uint64_t)(int64_t)cstep;
    const double frac_ph = carr_phase_cyc - floor(carr_phase_cyc);
    out->carr_phase = (uint32_t)(uint64_t)(int64_t)nearbyint(frac_ph * two32);
    out->code_step = (uint64_t)step_code;
    const double span = (double)int_periods * GC_CODE_LEN;
    double p = fmod(code_phase_chips, span);
    if (p < 0.0) p += span;
    const uint64_t W = (uint64_t)int_periods * GC_CODE_LEN * gc::kTwo32;
    out->code_phase = ((uint64_t)nearbyint(p * two32)) % W;
    out->carr_phase_f = frac_ph;
    out->carr_freq_f = carr_hz / fs_hz;
    return GC_OK;
}

gc_status gc_code_table(gc_ctx* ctx, int32_t prn, int8_t* host_out) {
    if (!ctx || !host_out || prn < 1 || prn > 32) return GC_EINVAL;
    DeviceGuard g(ctx->device);
    int8_t* d = nullptr;
    hipError_t e = hipMalloc(&d, 1024);
    if (e == hipSuccess) e = gc::launch_code_table(ctx->d_tables, kG2Delay[prn - 1], d, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host_out, d, GC_CODE_LEN, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (d) (void)hipFree(d);
    return from_hip(e);
}

gc_status gc_carrier_f32_error(gc_ctx* ctx, uint32_t first_bits, uint32_t count,
                               double* host_err) {
    if (!ctx || !host_err || count == 0) return GC_EINVAL;
    // every phase in [0, 1): bit patterns below that of 1.0f
    if (first_bits >= 0x3F800000u || count > 0x3F800000u - first_bits) return GC_EINVAL;
    DeviceGuard g(ctx->device);
    if (!g.ok) return GC_EDEVICE;
    unsigned long long* d = nullptr;
    unsigned long long h[2] = {0, 0};
    hipError_t e = hipMalloc(&d, sizeof(h));
    if (e == hipSuccess) e = hipMemsetAsync(d, 0, sizeof(h), ctx->stream);
    if (e == hipSuccess) e = gc::launch_carrier_sweep(first_bits, count, d, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (d) (void)hipFree(d);
    if (e == hipSuccess) {
        memcpy(&host_err[0], &h[0], sizeof(double));
        memcpy(&host_err[1], &h[1], sizeof(double));
    }
    return from_hip(e);
}

gc_status gc_plan_create(gc_ctx* ctx, gc_format fmt, gc_carrier carrier, const gc_chan_cfg* cfg,
                         int32_t n_chan, gc_plan** out) {
    if (!ctx || !cfg || !out) return GC_EINVAL;
    *out = nullptr;
    if (n_chan < 1 || n_chan > GC_MAX_CHANNELS) return GC_EINVAL;
    if (fmt != GC_I8_REAL && fmt != GC_I8_IQ && fmt != GC_I2_REAL && fmt != GC_I2_IQ)
        return GC_EINVAL;
    if (carrier != GC_CARRIER_LUT && carrier != GC_CARRIER_F32) return GC_EINVAL;
    std::vector<gc::DevChan> h((size_t)n_chan);
    int max_taps = 0;
    for (int i = 0; i < n_chan; ++i) {
        const gc_status st = gc::fill_devchan(cfg[i], h[(size_t)i]);
        if (st != GC_OK) return st;
        if (cfg[i].n_taps > max_taps) max_taps = cfg[i].n_taps;
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return GC_EDEVICE;
    gc_plan* p = new (std::nothrow) gc_plan();
    if (!p) return GC_ENOMEM;
    p->ctx = ctx;
    p->fmt = fmt;
    p->carrier = carrier;
    p->n_chan = n_chan;
    p->max_taps = max_taps;
    p->d_chans = nullptr;
    p->d_meta = nullptr;
    p->calls = 0;
    p->use_epl = max_taps <= 4;
    p->use_mtap = 0;
    if (carrier == GC_CARRIER_LUT && !p->use_epl)
        for (int i = 0; i < n_chan; ++i) p->use_mtap |= h[(size_t)i].mt_ok;
    p->kernels = GC_KERNEL_PERIODIC | GC_KERNEL_BINNED | GC_KERNEL_MTAP;
    p->epl_grid = ctx->n_cu;
    hipError_t e = hipMalloc(&p->d_chans, sizeof(gc::DevChan) * (size_t)n_chan);
    if (e == hipSuccess) e = hipMalloc(&p->d_meta, sizeof(gc::DevMeta) * (size_t)n_chan);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_chans, h.data(), sizeof(gc::DevChan) * (size_t)n_chan,
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (p->d_chans) (void)hipFree(p->d_chans);
        if (p->d_meta) (void)hipFree(p->d_meta);
        delete p;
        return from_hip(e);
    }
    *out = p;
    return GC_OK;
}

static void drop_timing(gc_plan* plan) {
    for (auto e : plan->ev_start) (void)hipEventDestroy(e);
    for (auto e : plan->ev_mid) (void)hipEventDestroy(e);
    for (auto e : plan->ev_stop) (void)hipEventDestroy(e);
    plan->ev_start.clear();
    plan->ev_mid.clear();
    plan->ev_stop.clear();
    plan->ev_used.clear();
}

gc_status gc_plan_timing(gc_plan* plan, int32_t n_slots) {
    if (!plan || n_slots < 0 || n_slots > 4096) return GC_EINVAL;
    DeviceGuard g(plan->ctx->device);
    (void)hipDeviceSynchronize();
    drop_timing(plan);
    for (int i = 0; i < n_slots; ++i) {
        hipEvent_t ev[3];
        for (int k = 0; k < 3; ++k) {
            if (hipEventCreateWithFlags(&ev[k], hipEventDisableSystemFence) != hipSuccess) {
                for (int j = 0; j < k; ++j) (void)hipEventDestroy(ev[j]);
                drop_timing(plan);
                return GC_EDEVICE;
            }
        }
        plan->ev_start.push_back(ev[0]);
        plan->ev_mid.push_back(ev[1]);
        plan->ev_stop.push_back(ev[2]);
    }
    plan->ev_used.assign((size_t)n_slots, 0);
    plan->calls = 0;
    return GC_OK;
}

gc_status gc_plan_kernel_ms(gc_plan* plan, int32_t slot, float* ms) {
    if (!plan || !ms || slot < 0 || (size_t)slot >= plan->ev_stop.size()) return GC_EINVAL;
    if (!plan->ev_used[(size_t)slot]) return GC_EINVAL;
    DeviceGuard g(plan->ctx->device);
    const size_t i = (size_t)slot;
    float a = 0.0f, b = 0.0f;
    hipError_t e = hipEventSynchronize(plan->ev_stop[i]);
    if (e == hipSuccess) e = hipEventElapsedTime(&a, plan->ev_start[i], plan->ev_mid[i]);
    if (e == hipSuccess) e = hipEventElapsedTime(&b, plan->ev_mid[i], plan->ev_stop[i]);
    if (e == hipSuccess) *ms = a > b ? a : b;
    return from_hip(e);
}

gc_status gc_plan_destroy(gc_plan* plan) {
    if (!plan) return GC_EINVAL;
    DeviceGuard g(plan->ctx->device);
    (void)hipDeviceSynchronize();
    drop_timing(plan);
    (void)hipFree(plan->d_chans);
    (void)hipFree(plan->d_meta);
    delete plan;
    return GC_OK;
}

gc_status gc_plan_set_kernels(gc_plan* plan, int32_t mask) {
    if (!plan || (mask & ~(GC_KERNEL_PERIODIC | GC_KERNEL_BINNED | GC_KERNEL_MTAP)))
        return GC_EINVAL;
    plan->kernels = mask;
    return GC_OK;
}

gc_status gc_plan_info(const gc_plan* plan, int32_t* tap_stride, int32_t* n_chan) {
    if (!plan || !tap_stride || !n_chan) return GC_EINVAL;
    *tap_stride = plan->max_taps;
    *n_chan = plan->n_chan;
    return GC_OK;
}

gc_status gc_loop_init(double carr_hz, double code_cps, gc_loop_state* out) {
    if (!out) return GC_EINVAL;
    memset(out, 0, sizeof(*out));
    out->carr_hz = carr_hz;
    out->code_cps = code_cps;
    out->fll_basis_hz = carr_hz;
    return GC_OK;
}

gc_status gc_track(gc_plan* plan, const void* samples, uint64_t n_samples,
                   const gc_loop_params* params, gc_chan_state* state, gc_loop_state* loop,
                   int32_t* rows, uint32_t* dump_n, uint32_t* n_dumps, int32_t* status,
                   uint32_t max_dumps, void* stream) {
    if (!plan || !params || !state || !loop || !rows || !dump_n || !n_dumps || !status)
        return GC_EINVAL;
    if (n_samples >= (1ull << 31) || max_dumps == 0 || (n_samples > 0 && !samples))
        return GC_EINVAL;
    if (plan->carrier != GC_CARRIER_LUT || plan->fmt == GC_I2_IQ) return GC_EINVAL;
    const gc_loop_params& q = *params;
    if (!(q.fs_hz > 0.0) || !(q.dll_bw_hz > 0.0) || !(q.dll_zeta > 0.0) || !(q.dll_gain > 0.0) ||
        !(q.pll_bw_hz > 0.0) || !(q.pll_zeta > 0.0) || !(q.pll_gain > 0.0) || !(q.fll_bw_hz >= 0.0))
        return GC_EINVAL;
    gc::TrackConsts c;
    c.fs = q.fs_hz;
    c.if_hz = q.if_hz;
    c.dll_bw = q.dll_bw_hz;
    c.dll_zeta = q.dll_zeta;
    c.dll_k = q.dll_gain;
    c.pll_bw = q.pll_bw_hz;
    c.pll_zeta = q.pll_zeta;
    c.pll_k = q.pll_gain;
    c.fll_bw = q.fll_bw_hz;
    // the CORDIC angles atan(2^-i) in units of 2^-30 rad, rounded to nearest
    for (int i = 0; i < gc::kCordicSteps; ++i)
        c.tab[i] = llround(atan(ldexp(1.0, -i)) * 1073741824.0);
    DeviceGuard g(plan->ctx->device);
    if (!g.ok) return GC_EDEVICE;
    return from_hip(gc::launch_track((const uint8_t*)samples, n_samples, plan->fmt, plan->d_chans,
                                     state, loop, c, plan->n_chan, rows, dump_n, n_dumps, status,
                                     max_dumps, plan->ctx->d_tables, (hipStream_t)stream));
}

gc_status gc_lock_metrics(gc_ctx* ctx, const int32_t* rows, int32_t row_stride,
                          int32_t prompt_col, const uint32_t* n_dumps, int32_t n_chan,
                          uint32_t max_dumps, uint32_t window, double dump_s, double lock_min,
                          const uint32_t* phase, double* cn0, double* lock, uint32_t max_windows,
                          uint32_t* n_windows, uint32_t* lock_fails, uint32_t* hist,
                          uint32_t* edge, uint8_t* bits, uint32_t max_bits, uint32_t* n_bits,
                          void* stream) {
    if (!ctx || !rows || !n_dumps || !n_windows || !lock_fails || !hist || !edge || !n_bits)
        return GC_EINVAL;
    if (n_chan < 1 || n_chan > GC_MAX_CHANNELS || max_dumps == 0 || window < 2 ||
        !(dump_s > 0.0) || row_stride < 2 || prompt_col < 0 || prompt_col + 1 >= row_stride ||
        (max_windows > 0 && (!cn0 || !lock)) || (max_bits > 0 && !bits))
        return GC_EINVAL;
    DeviceGuard g(ctx->device);
    if (!g.ok) return GC_EDEVICE;
    return from_hip(gc::launch_lock_metrics(rows, row_stride, prompt_col, n_dumps, n_chan,
                                            max_dumps, window, dump_s, lock_min, phase, cn0,
                                            lock, max_windows, n_windows, lock_fails, hist, edge,
                                            bits, max_bits, n_bits, (hipStream_t)stream));
}

gc_status gc_correlate(gc_plan* plan, const void* samples, uint64_t n_samples,
                       gc_chan_state* state, void* out, uint32_t* dump_n, uint32_t* n_dumps,
                       int32_t* status, uint32_t max_dumps, void* stream) {
    if (!plan || !state || !out || !dump_n || !n_dumps || !status) return GC_EINVAL;
    if (n_samples >= (1ull << 31) || max_dumps == 0) return GC_EINVAL;
    if (n_samples > 0 && !samples) return GC_EINVAL;
    DeviceGuard g(plan->ctx->device);
    if (!g.ok) return GC_EDEVICE;
    const size_t slot = plan->ev_stop.empty() ? 0 : (size_t)(plan->calls % plan->ev_stop.size());
    const bool timed = !plan->ev_start.empty();
    Launches L{};
    L.fmt = plan->fmt;
    L.carrier = plan->carrier;
    L.n_chan = plan->n_chan;
    L.tap_stride = plan->max_taps;
    L.periodic = plan->use_epl && (plan->kernels & GC_KERNEL_PERIODIC) &&
                 !gc::fmt_complex(plan->fmt) && plan->carrier == GC_CARRIER_LUT;
    L.binned = plan->use_epl && (plan->kernels & GC_KERNEL_BINNED);
    L.mtap = plan->use_mtap && (plan->kernels & GC_KERNEL_MTAP);
    L.grid = plan->epl_grid;
    L.chans = plan->d_chans;
    L.meta = plan->d_meta;
    L.tables = plan->ctx->d_tables;
    L.ev_start = timed ? plan->ev_start[slot] : nullptr;
    L.ev_mid = timed ? plan->ev_mid[slot] : nullptr;
    L.ev_stop = timed ? plan->ev_stop[slot] : nullptr;
    const hipError_t e = run_correlation(L, samples, n_samples, state, out, dump_n, n_dumps,
                                         status, max_dumps, (hipStream_t)stream);
    if (e == hipSuccess && timed) plan->ev_used[slot] = 1;
    plan->calls++;
    return from_hip(e);
}

gc_status gc_correlate_noalloc(gc_ctx* ctx, gc_format fmt, gc_carrier carrier,
                               const gc_chan_cfg* cfg, int32_t n_chan, int32_t tap_stride,
                               const void* samples, uint64_t n_samples, gc_chan_state* state,
                               void* out, uint32_t* dump_n, uint32_t* n_dumps, int32_t* status,
                               uint32_t max_dumps, void* stream) {
    if (!ctx || !cfg || !state || !out || !dump_n || !n_dumps || !status) return GC_EINVAL;
    if (fmt != GC_I8_REAL && fmt != GC_I8_IQ && fmt != GC_I2_REAL && fmt != GC_I2_IQ)
        return GC_EINVAL;
    if (carrier != GC_CARRIER_LUT && carrier != GC_CARRIER_F32) return GC_EINVAL;
    if (n_chan < 1 || n_chan > GC_NOALLOC_MAX_CHANNELS) return GC_EINVAL;
    if (tap_stride < 1 || tap_stride > GC_MAX_TAPS) return GC_EINVAL;
    if (n_samples >= (1ull << 31) || max_dumps == 0) return GC_EINVAL;
    if (n_samples > 0 && !samples) return GC_EINVAL;
    if (!ctx->d_scratch) return GC_EDEVICE;
    DeviceGuard g(ctx->device);
    if (!g.ok) return GC_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    // the kernel families a plan with these channels would use: tap_stride
    // stands for the plan's largest n_taps
    const bool use_epl = tap_stride <= 4;
    Launches L{};
    L.fmt = fmt;
    L.carrier = carrier;
    L.n_chan = n_chan;
    L.tap_stride = tap_stride;
    L.periodic = use_epl && !gc::fmt_complex(fmt) && carrier == GC_CARRIER_LUT;
    L.binned = use_epl;
    L.mtap = carrier == GC_CARRIER_LUT && !use_epl;
    L.grid = ctx->n_cu;
    L.chans = reinterpret_cast<gc::DevChan*>(ctx->d_scratch);
    L.meta = reinterpret_cast<gc::DevMeta*>(ctx->d_scratch + kNoallocChanBytes);
    L.tables = ctx->d_tables;
    hipError_t e = gc::launch_fill_chans(cfg, n_chan, tap_stride, L.chans, s);
    if (e == hipSuccess)
        e = run_correlation(L, samples, n_samples, state, out, dump_n, n_dumps, status,
                            max_dumps, s);
    return from_hip(e);
}

}  // extern "C"
