/*
 * gnsscorr.h -- C ABI of libgnsscorr, a GPS L1 C/A software correlator for
 * AMD Instinct MI355X (gfx950).
 *
 * The library implements the tracking correlator of a GPS software receiver:
 * per channel, carrier wipe-off, C/A code replica generation and a
 * multiply-accumulate per replica tap (early / prompt / late, or many taps),
 * integrated over code-epoch-aligned dumps.  This is the part of the
 * receiver that Schmidt & Akopian ("Exploiting Acceleration Features of
 * LabVIEW platform for Real-Time GNSS Software Receiver Optimization")
 * accelerate with SIMD software correlators (Sec. 3.7, Table 4) and that
 * dominates tracking time (Sec. 3.5).  Their tracking call takes the raw
 * sample block, its size, the system parameters and the array of channel
 * parameter clusters by reference (Sec. 3.4) and processes channels
 * independently (Sec. 3.5); this ABI keeps that shape:
 *
 *   system parameters   -> gc_format + the NCO words derived from fs and IF
 *   channel clusters    -> gc_chan_cfg (static) + gc_chan_state (in/out)
 *   raw block + size    -> device sample pointer + n_samples
 *
 * Conventions (the paper is silent on all of them; these are this
 * library's definitions, reproduced bit for bit by its test oracle):
 *   - C/A code: IS-GPS-200 Sec. 3.2.1.3 / Table 3-Ia; logic 0 -> +1,
 *     logic 1 -> -1 (Sec. 3.1 says only that chips are +1 and -1).
 *   - Carrier NCO: 32-bit phase word Phi (cycles * 2^32); Phi_n = Phi_0 +
 *     n*dPhi mod 2^32.  Table index l = Phi_n >> 24; the table holds
 *     round(24*cos(2*pi*(l+1/2)/256)) and round(24*sin(...)) (GC_LUT_AMP).
 *   - Wipe-off multiplies by exp(-j*theta): real x gives (x*c, -x*s);
 *     complex (xI, xQ) gives (xI*c + xQ*s, xQ*c - xI*s).
 *   - Code NCO: 64-bit phase U in Q32.32 chips, U_n = U_0 + n*dU; tap k
 *     uses chip floor((U_n + tap_q32[k]) / 2^32) mod 1023.  Positive
 *     offsets lead the prompt (early).
 *   - Dumps: a dump integrates int_periods code periods (window W =
 *     int_periods*1023*2^32 of code phase) and starts at a code epoch (Sec.
 *     4 uses 1 ms = one period).  Sample n belongs to window
 *     floor(U_n / W).  A dump is emitted once the code phase reached at the
 *     end of the block (U_N) has passed its end; the open dump is carried in
 *     gc_chan_state, so any split of a stream into blocks gives identical
 *     dumps.
 *   - Sample formats: GC_I8_REAL one int8 per sample; GC_I8_IQ int8 I then
 *     Q; GC_I2_REAL four samples per byte, sample j in bits [2j, 2j+1],
 *     value codes 0,1,2,3 -> -3,-1,+1,+3; GC_I2_IQ the same packing of the
 *     interleaved stream I0 Q0 I1 Q1 ..., two samples per byte, sample j's
 *     I in bits [4j, 4j+1] and its Q in bits [4j+2, 4j+3] (offline mode's
 *     recordings of I or I-Q samples, Sec. 3).
 *   - Integer path results are exact int32; a channel whose dump could
 *     leave int32 is refused (GC_ERANGE), never wrapped.
 *
 * Memory: every pointer named "device" is HIP device memory (e.g. a torch
 * tensor's data_ptr) owned by the caller and kept alive until the stream
 * reaches the call.  Calls are asynchronous and stream-ordered unless they
 * say otherwise.  A context or plan may be used from one host thread at a
 * time.  No call throws; all return gc_status.
 */
#ifndef GNSSCORR_H
#define GNSSCORR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GC_VERSION_MAJOR 1
#define GC_VERSION_MINOR 0
#define GC_LUT_BITS 8
#define GC_LUT_AMP 24
#define GC_CODE_LEN 1023
#define GC_MAX_TAPS 128
#define GC_MAX_CHANNELS 65536

typedef enum {
    GC_OK = 0,
    GC_EINVAL = -1,  /* bad argument: null pointer, PRN, format, taps, sizes */
    GC_ENOMEM = -2,  /* device or host allocation failed */
    GC_EDEVICE = -3, /* HIP runtime error */
    GC_ERANGE = -4,  /* a dump could leave int32 (bound on samples per dump) */
    GC_EBUSY = -5,   /* admission refused: over the HBM budget */
    GC_EAGAIN = -6,  /* result not ready yet */
    GC_ENOSPC = -7   /* more dumps close in this block than max_dumps */
} gc_status;

typedef enum { GC_I8_REAL = 0, GC_I8_IQ = 1, GC_I2_REAL = 2, GC_I2_IQ = 3 } gc_format;

typedef enum {
    GC_CARRIER_LUT = 0, /* integer NCO + sin/cos table, exact int32 results */
    GC_CARRIER_F32 = 1  /* FP32 sin/cos carrier, float results (FP64 block start phases) */
} gc_carrier;

typedef struct gc_ctx gc_ctx;
typedef struct gc_plan gc_plan;

/* Static part of one channel (the paper's per-channel cluster, Sec. 3.4). */
typedef struct {
    int32_t prn;                  /* satellite PRN, 1..32 */
    int32_t n_taps;               /* 1..GC_MAX_TAPS */
    int32_t int_periods;          /* code periods per dump, >= 1 */
    int32_t reserved;             /* must be 0 */
    int64_t tap_q32[GC_MAX_TAPS]; /* replica offsets from prompt, Q32 chips, |offset| < 2^40 */
} gc_chan_cfg;

/* Dynamic part of one channel, in/out for every call (device memory).
 * The layout is part of the ABI (size 2096 bytes, 8-byte aligned). */
typedef struct {
    uint64_t code_phase;   /* Q32.32 chips, in [0, W) */
    uint64_t code_step;    /* Q32.32 chips per sample, 1 .. 2^31-1 (>= 2 samples/chip) */
    uint32_t carr_phase;   /* cycles * 2^32 (GC_CARRIER_LUT) */
    uint32_t carr_step;    /* cycles * 2^32 per sample, two's complement */
    uint32_t acc_n;        /* samples in the open dump */
    uint32_t flags;        /* reserved, 0 */
    double carr_phase_f;   /* cycles in [0, 1) (GC_CARRIER_F32) */
    double carr_freq_f;    /* cycles per sample (GC_CARRIER_F32) */
    int32_t acc[GC_MAX_TAPS][2];   /* open dump I, Q per tap (GC_CARRIER_LUT) */
    float acc_f[GC_MAX_TAPS][2];   /* open dump I, Q per tap (GC_CARRIER_F32) */
} gc_chan_state;

/* Text of a status code.  Never NULL. */
const char* gc_strerror(gc_status s);

/* Library version (GC_VERSION_MAJOR/MINOR of the built library). */
gc_status gc_version(int32_t* major, int32_t* minor);

/* Create a context on HIP device `device`: selects the device, generates the
 * G1/G2 register sequences of IS-GPS-200 Sec. 3.2.1.3 on the GPU and keeps
 * them in device memory.  Synchronous.  *out is owned by the caller and
 * released with gc_destroy.  Errors: GC_EINVAL (null out, bad device),
 * GC_EDEVICE, GC_ENOMEM. */
gc_status gc_create(gc_ctx** out, int32_t device);

/* Release a context and everything it owns.  Plans made from it must be
 * destroyed first.  Synchronous (waits for the device). */
gc_status gc_destroy(gc_ctx* ctx);

/* Host helper: NCO words for one channel from physical parameters, into a
 * host gc_chan_state with empty open dump (Sec. 3.1: code-phase alignment
 * and carrier wipe-off are the correlator's inputs).
 *   carr_step  = round_half_even(carr_hz / fs_hz * 2^32) mod 2^32
 *   carr_phase = round_half_even(frac(carr_phase_cyc) * 2^32) mod 2^32
 *   code_step  = round_half_even(code_rate_cps / fs_hz * 2^32)
 *   code_phase = round_half_even((code_phase_chips mod W') * 2^32) mod W,
 *                W' = int_periods*1023 chips
 *   carr_phase_f = frac(carr_phase_cyc), carr_freq_f = carr_hz / fs_hz
 * Errors: GC_EINVAL (null out, fs <= 0, rate <= 0, int_periods < 1, or a
 * code step outside 1 .. 2^31-1). */
gc_status gc_nco_init(double fs_hz, double carr_hz, double carr_phase_cyc,
                      double code_rate_cps, double code_phase_chips,
                      int32_t int_periods, gc_chan_state* out);

/* C/A code of one PRN as generated on the GPU (G1 XOR delayed G2, IS-GPS-200
 * Table 3-Ia), copied to host: out[i] in {+1, -1}, i = 0..1022.
 * Synchronous.  Errors: GC_EINVAL (prn, null), GC_EDEVICE. */
gc_status gc_code_table(gc_ctx* ctx, int32_t prn, int8_t* host_out);

/* The stated error of the float carrier (GC_CARRIER_F32).  Its kernels
 * compute each sample's phase in cycles in fp32, reduced to [0, 1), from a
 * start phase computed in fp64, and take cos and sin of 2*pi*phase with the
 * GPU's sine and cosine instructions (argument in revolutions).  This call
 * evaluates that same sin/cos routine on the GPU for every fp32 phase whose
 * bit pattern lies in first_bits .. first_bits + count - 1 and returns the
 * largest absolute error against cos and sin in double precision:
 * host_err[0] for cos, host_err[1] for sin.  All 1,065,353,216 fp32 values
 * in [0, 1) are bit patterns 0 .. 0x3F7FFFFF.  Synchronous.
 * Errors: GC_EINVAL (null, count 0, a bit pattern at or above that of 1.0f),
 * GC_ENOMEM, GC_EDEVICE. */
gc_status gc_carrier_f32_error(gc_ctx* ctx, uint32_t first_bits, uint32_t count,
                               double* host_err);

/* Build a plan for a fixed set of channels that share one sample stream
 * (one receiver; channels run independently as in Sec. 3.5).  Validates
 * every cfg on the host, uploads them to device memory (synchronous) and
 * chooses kernels.  fmt and carrier apply to every channel of the plan.
 * *out is released with gc_plan_destroy.
 * Errors: GC_EINVAL (null, n_chan outside 1..GC_MAX_CHANNELS, fmt, carrier,
 * prn outside 1..32, n_taps outside 1..GC_MAX_TAPS, int_periods < 1,
 * reserved != 0, tap offset out of range), GC_ENOMEM, GC_EDEVICE. */
gc_status gc_plan_create(gc_ctx* ctx, gc_format fmt, gc_carrier carrier,
                         const gc_chan_cfg* cfg, int32_t n_chan, gc_plan** out);

/* Release a plan (waits for the device). */
gc_status gc_plan_destroy(gc_plan* plan);

/* Kernel families a plan may use for its E/P/L channels (bit mask).  Every
 * family computes the same integer sums (the definition of Eqs. (1)-(3)
 * with the table carrier; with the float carrier, sums within the stated
 * bound); the choice only changes speed.
 *   GC_KERNEL_PERIODIC  half chips of exactly 2, 4, 8 or 10 samples with a
 *                       bounded grid slip (fs an integer multiple of twice the
 *                       code rate), real input, table carrier
 *   GC_KERNEL_BINNED    any rate of >= 2^32/127 code step, chip by chip
 *                       (table or float carrier)
 *   GC_KERNEL_MTAP      plans with more than 4 taps: channels whose taps are
 *                       all multiples of 2^27 (1/32 chip) spanning at most 8
 *                       chip shifts, at <= 32 samples per chip (two-stage
 *                       int8 MFMA form, table carrier)
 * Channels that no allowed family takes, and every channel of a float-carrier
 * plan with more than 4 taps, use the direct per-sample kernel.  Default: all bits
 * set.  Takes effect at the next gc_correlate.
 * Errors: GC_EINVAL (null plan, bits outside the mask). */
#define GC_KERNEL_PERIODIC 1
#define GC_KERNEL_BINNED 2
#define GC_KERNEL_MTAP 4
gc_status gc_plan_set_kernels(gc_plan* plan, int32_t mask);

/* Query: taps per dump row in the output layout (the largest n_taps of the
 * plan's channels) and the number of channels. */
gc_status gc_plan_info(const gc_plan* plan, int32_t* tap_stride, int32_t* n_chan);

/* Correlate one block of samples for every channel of the plan.
 *
 *   samples   device, the block in the plan's format; n_samples samples
 *             (n_samples bytes, 2*n_samples bytes, ceil(n_samples/4) bytes or
 *             ceil(n_samples/2) bytes), starting on a 16-byte boundary (the
 *             kernels read it in aligned words of 4 to 16 bytes)
 *   n_samples 0 .. 2^31-1
 *   state     device, gc_chan_state[n_chan], read and updated in place:
 *             NCO phases advance by n_samples, the open dump is carried
 *   out       device, [n_chan][max_dumps][tap_stride][2] of int32 (LUT) or
 *             float (F32): I then Q of each tap of each dump closed here
 *   dump_n    device, uint32 [n_chan][max_dumps]: samples in each dump
 *             (including samples of the open dump from earlier blocks)
 *   n_dumps   device, uint32 [n_chan]: dumps closed by this block
 *   status    device, int32 [n_chan]: GC_OK, or per channel GC_EINVAL
 *             (state out of range: code_phase >= W or code_step not in
 *             1..2^31-1), GC_ENOSPC (more than max_dumps would close),
 *             GC_ERANGE (int32 bound: (floor((W-1)/code_step)+1) * max|w| must
 *             stay below 2^31, max|w| = 24*max|x| real, 34*max|x| complex);
 *             a refused channel's state and outputs are left untouched and
 *             its n_dumps is 0
 *   max_dumps rows per channel in out and dump_n
 *   stream    hipStream_t, or NULL for the default stream
 *
 * Asynchronous: returns once the work is enqueued.  Rows past n_dumps[c]
 * are left as they were.  Errors returned directly: GC_EINVAL (null
 * pointers, n_samples too large, max_dumps == 0), GC_EDEVICE. */
gc_status gc_correlate(gc_plan* plan, const void* samples, uint64_t n_samples,
                       gc_chan_state* state, void* out, uint32_t* dump_n,
                       uint32_t* n_dumps, int32_t* status, uint32_t max_dumps,
                       void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * correlation as gc_correlate without a plan.  The per-channel kernel
 * records and the per-call set-up values that a plan keeps in its own
 * device buffers live instead in one fixed array of the library, one per
 * GPU, reserved when the library is loaded and held until the process ends
 * (GC_NOALLOC_MAX_CHANNELS channels); this call allocates nothing, on the
 * device or the host.
 *
 *   cfg        DEVICE, gc_chan_cfg[n_chan] (the caller's copy; read by the
 *              call's first kernel, so it may be reused once the stream has
 *              passed the call)
 *   n_chan     1 .. GC_NOALLOC_MAX_CHANNELS
 *   tap_stride taps per output row, 1 .. GC_MAX_TAPS; it also picks the
 *              kernels as a plan's largest n_taps does (<= 4: the E/P/L
 *              kernels, the periodic one only with the table carrier; more:
 *              the multi-tap and direct kernels, the direct kernel alone
 *              with the float carrier)
 *   the rest   as for gc_correlate, with the plan's format and carrier given
 *              here
 * A channel whose cfg a plan would refuse (PRN, n_taps, int_periods,
 * reserved, tap offsets) or with n_taps > tap_stride gets status GC_EINVAL
 * and is left untouched, like a channel with a bad state.  Every call on
 * one GPU shares that GPU's array: calls that overlap on the device (two
 * streams, or two host threads) race and give wrong results; calls ordered
 * on one stream are safe, each rewrites what it uses.
 * Errors returned directly: GC_EINVAL (null pointers, fmt, carrier, n_chan
 * above GC_NOALLOC_MAX_CHANNELS or below 1, tap_stride, n_samples,
 * max_dumps == 0), GC_EDEVICE. */
#define GC_NOALLOC_MAX_CHANNELS 1024
gc_status gc_correlate_noalloc(gc_ctx* ctx, gc_format fmt, gc_carrier carrier,
                               const gc_chan_cfg* cfg, int32_t n_chan, int32_t tap_stride,
                               const void* samples, uint64_t n_samples, gc_chan_state* state,
                               void* out, uint32_t* dump_n, uint32_t* n_dumps, int32_t* status,
                               uint32_t max_dumps, void* stream);

/* Per-launch timing of the plan's main correlation kernel (the paper reports
 * tracking time per epoch per channel, Sec. 4, Table 5).  A call runs up to
 * two correlation kernels after its set-up (which one takes a channel is
 * decided on the device); with n_slots > 0, every later gc_correlate records
 * HIP events on its stream before, between and after them into slot (call
 * index mod n_slots); n_slots = 0 turns timing off.  At most 4096 slots.
 * Synchronous set-up.  Errors: GC_EINVAL, GC_ENOMEM, GC_EDEVICE. */
gc_status gc_plan_timing(gc_plan* plan, int32_t n_slots);

/* Duration in milliseconds of the longer of the two correlation kernels
 * timed in `slot` (the one that did the work); waits for its stop event.
 * Errors: GC_EINVAL (timing off, slot out of range or never recorded),
 * GC_EDEVICE. */
gc_status gc_plan_kernel_ms(gc_plan* plan, int32_t slot, float* ms);

/* ------------------------------------------------------------------------
 * Closed tracking loops (Table 3).
 *
 * gc_track runs the E/P/L correlator dump by dump and closes the tracking
 * loops of every channel after each dump: a 2nd-order DLL with the
 * normalised early-minus-late envelope discriminator (|E| - |L|) / (|E| +
 * |L|) and carrier aiding, and a 2nd-order PLL with the atan(Q_P / I_P)
 * discriminator assisted by a 1st-order FLL with an atan2 discriminator on
 * consecutive prompts (cross and dot products, the dot product's sign
 * removed so that navigation-bit flips do not count as frequency).  Loop
 * filter (softGNSS form): wn = B 8 z / (4 z^2 + 1), tau1 = k / wn^2, tau2 =
 * 2 z / wn, nco += (tau2 / tau1)(e - e_prev) + e T / tau1 with T the dump
 * length; the FLL adds 4 B_f T times its error (Hz) to the frequency basis.
 * Carrier = basis + PLL nco; code = 1.023 MHz (1 + (carrier - IF) /
 * 1575.42 MHz) + DLL nco; the new steps are round_half_even(f / fs 2^32)
 * and apply from the next dump.  Angles come from a 31-step vectoring
 * CORDIC on the integer dumps in units of 2^-30 rad; every other step is a
 * correctly rounded double operation, so results are reproducible bit for
 * bit.  A dump closes when the code phase reaches the window end, before
 * the next sample or at the end of the block, so any split of a stream into
 * blocks gives the same dumps and loop states.
 * ------------------------------------------------------------------------ */
typedef struct {
    double fs_hz;      /* sample rate */
    double if_hz;      /* carrier frequency of zero Doppler */
    double dll_bw_hz;  /* DLL noise bandwidth, damping ratio, gain (2, 0.7, 1) */
    double dll_zeta;
    double dll_gain;
    double pll_bw_hz;  /* PLL noise bandwidth, damping ratio, gain (25, 0.7, 0.25) */
    double pll_zeta;
    double pll_gain;
    double fll_bw_hz;  /* FLL noise bandwidth (10) */
} gc_loop_params;

/* Per-channel loop state, in/out for every gc_track call (device memory).
 * Layout fixed: 72 bytes. */
typedef struct {
    double carr_hz;        /* carrier NCO frequency */
    double code_cps;       /* code NCO rate, chips/s */
    double fll_basis_hz;   /* FLL frequency basis */
    double pll_nco_hz;     /* PLL filter output */
    double pll_err_prev;   /* previous PLL error, cycles */
    double dll_nco_cps;    /* DLL filter output, chips/s */
    double dll_err_prev;   /* previous DLL error */
    int32_t prompt_i_prev; /* prompt of the previous closed dump */
    int32_t prompt_q_prev;
    int32_t have_prev;     /* 1 once a dump has closed */
    int32_t reserved;      /* 0 */
} gc_loop_state;

/* Host helper: a loop state starting at carrier carr_hz and code rate
 * code_cps (the same values gc_nco_init turned into the channel's NCO
 * words), filters at rest.  Errors: GC_EINVAL (null out). */
gc_status gc_loop_init(double carr_hz, double code_cps, gc_loop_state* out);

/* Track one block: like gc_correlate for the plan's channels, each an E/P/L
 * channel (3 taps at +1/2, 0, -1/2 chip; others get GC_EINVAL), with the
 * loops closed after every dump.
 *   params  host, the loop parameters (by value at the call)
 *   state   device, gc_chan_state[n_chan] in/out (NCO words, open dump)
 *   loop    device, gc_loop_state[n_chan] in/out
 *   rows    device, int32 [n_chan][max_dumps][8]: per closed dump E I, E Q,
 *           P I, P Q, L I, L Q and the carrier and code steps used for it
 *           (their bit patterns)
 *   dump_n, n_dumps, status, max_dumps: as for gc_correlate
 * Per-channel status: GC_OK; GC_EINVAL (not an E/P/L channel, phase outside
 * the window); GC_ERANGE (a code step, given or set by the loops, outside
 * 1 .. 2^31-1 or letting a dump leave int32); GC_ENOSPC.  A channel with an
 * error keeps its state and loop state.  The plan must use GC_CARRIER_LUT
 * and a format other than GC_I2_IQ (GC_EINVAL).
 * Errors returned directly: GC_EINVAL, GC_EDEVICE. */
gc_status gc_track(gc_plan* plan, const void* samples, uint64_t n_samples,
                   const gc_loop_params* params, gc_chan_state* state, gc_loop_state* loop,
                   int32_t* rows, uint32_t* dump_n, uint32_t* n_dumps, int32_t* status,
                   uint32_t max_dumps, void* stream);

/* ------------------------------------------------------------------------
 * Lock metrics and bit synchronisation (Sec. 3.6, channel health; Sec. 3.1,
 * 20 code periods per navigation bit), over the closed dumps of channels.
 *
 * Channel c's dump k has its prompt I and Q at
 *   rows[(c * max_dumps + k) * row_stride + prompt_col]  and  [... + 1],
 * k = 0 .. min(n_dumps[c], max_dumps) - 1, one code period per dump (so
 * gc_track's rows with row_stride 8, prompt_col 2, or gc_correlate's out with
 * row_stride 2 * tap_stride and prompt_col 2 * the prompt tap).
 *
 * C/N0 per window of `window` consecutive dumps by the moments (M2M4)
 * estimator: with P = I^2 + Q^2, M2 = mean P, M4 = mean P^2, A = sqrt(2 M2^2
 * - M4), C/N0 = 10 log10(A / (M2 - A) / dump_s) dB-Hz, NaN where 2 M2^2 - M4
 * <= 0 or M2 <= A.  Carrier lock ratio per window (the estimate of cos 2x
 * the phase error): sum(I^2 - Q^2) / sum(I^2 + Q^2), 0 for an all-zero
 * window; a window below lock_min counts as a lock failure.  Bit edge: each
 * sign change of prompt I from dump k-1 to dump k (zero counts as positive)
 * adds one to histogram position (k + phase[c]) mod 20; the edge is the
 * position with the most counts, the lowest on ties.  Bit j sums I over the
 * 20 dumps of the j-th whole period that starts at an edge position and is
 * 1 when the sum is negative.
 *
 *   rows, n_dumps         device, as above
 *   phase                 device, uint32 [n_chan], position of dump 0 in the
 *                         20-dump cycle, or NULL for 0
 *   cn0, lock             device, double [n_chan][max_windows] (may be NULL
 *                         when max_windows is 0)
 *   n_windows             device, uint32 [n_chan]: windows written,
 *                         min(n / window, max_windows)
 *   lock_fails            device, uint32 [n_chan]: failures over all n /
 *                         window windows
 *   hist                  device, uint32 [n_chan][20]
 *   edge                  device, uint32 [n_chan]
 *   bits                  device, uint8 [n_chan][max_bits] (0 or 1)
 *   n_bits                device, uint32 [n_chan]: bits written (at most
 *                         max_bits)
 * Sums are fp64 in dump order, so results match a sequential double
 * evaluation exactly apart from the last bits of log10.  Errors: GC_EINVAL
 * (null pointers, n_chan outside 1 .. GC_MAX_CHANNELS, window < 2, dump_s
 * <= 0, prompt_col + 1 >= row_stride), GC_EDEVICE.
 * ------------------------------------------------------------------------ */
gc_status gc_lock_metrics(gc_ctx* ctx, const int32_t* rows, int32_t row_stride,
                          int32_t prompt_col, const uint32_t* n_dumps, int32_t n_chan,
                          uint32_t max_dumps, uint32_t window, double dump_s, double lock_min,
                          const uint32_t* phase, double* cn0, double* lock, uint32_t max_windows,
                          uint32_t* n_windows, uint32_t* lock_fails, uint32_t* hist,
                          uint32_t* edge, uint8_t* bits, uint32_t max_bits, uint32_t* n_bits,
                          void* stream);

/* ------------------------------------------------------------------------
 * Acquisition (Sec. 3.3: the ACQ module searches a buffer of whole code
 * periods for the satellites to track; Sec. 3.7: FFT-based search).
 *
 * A parallel code-phase search over Doppler bins and PRNs, computed exactly
 * in integers.  The buffer holds `blocks` blocks of `coherent_periods` code
 * periods at R = samples_per_chip samples per chip (fs = R * 1.023 MHz, N =
 * 1023 R samples per period).  Bin d has the carrier frequency if_hz +
 * (f_lo_hz + d * f_step_hz) and the NCO step round_half_even(f / fs * 2^32)
 * mod 2^32.  Its phase is 0 at sample 0 of the buffer and runs on across
 * blocks.  The wipe-off uses the correlator's carrier table.  At code phase
 * tau (0 <= tau < N samples), sample n meets chip floor((n + tau) / R) mod
 * 1023 of the PRN's code.  For each block the kernel forms the complex sum
 * Y of wiped-off sample times chip over the block, and the power is
 *   P[p][d][tau] = sum over blocks of (Y_I^2 + Y_Q^2)     (uint64, exact).
 * Detection per PRN: the peak is the largest P; ties go to the lower bin,
 * then the lower tau.  The second peak is the largest P in the peak's bin
 * over the chips floor(tau / R) at least two chips (circularly) from the
 * peak's chip.  metric = peak / second in double (+inf when second is 0),
 * and the PRN counts as acquired when metric >= threshold.
 * ------------------------------------------------------------------------ */
#define GC_ACQ_MAX_SPC 32     /* samples per chip */
#define GC_ACQ_MAX_BINS 1024
#define GC_ACQ_MAX_PRNS 1024

typedef struct gc_acq gc_acq;

/* One PRN's detection (device memory, written by gc_acquire).  Layout
 * fixed: 56 bytes. */
typedef struct {
    int32_t prn;
    int32_t bin;              /* Doppler bin of the peak */
    int32_t tau;              /* code phase of the peak, samples */
    int32_t acquired;         /* 1 when metric >= threshold */
    uint64_t peak;            /* P at the peak */
    uint64_t second;          /* second peak (see above) */
    double doppler_hz;        /* f_lo_hz + bin * f_step_hz */
    double code_phase_chips;  /* tau / R: code phase at sample 0 of the buffer */
    double metric;            /* peak / second */
} gc_acq_result;

/* A search plan: validates the bounds, computes the bin steps and allocates
 * the device scratch (gc_acq_info reports its size).
 *   fmt                  sample format of the buffer (GC_I2_IQ is refused)
 *   samples_per_chip     R, 1 .. GC_ACQ_MAX_SPC
 *   prns                 host, n_prn PRN numbers 1..32 (repeats allowed)
 *   coherent_periods     Mc, 1 .. 1000
 *   blocks               Knc, 1 .. 1000 (non-coherent sum)
 * The bounds on the exact integer arithmetic: Mc * R * max|w| < 2^28, where
 * max|w| is 72 for 2-bit, 3072 for int8 real and 4352 for int8 I/Q, and
 * Knc * 2 * (Mc * N * max|w|)^2 < 9.0e18.
 * Errors: GC_EINVAL (null pointers, values out of range, bounds),
 * GC_ENOMEM, GC_EDEVICE. */
gc_status gc_acq_create(gc_ctx* ctx, gc_format fmt, int32_t samples_per_chip, double if_hz,
                        double f_lo_hz, double f_step_hz, int32_t n_bins, const int32_t* prns,
                        int32_t n_prn, int32_t coherent_periods, int32_t blocks, gc_acq** out);

/* Run the search on the first Knc * Mc * N samples of a device buffer.
 *   samples    device, at least that many samples
 *   surface    device, uint64 [n_prn][n_bins][N] power, or NULL
 *   results    device, gc_acq_result[n_prn]
 * Calls on one plan share its scratch: run them in one stream.
 * Errors: GC_EINVAL (null, too few samples), GC_EDEVICE. */
gc_status gc_acquire(gc_acq* acq, const void* samples, uint64_t n_samples, double threshold,
                     uint64_t* surface, gc_acq_result* results, void* stream);

/* Query (any pointer may be NULL): int8 digits per box sum (2 or 4), device
 * scratch bytes, samples a call reads, operand rows per block of the
 * contraction (96 or 128, chosen at creation for the fewest rows in the
 * last round of blocks).  Errors: GC_EINVAL. */
gc_status gc_acq_info(gc_acq* acq, int32_t* digits, uint64_t* scratch_bytes,
                      uint64_t* samples_needed, int32_t* row_tile);

/* Per-kernel timing of gc_acquire: with n_slots > 0 every later call records
 * HIP events on its stream before and after each of its four kernels (box
 * sums, contraction, chip reduction, detection) into slot (call index mod
 * n_slots); 0 turns timing off.  At most 4096 slots.  Errors: GC_EINVAL,
 * GC_ENOMEM, GC_EDEVICE. */
gc_status gc_acq_timing(gc_acq* acq, int32_t n_slots);

/* The four kernel durations (ms) of `slot`; waits for its last event.
 * Errors: GC_EINVAL (timing off, slot out of range or never recorded),
 * GC_EDEVICE. */
gc_status gc_acq_kernel_ms(gc_acq* acq, int32_t slot, float* ms4);

/* Free a plan (after its last call has finished).  Errors: GC_EINVAL. */
gc_status gc_acq_destroy(gc_acq* acq);

/* ------------------------------------------------------------------------
 * Batches: many receivers in one persistent launch.
 *
 * A batch binds the sample blocks of n_rx receivers (each with its own
 * format and length) and the channels that track them (Sec. 3.5: channels
 * are independent given their receiver's samples), and correlates all of
 * them with two persistent launches: the periodic-bin E/P/L kernel over
 * (receiver, channel group, tile chunk) work items for channels whose half
 * chips span a fixed 2, 4, 8 or 10 samples, then the chip-by-chip kernel over
 * (receiver, tile) work items for the others; the per-call set-up and both
 * launches are captured once into a HIP graph and replayed by
 * gc_batch_launch.  Results
 * are those of gc_correlate on one plan per receiver, bit for bit.
 * ------------------------------------------------------------------------ */
typedef struct gc_batch gc_batch;

typedef struct {
    const void* samples;  /* device, the receiver's block in its format */
    uint64_t n_samples;   /* 0 .. 2^31-1 */
    int32_t fmt;          /* GC_I8_REAL, GC_I8_IQ or GC_I2_REAL */
    int32_t reserved;     /* must be 0 */
} gc_rx_desc;

/* Bind a batch.
 *   rx[n_rx]      receivers (host array; the sample pointers are device
 *                 pointers that must stay valid while the batch is used)
 *   cfg[n_chan]   channel configurations, at most 4 taps each
 *   chan_rx[n_chan] receiver index of each channel, non-decreasing (the
 *                 channels of a receiver are contiguous)
 *   state, out, dump_n, n_dumps, status, max_dumps: as for gc_correlate,
 *                 device buffers owned by the caller and bound to the batch
 *                 (every launch reads and updates state in place)
 * Every launch correlates each receiver's whole block.  The default shape
 * is shape 0 with one block per compute unit until gc_batch_tune or
 * gc_batch_configure picks another.
 * Errors: GC_EINVAL (null, counts outside 1..GC_MAX_CHANNELS / 1..65536,
 * fmt, n_samples, reserved, chan_rx out of range or decreasing, a channel
 * with more than 4 taps, max_dumps == 0), GC_ENOMEM, GC_EDEVICE. */
gc_status gc_batch_create(gc_ctx* ctx, const gc_rx_desc* rx, int32_t n_rx,
                          const gc_chan_cfg* cfg, const int32_t* chan_rx, int32_t n_chan,
                          gc_chan_state* state, void* out, uint32_t* dump_n,
                          uint32_t* n_dumps, int32_t* status, uint32_t max_dumps,
                          gc_batch** out_batch);

/* Choose the chip-by-chip kernel's block shape (0 .. n_shapes-1, see
 * gc_batch_info) and number of persistent blocks (0: one per compute unit),
 * and the periodic kernel's work-item size in sample tiles (0: the default
 * of 4, -1: periodic kernel off, every channel on the chip-by-chip kernel;
 * values below 2 are raised to 2).  Drops the captured graph.
 * Errors: GC_EINVAL, GC_EDEVICE. */
gc_status gc_batch_configure(gc_batch* b, int32_t shape, int32_t grid, int32_t periodic_chunk);

/* Autotune: time every shape of the chip-by-chip kernel with 1x and 2x one
 * block per compute unit, then (unless the periodic kernel is off) periodic
 * work items of 2, 4 and 8 tiles, `reps` launches each, restoring the bound
 * channel states before every launch (the states are left as they were),
 * and keep the fastest.
 * Synchronous.  Errors: GC_EINVAL (reps outside 1..100), GC_ENOMEM,
 * GC_EDEVICE. */
gc_status gc_batch_tune(gc_batch* b, int32_t reps);

/* Enqueue one correlation of every receiver's block on `stream` (HIP
 * stream, NULL = default): replays the captured graph, capturing it first
 * when needed.  Errors: GC_EDEVICE. */
gc_status gc_batch_launch(gc_batch* b, void* stream);

/* Query: shape, grid and work items of the chip-by-chip kernel, the number
 * of shapes, the best time per launch measured by gc_batch_tune (ms, 0 when
 * not tuned), and the periodic kernel's tiles per work item (-1: off) and
 * work items.  Any output pointer may be NULL. */
gc_status gc_batch_info(const gc_batch* b, int32_t* shape, int32_t* grid, int32_t* n_items,
                        int32_t* n_shapes, float* tuned_ms, int32_t* periodic_chunk,
                        int32_t* periodic_items);

/* Release a batch (waits for the device). */
gc_status gc_batch_destroy(gc_batch* b);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of requests from many receivers.
 *
 * A server owns the channels of its registered receivers (configuration and
 * NCO state stay resident in device memory between requests, Sec. 3.5: a
 * channel continues from the state of its previous block) and a device
 * arena for request samples of hbm_budget_bytes.  A request is one sample
 * block of one receiver, given in host memory: gc_server_submit admits it
 * when its samples fit the arena and the pinned host arena, else refuses it
 * with GC_EBUSY (the caller retries after collecting results).  The
 * server's dispatcher thread keeps up to n_streams launches in flight; each
 * runs the oldest waiting request of up to max_batch_rx idle receivers
 * together (set-up and one persistent launch of the chip-by-chip E/P/L
 * kernel over all their tiles), so requests that arrive while others run
 * join the next launch.  The requests of one receiver run in submission
 * order.  Results equal those of gc_correlate on one plan per receiver
 * called once per request, bit for bit, whatever the mix.  With
 * GC_SERVER_PLAIN every request runs alone and every channel with its own
 * set-up and direct-kernel launch (the per-channel baseline).
 * Every function is thread-safe except gc_server_destroy.
 * ------------------------------------------------------------------------ */
typedef struct gc_server gc_server;

#define GC_SERVER_PLAIN 1

/* Create a server on the context's device.
 *   hbm_budget_bytes   device arena for admitted request samples (>= 4096)
 *   host_budget_bytes  pinned host arena for staged samples and results
 *   max_channels       channel capacity over all receivers (1..GC_MAX_CHANNELS)
 *   max_receivers      receiver capacity (1..65536)
 *   max_dumps          output rows per channel per request (2..4096); a
 *                      request that would close more reports GC_ENOSPC in
 *                      its channels' status
 *   n_streams          launches in flight (1..16), each on its own
 *                      default-priority HIP stream
 *   max_batch_rx       receivers per launch (1..4096)
 *   flags              0 or GC_SERVER_PLAIN
 * Errors: GC_EINVAL, GC_ENOMEM, GC_EDEVICE. */
gc_status gc_server_create(gc_ctx* ctx, uint64_t hbm_budget_bytes, uint64_t host_budget_bytes,
                           int32_t max_channels, int32_t max_receivers, uint32_t max_dumps,
                           int32_t n_streams, int32_t max_batch_rx, int32_t flags,
                           gc_server** out);

/* Register a receiver: sample format (GC_I8_REAL, GC_I8_IQ or GC_I2_REAL), n_chan
 * channel configurations with at most 4 taps each, and their initial NCO
 * states (host arrays, copied).  Its id, counted from 0, goes to *rx_id.
 * Synchronous.  Errors: GC_EINVAL (null, fmt, a configuration), GC_ENOMEM
 * (channel or receiver capacity reached), GC_EDEVICE. */
gc_status gc_server_open_rx(gc_server* s, int32_t fmt, const gc_chan_cfg* cfg,
                            const gc_chan_state* state0, int32_t n_chan, int32_t* rx_id);

/* Submit a request: n_samples (0 .. 2^31-1) samples of receiver rx_id in its
 * format, in host memory (copied before return; the buffer may be reused at
 * once).  The request id (never 0) goes to *req_id.
 * Errors: GC_EINVAL, GC_EBUSY (over the HBM or host budget: nothing was
 * queued), GC_EDEVICE (also after an earlier device error). */
gc_status gc_server_submit(gc_server* s, int32_t rx_id, const void* host_samples,
                           uint64_t n_samples, uint64_t* req_id);

/* Stop (hold = 1) or resume (hold = 0) forming launches; launches already
 * made run to completion and submissions are still admitted.  For callers
 * that submit a group of requests to run together, and for draining.
 * Errors: GC_EINVAL. */
gc_status gc_server_hold(gc_server* s, int32_t hold);

/* Collect up to max_n ids of finished requests, oldest first, into ids
 * (host); their number goes to *n_done.  Non-blocking.
 * Errors: GC_EINVAL, GC_EDEVICE (a launch failed; results are not valid). */
gc_status gc_server_poll(gc_server* s, uint64_t* ids, int32_t max_n, int32_t* n_done);

/* Copy a finished request's results to host arrays (any may be NULL) and
 * release it:
 *   out        int32 [n_chan][max_dumps][4][2]   (dump I, Q per tap slot)
 *   dump_n     uint32 [n_chan][max_dumps]
 *   n_dumps    uint32 [n_chan]
 *   status     int32 [n_chan]
 *   service_s  double [1]: seconds from submission to the host seeing the
 *              launch complete
 * with n_chan the receiver's channel count, rows as gc_correlate writes
 * them.  Errors: GC_EINVAL (unknown id), GC_EAGAIN (not finished). */
gc_status gc_server_result(gc_server* s, uint64_t req_id, int32_t* out, uint32_t* dump_n,
                           uint32_t* n_dumps, int32_t* status, double* service_s);

/* Wait until the receiver has no request queued or running, then copy its
 * channels' NCO states to host_out[n_chan].  Errors: GC_EINVAL, GC_EDEVICE. */
gc_status gc_server_state(gc_server* s, int32_t rx_id, gc_chan_state* host_out);

/* Query (any pointer may be NULL): rows per channel, tap stride (4),
 * requests admitted and not finished, device arena bytes in use, launches
 * made and requests they carried. */
gc_status gc_server_info(gc_server* s, uint32_t* max_dumps, int32_t* tap_stride,
                         int32_t* in_flight, uint64_t* hbm_in_use, uint64_t* launches,
                         uint64_t* launched_requests);

/* Host-side timing of the serving loop since creation (for latency
 * diagnostics): per launch, the time the dispatcher spent enqueueing it
 * (copies and kernel launches) and the time from the end of that enqueue to
 * the dispatcher seeing it complete; and the longest HIP-call time of a
 * submission (the sample upload).  Layout fixed: 56 bytes. */
typedef struct {
    uint64_t launches;
    uint64_t launched_requests;
    double enqueue_mean_ms;
    double enqueue_max_ms;
    double device_mean_ms;
    double device_max_ms;
    double submit_max_ms;
} gc_server_timing;

/* Errors: GC_EINVAL. */
gc_status gc_server_stats(gc_server* s, gc_server_timing* out);

/* Stop the dispatcher, wait for the device and release everything
 * (unfetched results are dropped). */
gc_status gc_server_destroy(gc_server* s);

#ifdef __cplusplus
}
#endif

#endif /* GNSSCORR_H */
