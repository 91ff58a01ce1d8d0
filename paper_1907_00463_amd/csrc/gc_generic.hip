// gc_generic.hip -- direct-form correlator kernel for any tap set.
//
// Every thread takes samples n = t0 + tid + 256*j of its block's tile and,
// for each of up to 4 taps of the block's tap group, evaluates the replica
// chip floor((U_n + delta_k) / 2^32) mod 1023 from the 64-bit code phase
// and multiply-accumulates the wiped-off sample.  It is the plain per-sample
// form of the method: the reference path for arbitrary taps and the
// "one launch, no binning" comparator for the binned kernels.
//
// Grid: x = sample tiles of kTile samples (or fewer blocks looping over the
// tiles), y = channel, z = tap group of 4.
// A tile that straddles dump boundaries is split into per-window segments;
// each segment ends in a block reduction and one atomic add per output
// word (integer atomics are order-free, so results are exact).
#include "gc_device.h"

namespace gc {

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 4096;
constexpr int kTapGroup = 4;

template <int FMT, int CARR>
__global__ __launch_bounds__(kThreads) void k_generic(const uint8_t* __restrict__ samples,
                                                      uint64_t n_samples,
                                                      const DevChan* __restrict__ chans,
                                                      const DevMeta* __restrict__ metas,
                                                      gc_chan_state* __restrict__ state,
                                                      void* __restrict__ out, int tap_stride,
                                                      uint32_t max_dumps,
                                                      const uint32_t* __restrict__ tables) {
    using acc_t = typename std::conditional<CARR == GC_CARRIER_LUT, int, float>::type;
    const int ch = blockIdx.y;
    const int tid = threadIdx.x;
    const DevMeta m = metas[ch];
    if (m.status != GC_OK || m.path == kPathMtap) return;
    const int K = chans[ch].n_taps;
    const int k0 = blockIdx.z * kTapGroup;
    if (k0 >= K) return;
    const int nk = min(kTapGroup, K - k0);
    const int d = chans[ch].g2_delay;

    __shared__ int8_t s_code[1024];
    __shared__ uint32_t s_lut[256];
    __shared__ int64_t s_taps[kTapGroup];
    __shared__ acc_t s_red[kThreads / 64][2 * kTapGroup];
    for (int i = tid; i < kCodeLen; i += kThreads) s_code[i] = ca_chip(tables, d, i);
    if (CARR == GC_CARRIER_LUT) s_lut[tid] = tables[kTabLut + tid];
    if (tid < kTapGroup) s_taps[tid] = tid < nk ? chans[ch].taps[k0 + tid] : 0;
    __syncthreads();

    const uint64_t n_tiles = (n_samples + kTile - 1) / kTile;
    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const uint64_t t0 = tile * kTile;
    const uint64_t t1 = min(n_samples, t0 + kTile);
    const uint64_t W = m.window;
    const uint64_t m_a = (m.p0 + t0 * m.dp) / W;
    const uint64_t m_b = (m.p0 + (t1 - 1) * m.dp) / W;
    int64_t tap[kTapGroup];
#pragma unroll
    for (int k = 0; k < kTapGroup; ++k) tap[k] = s_taps[k];

    for (uint64_t w = m_a; w <= m_b; ++w) {
        const uint64_t lo = max(t0, window_start(w, W, m.p0, m.dp));
        const uint64_t hi = min(t1, window_start(w + 1, W, m.p0, m.dp));
        acc_t ai[kTapGroup], aq[kTapGroup];
#pragma unroll
        for (int k = 0; k < kTapGroup; ++k) { ai[k] = 0; aq[k] = 0; }
        float ph = 0.0f, dph = 0.0f;
        if constexpr (CARR == GC_CARRIER_F32) {
            // per-thread start phase in FP64, FP32 steps of 256 samples after that
            double p = m.phf0 + (double)(lo + tid) * m.ff;
            ph = (float)(p - floor(p));
            double q = (double)kThreads * m.ff;
            dph = (float)(q - floor(q));
        }
        for (uint64_t n = lo + tid; n < hi; n += kThreads) {
            int xi, xq;
            load_sample<FMT>(samples, n, xi, xq);
            acc_t wi, wq;
            if constexpr (CARR == GC_CARRIER_LUT) {
                const uint32_t phi = m.phi0 + (uint32_t)n * m.dphi;
                int c, s;
                lut_cs(s_lut[phi >> 24], c, s);
                wipe<FMT, int>(xi, xq, c, s, wi, wq);
            } else {
                float c, s;
                carrier_f32(ph, c, s);
                wipe<FMT, float>((float)xi, (float)xq, c, s, wi, wq);
                ph += dph;
                ph -= floorf(ph);
            }
            const uint64_t u = m.p0 + n * m.dp;
#pragma unroll
            for (int k = 0; k < kTapGroup; ++k) {
                const int64_t v = (int64_t)u + tap[k];
                int32_t c = (int32_t)(v >> 32);  // floor division by 2^32
                c %= kCodeLen;
                if (c < 0) c += kCodeLen;
                const int r = s_code[c];
                ai[k] += wi * (acc_t)r;
                aq[k] += wq * (acc_t)r;
            }
        }
        // block reduction, then one atomic per output word
        const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
        for (int k = 0; k < kTapGroup; ++k) {
            acc_t a = wave_sum(ai[k]);
            acc_t b = wave_sum(aq[k]);
            if (lane == 0) { s_red[wv][2 * k] = a; s_red[wv][2 * k + 1] = b; }
        }
        __syncthreads();
        if (tid < 2 * nk) {
            acc_t v = 0;
#pragma unroll
            for (int j = 0; j < kThreads / 64; ++j) v += s_red[j][tid];
            const int k = k0 + tid / 2, comp = tid & 1;
            acc_t* dst;
            if (w < m.m_close) {
                dst = (acc_t*)out + (((uint64_t)ch * max_dumps + w) * tap_stride + k) * 2 + comp;
            } else if constexpr (CARR == GC_CARRIER_LUT) {
                dst = &state[ch].acc[k][comp];
            } else {
                dst = &state[ch].acc_f[k][comp];
            }
            atomicAdd(dst, v);
        }
        __syncthreads();
    }
    }
}

template <int FMT, int CARR>
void launch_one(const uint8_t* samples, uint64_t n, const DevChan* chans, const DevMeta* meta,
                gc_chan_state* state, int n_chan, int max_taps, void* out, int tap_stride,
                uint32_t max_dumps, const uint32_t* tables, int grid_x, hipStream_t s) {
    const uint64_t n_tiles = (n + kTile - 1) / kTile;
    dim3 grid((unsigned)(grid_x > 0 ? min((uint64_t)grid_x, n_tiles) : n_tiles), (unsigned)n_chan,
              (unsigned)((max_taps + kTapGroup - 1) / kTapGroup));
    hipLaunchKernelGGL((k_generic<FMT, CARR>), grid, dim3(kThreads), 0, s, samples, n, chans,
                       meta, state, out, tap_stride, max_dumps, tables);
}

// Largest |error| of carrier_f32 over the fp32 phases with bit patterns
// first .. first + count - 1 (all in [0, 1)), against cos and sin of
// 2*pi*phase in double precision: out[0] cos, out[1] sin, as the bit
// patterns of non-negative doubles (which order like the integers).
__global__ __launch_bounds__(256) void k_carrier_sweep(uint32_t first, uint32_t count,
                                                        unsigned long long* __restrict__ out) {
    double ec = 0.0, es = 0.0;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const float ph = __uint_as_float(first + i);
        float c, s;
        carrier_f32(ph, c, s);
        double sd, cd;
        sincos(6.283185307179586476925286766559 * (double)ph, &sd, &cd);
        ec = fmax(ec, fabs((double)c - cd));
        es = fmax(es, fabs((double)s - sd));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        ec = fmax(ec, __shfl_xor(ec, o, 64));
        es = fmax(es, __shfl_xor(es, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(out, (unsigned long long)__double_as_longlong(ec));
        atomicMax(out + 1, (unsigned long long)__double_as_longlong(es));
    }
}

}  // namespace

hipError_t launch_carrier_sweep(uint32_t first, uint32_t count, unsigned long long* out,
                                hipStream_t s) {
    if (count == 0) return hipSuccess;
    const uint32_t blocks = min((count + 255u) / 256u, 8192u);
    hipLaunchKernelGGL(k_carrier_sweep, dim3(blocks), dim3(256), 0, s, first, count, out);
    return hipGetLastError();
}

hipError_t launch_generic(const uint8_t* samples, uint64_t n, int fmt, int carrier,
                          const DevChan* chans, const DevMeta* meta, gc_chan_state* state,
                          int n_chan, int max_taps, void* out, int tap_stride,
                          uint32_t max_dumps, const uint32_t* tables, int grid_x,
                          hipStream_t s) {
    if (n == 0) return hipSuccess;
#define GC_CASE(F, C)                                                                        \
    if (fmt == F && carrier == C) {                                                         \
        launch_one<F, C>(samples, n, chans, meta, state, n_chan, max_taps, out, tap_stride, \
                         max_dumps, tables, grid_x, s);                                     \
        return hipGetLastError();                                                          \
    }
    GC_CASE(GC_I8_REAL, GC_CARRIER_LUT)
    GC_CASE(GC_I8_IQ, GC_CARRIER_LUT)
    GC_CASE(GC_I2_REAL, GC_CARRIER_LUT)
    GC_CASE(GC_I2_IQ, GC_CARRIER_LUT)
    GC_CASE(GC_I8_REAL, GC_CARRIER_F32)
    GC_CASE(GC_I8_IQ, GC_CARRIER_F32)
    GC_CASE(GC_I2_REAL, GC_CARRIER_F32)
    GC_CASE(GC_I2_IQ, GC_CARRIER_F32)
#undef GC_CASE
    return hipErrorInvalidValue;
}

}  // namespace gc
