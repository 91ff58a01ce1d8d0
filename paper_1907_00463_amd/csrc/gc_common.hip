// gc_common.hip -- context tables and per-call set-up kernels of libgnsscorr.
//
// Tables generated on the GPU at context creation:
//   * the G1 and G2 register sequences of IS-GPS-200 Sec. 3.2.1.3 (1023 bits
//     each, bit i of word i/32), from which every block composes its PRN's
//     C/A code in LDS as G1[i] XOR G2[i - delay] (delay from Table 3-Ia);
//   * the carrier table: entry l = round_half_away(24*cos(2*pi*(l+1/2)/256))
//     in the low 16 bits and the same of sin in the high 16 bits.
#include "gc_internal.h"
#include "gc_device.h"

namespace gc {

// One thread steps both 10-stage registers (all ones at the epoch; G1 taps
// 3,10; G2 taps 2,3,6,8,9,10; output stage 10).  Threads 0..255 fill the
// carrier table.
// G2 delay in chips of PRN 1..32 (IS-GPS-200, Table 3-Ia), for the sign tables.
__constant__ int32_t c_g2_delay_dev[32] = {5,   6,   7,   8,   17,  18,  139, 140, 141, 251, 252,
                                           254, 255, 256, 257, 258, 469, 470, 471, 472, 473, 474,
                                           509, 512, 513, 514, 515, 516, 859, 860, 861, 862};

__global__ void k_init_tables(uint32_t* tables) {
    uint32_t* g1 = tables + kTabG1;
    uint32_t* g2 = tables + kTabG2;
    uint32_t* lut = tables + kTabLut;
    const int t = threadIdx.x;
    if (t == 0) {
        uint32_t r1 = 0x3FF, r2 = 0x3FF;  // bit s-1 holds stage s
        for (int w = 0; w < 32; ++w) { g1[w] = 0; g2[w] = 0; }
        for (int i = 0; i < kCodeLen; ++i) {
            g1[i >> 5] |= ((r1 >> 9) & 1u) << (i & 31);
            g2[i >> 5] |= ((r2 >> 9) & 1u) << (i & 31);
            uint32_t f1 = ((r1 >> 2) ^ (r1 >> 9)) & 1u;
            uint32_t f2 = ((r2 >> 1) ^ (r2 >> 2) ^ (r2 >> 5) ^ (r2 >> 7) ^ (r2 >> 8) ^ (r2 >> 9)) & 1u;
            r1 = ((r1 << 1) | f1) & 0x3FF;
            r2 = ((r2 << 1) | f2) & 0x3FF;
        }
    }
    if (t < 256) {
        // 2-bit byte t -> its four samples (codes 0..3 -> -3,-1,+1,+3) as int16
        for (int h = 0; h < 2; ++h) {
            uint32_t ex = 0;
            for (int j = 0; j < 2; ++j) {
                const int v = 2 * (int)((t >> (2 * (2 * h + j))) & 3) - 3;
                ex |= (uint32_t)(uint16_t)(int16_t)v << (16 * j);
            }
            tables[kTabExpand + 2 * t + h] = ex;
        }
    }
    __syncthreads();
    // code signs of every PRN, (s, s) as int16 pairs, chips 0..1022 then a
    // wrapped copy so that runs of chips need no modulo
    for (int idx = t; idx < 32 * kSignLen; idx += blockDim.x) {
        const int prn = idx / kSignLen + 1;
        const int i = (idx % kSignLen) % kCodeLen;
        tables[kTabSign + idx] = ca_chip(tables, c_g2_delay_dev[prn - 1], i) < 0 ? 0xFFFFFFFFu : 0x00010001u;
    }
    // the multi-tap replica operand: chip (2y + r) mod 1023 as an int8 in byte b
    for (int idx = t; idx < 32 * 4 * kMtapCodeWords; idx += blockDim.x) {
        const int prn = idx / (4 * kMtapCodeWords) + 1;
        const int b = (idx / kMtapCodeWords) % 4;
        const int r = (idx / kMtapHalfWords) % 2;
        const int i = (2 * (idx % kMtapHalfWords) + r) % kCodeLen;
        const int c = ca_chip(tables, c_g2_delay_dev[prn - 1], i);
        tables[kTabMtapCode + idx] = (uint32_t)(uint8_t)(int8_t)c << (8 * b);
    }
    if (t < 256) {
        double ang = 6.283185307179586476925286766559 * ((double)t + 0.5) / 256.0;
        double vc = (double)GC_LUT_AMP * cos(ang);
        double vs = (double)GC_LUT_AMP * sin(ang);
        int ic = (int)(vc >= 0.0 ? floor(vc + 0.5) : -floor(-vc + 0.5));
        int is = (int)(vs >= 0.0 ? floor(vs + 0.5) : -floor(-vs + 0.5));
        lut[t] = ((uint32_t)(uint16_t)(int16_t)ic) | ((uint32_t)(uint16_t)(int16_t)is << 16);
    }
}

__global__ void k_code_table(const uint32_t* tables, int d, int8_t* out) {
    for (int i = threadIdx.x; i < kCodeLen; i += blockDim.x) out[i] = ca_chip(tables, d, i);
}

hipError_t launch_make_tables(uint32_t* d_tables, hipStream_t s) {
    hipLaunchKernelGGL(k_init_tables, dim3(1), dim3(256), 0, s, d_tables);
    return hipGetLastError();
}

// Channel records from device-resident configurations, one thread per
// channel: the checks and derived fields of the host's fill_devchan (E/P/L
// tap slots, the 1/32-chip grid test), plus n_taps <= tap_stride.  A
// configuration that fails a check leaves an all-zero record (prn 0), which
// k_setup refuses with GC_EINVAL.
__global__ __launch_bounds__(64) void k_fill_chans(const gc_chan_cfg* __restrict__ cfg,
                                                    int n_chan, int tap_stride,
                                                    DevChan* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_chan) return;
    const gc_chan_cfg& c = cfg[i];
    DevChan d;
    d.prn = 0;
    d.n_taps = 0;
    d.int_periods = 0;
    d.g2_delay = 0;
    d.window = 0;
    d.epl = 0;
    d.slot_e = d.slot_p = d.slot_l = -1;
    d.mt_ok = 0;
    d.mt_jmin = 0;
    d.mt_nj = 0;
    d.rx = 0;
    for (int k = 0; k < GC_MAX_TAPS; ++k) d.taps[k] = 0;
    bool ok = c.prn >= 1 && c.prn <= 32 && c.n_taps >= 1 && c.n_taps <= tap_stride &&
              c.int_periods >= 1 && c.int_periods <= 1000 && c.reserved == 0;
    const int K = ok ? c.n_taps : 0;
    const int64_t lim = int64_t(1) << 40;
    bool grid = true;
    int64_t dmin = 0, dmax = 0;
    for (int k = 0; k < K; ++k) {
        const int64_t t = c.tap_q32[k];
        if (t <= -lim || t >= lim) ok = false;
        d.taps[k] = t;
        if (t & ((int64_t(1) << 27) - 1)) grid = false;
        const int64_t dk = t >> 27;
        if (k == 0 || dk < dmin) dmin = dk;
        if (k == 0 || dk > dmax) dmax = dk;
    }
    if (ok) {
        d.prn = c.prn;
        d.n_taps = c.n_taps;
        d.int_periods = c.int_periods;
        d.g2_delay = c_g2_delay_dev[c.prn - 1];
        d.window = (uint64_t)c.int_periods * kCodeLen * kTwo32;
        if (K == 3) {
            const int64_t h = int64_t(1) << 31;
            for (int k = 0; k < 3; ++k) {
                if (c.tap_q32[k] == h) d.slot_e = k;
                else if (c.tap_q32[k] == 0) d.slot_p = k;
                else if (c.tap_q32[k] == -h) d.slot_l = k;
            }
            d.epl = d.slot_e >= 0 && d.slot_p >= 0 && d.slot_l >= 0;
        }
        // floor division by 32 of the 1/32-chip indices
        const int64_t jmin = dmin >= 0 ? dmin / 32 : -((31 - dmin) / 32);
        const int64_t hi = dmax + 31;
        const int64_t jmax = hi >= 0 ? hi / 32 : -((31 - hi) / 32);
        d.mt_ok = grid && jmax - jmin + 1 <= 8;
        d.mt_jmin = (int32_t)jmin;
        d.mt_nj = (int32_t)(jmax - jmin + 1);
    } else {
        for (int k = 0; k < GC_MAX_TAPS; ++k) d.taps[k] = 0;
    }
    out[i] = d;
}

hipError_t launch_fill_chans(const gc_chan_cfg* cfg, int n_chan, int tap_stride, DevChan* out,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_fill_chans, dim3((n_chan + 63) / 64), dim3(64), 0, s, cfg, n_chan,
                       tap_stride, out);
    return hipGetLastError();
}

hipError_t launch_code_table(const uint32_t* d_tables, int g2_delay, int8_t* d_out, hipStream_t s) {
    hipLaunchKernelGGL(k_code_table, dim3(1), dim3(256), 0, s, d_tables, g2_delay, d_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-call set-up, one block per channel (k_setup):
//   * validate the channel state and compute M = floor(U_N / W), the number
//     of dumps this block closes;
//   * start output row 0 from the open dump carried in the state;
//   * move the NCO words of the state to the end of the block.
// then k_rows clears rows 1..M-1 and writes the sample count of every row.
// The accumulation kernels read the start-of-block NCO words from DevMeta
// and add into the rows (windows < M) or into the state's open dump (M).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_setup(const DevChan* __restrict__ chans,
                                               DevMeta* __restrict__ metas,
                                               gc_chan_state* __restrict__ state,
                                               uint64_t n, int fmt, int carrier,
                                               uint32_t max_dumps, void* out, int tap_stride,
                                               uint32_t* __restrict__ dump_n,
                                               uint32_t* __restrict__ n_dumps,
                                               int32_t* __restrict__ status_out,
                                               int32_t allow,
                                               const DevRx* __restrict__ rx,
                                               const int32_t* __restrict__ list,
                                               const int32_t* __restrict__ list_rx) {
    const int ch = list ? list[blockIdx.x] : (int)blockIdx.x;
    const int tid = threadIdx.x;
    const DevChan& c = chans[ch];
    if (rx) {  // batch: the block and format of the channel's receiver
        const int r = list_rx ? list_rx[blockIdx.x] : c.rx;
        n = rx[r].n;
        fmt = rx[r].fmt;
    }
    gc_chan_state* st = state + ch;
    __shared__ DevMeta sm;
    if (tid == 0) {
        DevMeta m;
        m.p0 = st->code_phase;
        m.dp = st->code_step;
        m.window = c.window;
        m.phi0 = st->carr_phase;
        m.dphi = st->carr_step;
        m.phf0 = st->carr_phase_f;
        m.ff = st->carr_freq_f;
        m.acc_n0 = st->acc_n;
        m.m_close = 0;
        m.path = kPathDirect;
        m.c_full0 = m.c_full1 = 0;
        m.head_end = m.tail_beg = 0;
        m.bin_len = 0;
        m.pad2 = 0;
        int32_t s = GC_OK;
        if (c.prn < 1 || m.dp == 0 || m.dp >= (1ull << 31) || m.p0 >= m.window) {
            s = GC_EINVAL;
        } else {
            const uint64_t u_end = m.p0 + n * m.dp;
            const uint64_t mc = u_end / m.window;
            const uint64_t nmax = (m.window - 1) / m.dp + 1;
            const uint64_t maxw = fmt == GC_I8_REAL ? 128ull * GC_LUT_AMP
                                : fmt == GC_I8_IQ   ? 128ull * kLutAbsSumMax
                                : fmt == GC_I2_IQ   ? 3ull * kLutAbsSumMax
                                                    : 3ull * GC_LUT_AMP;
            if (carrier == GC_CARRIER_LUT && nmax * maxw > 2147483647ull) s = GC_ERANGE;
            else if (mc > max_dumps) s = GC_ENOSPC;
            else m.m_close = (uint32_t)mc;
            // whole chips of this block: [c_full0, c_full1); the samples before
            // and after them are handled by the direct per-sample path
            m.c_full0 = (m.p0 + 0xFFFFFFFFull) >> 32;
            m.c_full1 = u_end >> 32;
            auto chip_start = [&](uint64_t c) -> uint64_t {
                const uint64_t ph = c << 32;
                return ph <= m.p0 ? 0 : (ph - m.p0 + m.dp - 1) / m.dp;
            };
            const uint64_t he = min(n, chip_start(m.c_full0));
            uint64_t tb = m.c_full1 > m.c_full0 ? chip_start(m.c_full1) : he;
            if (tb < he) tb = he;
            m.head_end = (uint32_t)he;
            m.tail_beg = (uint32_t)tb;
            m.path = kPathDirect;
            m.bin_len = 0;
            const bool lut = carrier == GC_CARRIER_LUT;
            const bool epl_ok = c.epl && m.c_full1 > m.c_full0;
            if (epl_ok && lut && (allow & kAllowPeriodic) && !fmt_complex(fmt)) {
                m.bin_len = periodic_bin_len(fmt, m.dp);
                if (m.bin_len) m.path = kPathPeriodic;
            }
            // (float bin sums have no int16 bound)
            if (m.path == kPathDirect && epl_ok && (allow & kAllowBinned) &&
                (lut ? binned_ok(fmt, m.dp) : binned_geometry_ok(m.dp)))
                m.path = kPathBinned;
            // dense taps on the 1/32-chip grid: at most one sample per 1/32 chip
            if (m.path == kPathDirect && (allow & kAllowMtap) && c.mt_ok &&
                carrier == GC_CARRIER_LUT && m.dp >= (1ull << 27))
                m.path = kPathMtap;
        }
        m.status = s;
        metas[ch] = m;
        status_out[ch] = s;
        n_dumps[ch] = s == GC_OK ? m.m_close : 0u;
        sm = m;
    }
    __syncthreads();
    const DevMeta m = sm;
    if (m.status != GC_OK) return;
    const uint32_t M = m.m_close;
    const int K = c.n_taps;
    // row 0 starts with the dump carried in the state; the state's open dump
    // restarts at zero when at least one window closes in this block
    // (rows 1 .. M-1 are cleared by k_rows)
    if (M >= 1) {
        const uint64_t row = (uint64_t)ch * max_dumps * tap_stride * 2;
        for (int k = tid; k < K; k += blockDim.x) {
            if (carrier == GC_CARRIER_LUT) {
                int32_t* o = (int32_t*)out + row;
                o[2 * k] = st->acc[k][0];
                o[2 * k + 1] = st->acc[k][1];
                st->acc[k][0] = 0;
                st->acc[k][1] = 0;
            } else {
                float* o = (float*)out + row;
                o[2 * k] = st->acc_f[k][0];
                o[2 * k + 1] = st->acc_f[k][1];
                st->acc_f[k][0] = 0.0f;
                st->acc_f[k][1] = 0.0f;
            }
        }
    }
    if (tid == 0) {
        const uint64_t u_end = m.p0 + n * m.dp;
        const uint64_t sM = M == 0 ? 0 : window_start(M, m.window, m.p0, m.dp);
        st->acc_n = M == 0 ? m.acc_n0 + (uint32_t)n : (uint32_t)(n - sM);
        st->carr_phase = m.phi0 + (uint32_t)n * m.dphi;
        st->code_phase = u_end - (uint64_t)M * m.window;
        double t = m.phf0 + (double)n * m.ff;
        st->carr_phase_f = t - floor(t);
    }
}

// ceil(num / d) for d >= 1: a double estimate made exact with integer checks
// (the estimate is within one of the quotient for d >= 2^20).
// ceil(num / d) for d >= 2^20 from inv = 1 / d in double: the estimate
// num * inv is within one of the quotient (below 2^44, relative error a few
// units in 2^-53), so two exact integer steps each way make it exact.
__device__ __forceinline__ uint64_t udiv_ceil(uint64_t num, uint64_t d, double inv) {
    uint64_t q = (uint64_t)((double)num * inv);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        if (q * d < num) ++q;
        if (q > 0 && (q - 1) * d >= num) --q;
    }
    return q;
}

// The items of the chip-by-chip batch kernel with work: receivers with a
// channel that is neither refused nor periodic, their tiles in order, into
// order[0 .. *count); also zeroes *queue (the periodic batch kernel's item
// queue).  Run by one block of k_rows (any block size up to 256).
__device__ void select_items(const SelectArgs& a, const DevChan* __restrict__ chans,
                             const DevMeta* __restrict__ metas) {
    __shared__ uint32_t s_part[256];
    __shared__ uint32_t s_need[256];
    __shared__ uint32_t s_base;
    const int t = threadIdx.x, nt = blockDim.x;
    if (t == 0) {
        s_base = 0;
        if (a.queue) *a.queue = 0;
    }
    for (int r0 = 0; r0 < a.n_rx; r0 += nt) {
        const int r1 = min(a.n_rx, r0 + nt);
        s_need[t] = 0;
        __syncthreads();
        for (int c = t; c < a.n_chan; c += nt) {
            const int cr = chans[c].rx;
            if (cr >= r0 && cr < r1 && metas[c].status == GC_OK && metas[c].path != kPathPeriodic)
                s_need[cr - r0] = 1u;
        }
        __syncthreads();
        const int r = r0 + t;
        uint32_t cnt = 0;
        if (r < r1 && s_need[t]) {
            const uint32_t te = r + 1 < a.n_rx ? a.rx[r + 1].tile_begin : a.n_items;
            cnt = te - a.rx[r].tile_begin;
        }
        s_part[t] = cnt;
        __syncthreads();
        for (int off = 1; off < nt; off <<= 1) {  // inclusive scan
            const uint32_t v = t >= off ? s_part[t - off] : 0u;
            __syncthreads();
            s_part[t] += v;
            __syncthreads();
        }
        // each needing receiver's items, written by the whole block
        for (int i = 0; i < r1 - r0; ++i) {
            const uint32_t end = s_part[i], beg = i > 0 ? s_part[i - 1] : 0u;
            if (end == beg) continue;
            const uint32_t tb = a.rx[r0 + i].tile_begin;
            for (uint32_t j = (uint32_t)t; j < end - beg; j += (uint32_t)nt)
                a.order[s_base + beg + j] = tb + j;
        }
        __syncthreads();
        if (t == nt - 1) s_base += s_part[nt - 1];
        __syncthreads();
    }
    if (t == 0) *a.count = s_base;
}

// Per-call output rows 1 .. M-1 of every channel: cleared (all tap_stride
// taps of a row), and the sample count of each emitted dump (row 0 also holds
// the samples carried in).  With a selection (sel.rx not null) the grid has
// one more column of blocks, whose first block runs select_items.
__global__ __launch_bounds__(256) void k_rows(const DevChan* __restrict__ chans,
                                              const DevMeta* __restrict__ metas, int carrier,
                                              uint32_t max_dumps, void* out, int tap_stride,
                                              uint32_t* __restrict__ dump_n,
                                              const int32_t* __restrict__ list, SelectArgs sel) {
    const uint32_t nx = sel.rx ? gridDim.x - 1 : gridDim.x;
    if (blockIdx.x == nx) {
        if (blockIdx.y == 0) select_items(sel, chans, metas);
        return;
    }
    const int ch = list ? list[blockIdx.y] : (int)blockIdx.y;
    const DevMeta m = metas[ch];
    if (m.status != GC_OK) return;
    const uint32_t M = m.m_close;
    const uint32_t stride = nx * blockDim.x;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (m.dp >= (1ull << 20)) {
        const double inv = 1.0 / (double)m.dp;
        for (uint32_t r = t; r < M; r += stride) {
            const uint64_t s0 = r == 0 ? 0 : udiv_ceil(r * m.window - m.p0, m.dp, inv);
            const uint64_t s1 = udiv_ceil((r + 1) * m.window - m.p0, m.dp, inv);
            dump_n[(uint64_t)ch * max_dumps + r] = (uint32_t)(s1 - s0) + (r == 0 ? m.acc_n0 : 0u);
        }
    } else {
        for (uint32_t r = t; r < M; r += stride) {
            const uint64_t s0 = r == 0 ? 0 : (r * m.window - m.p0 + m.dp - 1) / m.dp;
            const uint64_t s1 = ((r + 1) * m.window - m.p0 + m.dp - 1) / m.dp;
            dump_n[(uint64_t)ch * max_dumps + r] = (uint32_t)(s1 - s0) + (r == 0 ? m.acc_n0 : 0u);
        }
    }
    // rows 1 .. M-1 are contiguous: clear their 4-byte words, 16 bytes per
    // store where the row block is aligned (carrier-independent: 0 and 0.0f
    // share their bits)
    if (M <= 1) return;
    (void)carrier;
    uint32_t* o = (uint32_t*)out + ((uint64_t)ch * max_dumps + 1) * tap_stride * 2;
    const uint64_t words = (uint64_t)(M - 1) * tap_stride * 2;
    const uint64_t head = min(words, (uint64_t)((16 - ((uintptr_t)o & 15)) & 15) / 4);
    for (uint64_t i = t; i < head; i += stride) o[i] = 0u;
    uint4* o4 = reinterpret_cast<uint4*>(o + head);
    const uint64_t n4 = (words - head) / 4;
    for (uint64_t i = t; i < n4; i += stride) o4[i] = uint4{0u, 0u, 0u, 0u};
    for (uint64_t i = head + 4 * n4 + t; i < words; i += stride) o[i] = 0u;
}

hipError_t launch_setup(const DevChan* chans, DevMeta* meta, gc_chan_state* state, int n_chan,
                        uint64_t n_samples, int fmt, int carrier, uint32_t max_dumps, void* out,
                        int tap_stride, uint32_t* dump_n, uint32_t* n_dumps, int32_t* status,
                        int32_t allow, const DevRx* rx, const int32_t* list,
                        const int32_t* list_rx, hipStream_t s, const SelectArgs* sel) {
    hipLaunchKernelGGL(k_setup, dim3(n_chan), dim3(64), 0, s, chans, meta, state, n_samples, fmt,
                       carrier, max_dumps, out, tap_stride, dump_n, n_dumps, status, allow, rx,
                       list, list_rx);
    const uint32_t gx = min((max_dumps + 255u) / 256u, 256u);
    const SelectArgs none{};
    hipLaunchKernelGGL(k_rows, dim3(gx + (sel ? 1u : 0u), n_chan), dim3(256), 0, s, chans, meta,
                       carrier, max_dumps, out, tap_stride, dump_n, list, sel ? *sel : none);
    return hipGetLastError();
}

}  // namespace gc
