// gc_mtap.hip -- dense multi-tap correlator (many taps on a 1/32-chip grid)
// as an exact two-stage contraction on int8 MFMA.
//
// Taps delta_k = d_k * 2^27 (d_k integer, 1/32 chip).  Write the code phase
// of sample n as U_n = c_n*2^32 + q_n*2^27 + e (q_n in [0, 32), e < 2^27).
// Then the replica chip of tap k is
//     floor((U_n + delta_k) / 2^32) = c_n + floor((q_n + d_k) / 32),
// so with S[q][c] = the wiped-off sample whose (q_n, c_n) = (q, c), or 0
// (at most one sample per cell when a chip spans <= 32 samples):
//     T[q][j] = sum_c S[q][c] * C[(c + j) mod 1023]      (stage 2, MFMA)
//     Y_k     = sum_q T[q][floor((q + d_k) / 32)]         (stage 3)
// Stage 1 scatters the samples into S, one 32-chip chunk at a time, in LDS.
// A cell holds four int8: the wiped-off I and Q (|w| <= 128*34) each split
// as w = 64*hi + lo with lo = w & 63 in [0, 63] and hi = w >> 6 in [-68, 68].
// The contraction index runs over (chip, byte of the cell); the replica
// operand holds (C, 64*C, 0, 0) per chip in its I columns and (0, 0, C, 64*C)
// in its Q columns (8 chip shifts each), so one v_mfma_i32_16x16x64_i8 over
// 16 chips yields exact int32 T for I and Q at once.  T accumulates over the
// chunks of a dump; at the dump's end prefix sums over q turn every tap into
// two range sums (stage 3), and the dump is stored.
//
// One wave per channel (16 per block), blocks take contiguous chunks of
// sample tiles; the tile (8 B per sample: (xI, xQ) and (xQ, -xI) as int16)
// and a 16-copy carrier table are shared by the block's waves.  The complex
// wipe-off is two v_dot2 per sample; lanes take consecutive samples, so
// sample and table reads are conflict-free, and a row stride of 34 dwords
// keeps the cells one instruction writes in distinct banks (rows q differ
// by less than 32) as well as the 8-byte operand reads of 16 rows.
#include "gc_device.h"

namespace gc {

namespace {

constexpr int kWaves = 16;
constexpr int kChunkChips = 32;                  // chips per chunk (two MFMA K steps)
constexpr int kRows = 32;                        // q
constexpr int kRowBytes = 136;                   // 32 chips x 4 B + 8 pad (34 dwords)
constexpr int kSBytes = kRows * kRowBytes;       // 4352 per wave
constexpr int kLutCopies = 16;
constexpr int kLutStride = 257;                  // words between copies
constexpr int kLutBytes = kLutCopies * kLutStride * 4;
constexpr int kTile = 8576;                      // samples per tile
constexpr int kMargin = kChunkChips * 32 + 64;   // a chunk spans <= 32 chips of <= 32 samples
constexpr int kXSamples = kTile + kMargin;
constexpr int kOffS = kLutBytes;
constexpr int kOffX = kOffS + kWaves * kSBytes;
constexpr int kOffList = kOffX + kXSamples * 8;
constexpr int kLdsBytes = kOffList + 4 * (kWaves + 1);
static_assert(kLdsBytes <= 160 * 1024, "LDS per block");
static_assert(kTile % 16 == 0 && kXSamples % 16 == 0, "staging granule");
static_assert(2 * 8 * 33 * 4 <= kSBytes, "stage-3 prefix sums fit the wave's S area");
static_assert(kOffS % 8 == 0 && kSBytes % 8 == 0 && kRowBytes % 8 == 0, "8-byte operand reads");

typedef short short2_t __attribute__((ext_vector_type(2)));
typedef int int4_t __attribute__((ext_vector_type(4)));
typedef int int2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ short2_t as_s2(uint32_t v) { return __builtin_bit_cast(short2_t, v); }

__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ceil(num / d), d in [2^27, 2^31): a double estimate made exact.
__device__ __forceinline__ uint64_t ceil_div(uint64_t num, uint64_t d) {
    uint64_t q = (uint64_t)((double)num / (double)d);
    while (q * d < num) ++q;
    while (q > 0 && (q - 1) * d >= num) --q;
    return q;
}

// One 32-chip chunk of a dump: chips [cs, ce), samples [sa, sb).  Chunks
// are walked in order; the first sample of the next chunk follows from the
// overshoot of this one (e = sb*dp - (ce*2^32 - p0), in [0, dp)) without a
// division by the code step.
struct Chunk {
    uint64_t cs, ce;   // chips [cs, ce)
    uint64_t d0;       // first chip of the dump (span * m)
    uint64_t sa, sb;   // samples [sa, sb), clipped to [0, n]
    uint64_t fb;       // first sample of chip ce (unclipped)
    uint64_t eb;       // its overshoot
    uint32_t m;        // dump (window) index
    uint32_t cmod;     // cs mod 1023
    bool first, last;  // first / last chunk of its dump
};

// First sample of chip c (code phase c*2^32) with its overshoot; chips that
// start before the block give sample 0 and overshoot 0.
__device__ __forceinline__ void chip_first(uint64_t c, uint64_t p0, uint64_t dp, uint64_t& f,
                                           uint64_t& e) {
    const uint64_t ph = c << 32;
    if (ph <= p0) {
        f = 0;
        e = 0;
        return;
    }
    f = ceil_div(ph - p0, dp);
    e = f * dp - (ph - p0);
}

// The chunk of chip c: chips [span*m + 32a, min(+32, span*(m+1))).
__device__ __forceinline__ Chunk chunk_of(uint64_t c, uint64_t span, uint64_t p0, uint64_t dp,
                                          uint64_t n) {
    Chunk k;
    k.m = (uint32_t)(c / span);
    k.d0 = (uint64_t)k.m * span;
    k.cs = k.d0 + ((c - k.d0) / kChunkChips) * kChunkChips;
    k.ce = min(k.cs + kChunkChips, k.d0 + span);
    k.first = k.cs == k.d0;
    k.last = k.ce == k.d0 + span;
    k.cmod = (uint32_t)((k.cs - k.d0) % kCodeLen);
    uint64_t fa, ea;
    chip_first(k.cs, p0, dp, fa, ea);
    chip_first(k.ce, p0, dp, k.fb, k.eb);
    k.sa = min(n, fa);
    k.sb = min(n, k.fb);
    return k;
}

// The chunk after k: its first sample is k's end; its end advances by
// ceil(((ce' - ce)*2^32 - eb) / dp) samples (one or two candidates around a
// float estimate, checked exactly).
__device__ __forceinline__ void chunk_next(Chunk& k, uint64_t span, uint64_t dp, float inv_dp,
                                           uint64_t n) {
    if (k.last) {
        k.m += 1;
        k.d0 += span;
        k.cmod = 0;  // a dump starts on a code epoch
    } else {
        k.cmod += kChunkChips;
        if (k.cmod >= kCodeLen) k.cmod -= kCodeLen;
    }
    k.cs = k.ce;
    k.ce = min(k.cs + kChunkChips, k.d0 + span);
    k.first = k.cs == k.d0;
    k.last = k.ce == k.d0 + span;
    k.sa = k.sb;
    const uint32_t nch = (uint32_t)(k.ce - k.cs);          // 1 .. 32
    const uint64_t num = ((uint64_t)nch << 32) - k.eb;      // > 0
    const float est = ((float)nch * 4294967296.0f - (float)(uint32_t)k.eb) * inv_dp;
    uint64_t q = (uint64_t)(uint32_t)max(0.0f, est - 2.0f);
    while (q * dp < num) ++q;
    k.fb += q;
    k.eb = q * dp - num;
    k.sb = min(n, k.fb);
}

// Tile samples [t0, t0 + kXSamples) as two int16 pairs each: (xI, xQ) and
// (xQ, -xI) (real input: (x, 0) and (0, -x)); zero past the block.  Each
// thread takes units of 8 samples: one 16-byte (complex int8), 8-byte (real
// int8) or 2-byte (2-bit) load, four 16-byte LDS stores.
template <int FMT>
__device__ __forceinline__ void stage_tile(const uint8_t* __restrict__ samples, uint64_t n,
                                           uint64_t t0, uint8_t* lds, int nthreads) {
    static_assert(kXSamples % 8 == 0, "staging unit");
    uint4* dst = reinterpret_cast<uint4*>(lds + kOffX);
    const uint32_t avail = (uint32_t)min(n - t0, (uint64_t)kXSamples);
    for (int u = threadIdx.x; u < kXSamples / 8; u += nthreads) {
        const uint32_t s0 = 8u * (uint32_t)u;
        const bool whole = s0 + 8 <= avail;
        int xi[8], xq[8];
        if constexpr (FMT == GC_I8_IQ) {
            const uint8_t* src = samples + 2 * (t0 + s0);
            uint32_t w[4] = {0, 0, 0, 0};
            if (whole) {
                const uint4 q = *reinterpret_cast<const uint4*>(src);
                w[0] = q.x; w[1] = q.y; w[2] = q.z; w[3] = q.w;
            } else {
                for (uint32_t b = 0; b < 16; ++b)
                    if (s0 + b / 2 < avail) w[b / 4] |= (uint32_t)src[b] << (8 * (b % 4));
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint32_t v = w[k / 2] >> (16 * (k % 2));
                xi[k] = (int)(int8_t)(v & 0xFF);
                xq[k] = (int)(int8_t)((v >> 8) & 0xFF);
            }
        } else if constexpr (FMT == GC_I8_REAL) {
            const uint8_t* src = samples + t0 + s0;
            uint32_t w[2] = {0, 0};
            if (whole) {
                const uint2 q = *reinterpret_cast<const uint2*>(src);
                w[0] = q.x; w[1] = q.y;
            } else {
                for (uint32_t b = 0; b < 8; ++b)
                    if (s0 + b < avail) w[b / 4] |= (uint32_t)src[b] << (8 * (b % 4));
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                xi[k] = (int)(int8_t)((w[k / 4] >> (8 * (k % 4))) & 0xFF);
                xq[k] = 0;
            }
        } else {
            const uint8_t* src = samples + (t0 + s0) / 4;
            uint32_t w = 0;
            if (whole) {
                w = *reinterpret_cast<const uint16_t*>(src);
            } else {
                for (uint32_t b = 0; b < 2; ++b)
                    if (s0 + 4 * b < avail) w |= (uint32_t)src[b] << (8 * b);
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                xi[k] = s0 + k < avail ? 2 * (int)((w >> (2 * k)) & 3u) - 3 : 0;
                xq[k] = 0;
            }
        }
        if (!whole) {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (s0 + k >= avail) xi[k] = xq[k] = 0;
        }
#pragma unroll
        for (int k = 0; k < 8; k += 2) {
            uint4 o;
            o.x = (uint32_t)(uint16_t)xi[k] | ((uint32_t)(uint16_t)xq[k] << 16);
            o.y = (uint32_t)(uint16_t)xq[k] | ((uint32_t)(uint16_t)(-xi[k]) << 16);
            o.z = (uint32_t)(uint16_t)xi[k + 1] | ((uint32_t)(uint16_t)xq[k + 1] << 16);
            o.w = (uint32_t)(uint16_t)xq[k + 1] | ((uint32_t)(uint16_t)(-xi[k + 1]) << 16);
            dst[(s0 + k) / 2] = o;
        }
    }
}

// Stage 1, one sample per lane: wipe-off, split into the four int8 of the
// cell, one dword store into row q, column (chip - cs).
template <bool CHECK>
__device__ __forceinline__ void scatter_step(uint8_t* lds, uint32_t xaddr, uint32_t ph,
                                             uint32_t lut_base, uint64_t U, uint32_t cbase,
                                             bool valid) {
    if (CHECK && !valid) return;
    const uint2 xw = *reinterpret_cast<const uint2*>(lds + xaddr);
    const uint32_t cs = *reinterpret_cast<const uint32_t*>(lds + lut_base + ((ph >> 24) << 2));
    // (wI, wQ) = (xI, xQ) c + (xQ, -xI) s as int16 pairs: every product and
    // sum stays below 2^15 in magnitude (|x c| <= 3072, |w| <= 4352), so the
    // 16-bit lanes hold the exact values
    const short2_t c2 = as_s2(cs);
    const short2_t cc = __builtin_shufflevector(c2, c2, 0, 0);
    const short2_t ss = __builtin_shufflevector(c2, c2, 1, 1);
    const short2_t w2 = as_s2(xw.x) * cc + as_s2(xw.y) * ss;
    // per half: bits 0-5 stay, bits 6-13 move to the upper byte (w >> 6 as a
    // two's complement byte)
    const uint32_t h = __builtin_bit_cast(uint32_t, w2);
    const uint32_t cell = ((h << 2) & 0xFF00FF00u) | (h & 0x003F003Fu);
    // row q, column chip - cs: cbase = s_base - 4*cs (mod 2^32)
    const uint32_t lo = (uint32_t)U, hi = (uint32_t)(U >> 32);
    const uint32_t q = lo >> 27;
    const uint32_t a = __umul24(q, kRowBytes) + (hi * 4u + cbase);
    *reinterpret_cast<uint32_t*>(lds + a) = cell;
}

struct Dest {
    int32_t* out;
    gc_chan_state* st;
    uint64_t row0;
    int tap_stride;
    uint32_t m_close;
};

// Stage 3 for the dump held in acc (T[q][col]: col < 8 the I sums of shift
// jmin + col, col >= 8 the Q sums of shift jmin + col - 8): prefix sums over q
// in the wave's S area, two range sums per tap, stored (plain or atomic).
__device__ __forceinline__ void finish_dump(int4_t (&acc)[2], uint8_t* lds, uint32_t s_base,
                                            uint32_t lane, const DevChan& ch, int jmin,
                                            uint32_t m, bool plain, const Dest& d) {
    int32_t* P = reinterpret_cast<int32_t*>(lds + s_base);  // [plane][j][33]
    const uint32_t col = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) P[col * 33 + 16 * t + 4 * g + v] = acc[t][v];
    }
    wave_fence();
    if (lane < 16) {  // exclusive prefix over q of sequence (plane, j) = (lane/8, lane%8)
        int32_t* r = P + lane * 33;
        int run = 0;
        for (int q = 0; q < 32; ++q) {
            const int t = r[q];
            r[q] = run;
            run += t;
        }
        r[32] = run;
    }
    wave_fence();
    const int K = ch.n_taps;
    for (int k = (int)lane; k < K; k += 64) {
        const int dk = (int)(ch.taps[k] >> 27);
        const int fl = dk >= 0 ? dk / 32 : -((31 - dk) / 32);
        const int r = dk - 32 * fl;  // in [0, 32)
        const int jA = fl - jmin;
        const int b = 32 - r;
        int y[2];
#pragma unroll
        for (int pl = 0; pl < 2; ++pl) {
            const int32_t* PA = P + (pl * 8 + jA) * 33;
            y[pl] = PA[b];
            if (r > 0) {
                const int32_t* PB = PA + 33;
                y[pl] += PB[32] - PB[b];
            }
        }
        if (m < d.m_close) {
            int32_t* o = d.out + ((d.row0 + m) * d.tap_stride + k) * 2;
            if (plain) {
                o[0] = y[0];
                o[1] = y[1];
            } else {
                if (y[0]) atomicAdd(o, y[0]);
                if (y[1]) atomicAdd(o + 1, y[1]);
            }
        } else {
            if (y[0]) atomicAdd(&d.st->acc[k][0], y[0]);
            if (y[1]) atomicAdd(&d.st->acc[k][1], y[1]);
        }
    }
    wave_fence();
    acc[0] = int4_t{0, 0, 0, 0};
    acc[1] = int4_t{0, 0, 0, 0};
}

template <int FMT>
__global__ __launch_bounds__(kWaves * 64) void k_mtap(const uint8_t* __restrict__ samples,
                                                      uint64_t n,
                                                      const DevChan* __restrict__ chans,
                                                      const DevMeta* __restrict__ metas,
                                                      gc_chan_state* __restrict__ state,
                                                      int32_t* __restrict__ out, int tap_stride,
                                                      uint32_t max_dumps,
                                                      const uint32_t* __restrict__ tables,
                                                      int n_chan, uint32_t n_tiles) {
    __shared__ __attribute__((aligned(16))) uint8_t s_lds[kLdsBytes];
    int* s_list = reinterpret_cast<int*>(s_lds + kOffList);
    const int tid = threadIdx.x;
    const int nthreads = blockDim.x;
    const int wave = tid / 64;
    const uint32_t lane = tid & 63;

    if (tid == 0) {  // this block's channel group
        const int first = (int)blockIdx.y * kWaves;
        int k = 0, seen = 0;
        for (int c = 0; c < n_chan && k < kWaves; ++c) {
            const DevMeta& m = metas[c];
            if (m.status == GC_OK && m.path == kPathMtap) {
                if (seen >= first) s_list[k++] = c;
                ++seen;
            }
        }
        s_list[kWaves] = k;
    }
    __syncthreads();
    const int nlist = s_list[kWaves];
    if (nlist == 0) return;
    {
        uint32_t* lut = reinterpret_cast<uint32_t*>(s_lds);
        for (int i = tid; i < kLutCopies * kLutStride; i += nthreads) {
            const int e = i % kLutStride;
            lut[i] = e < 256 ? tables[kTabLut + e] : 0u;
        }
    }

    const bool active = wave < nlist;
    const int chn = __builtin_amdgcn_readfirstlane(active ? s_list[wave] : 0);
    const DevChan& ch = chans[chn];
    const DevMeta m = metas[chn];
    const Dest d{out, state + chn, (uint64_t)chn * max_dumps, tap_stride, m.m_close};
    const uint64_t span = m.window >> 32;
    const uint32_t s_base = kOffS + wave * kSBytes;
    const uint32_t lut_base = (lane & (kLutCopies - 1)) * kLutStride * 4;
    const int jmin = ch.mt_jmin;
    const float inv_dp = 1.0f / (float)m.dp;
    // lane's operand columns: chips 4g.. of each 16-chip K step, shift
    // jmin + (lane & 7), as an offset in [0, 1023) from the chunk's first
    // chip; lanes 8..15 of a row group read the Q table (pairs in the upper
    // half-word)
    const uint32_t b_off = (uint32_t)(4 * (int)(lane >> 4) + (int)(lane & 7) + 2 * kCodeLen + jmin) %
                           kCodeLen;
    // replica operand source: (C, 64*C) int8 pairs of this PRN, one word per
    // chip, then the same pairs in the upper half-words
    const uint32_t* cpair = tables + kTabCodePair + (ch.prn - 1) * 2 * kCodePairWords;
    const uint32_t* cpl = cpair + ((lane & 8) ? kCodePairWords : 0);

    // contiguous chunk of tiles for this block; chunks belong to the tile
    // holding their first sample
    const uint32_t tb0 = (uint32_t)(((uint64_t)blockIdx.x * n_tiles) / gridDim.x);
    const uint32_t tb1 = (uint32_t)(((uint64_t)(blockIdx.x + 1) * n_tiles) / gridDim.x);
    const uint64_t T0 = (uint64_t)tb0 * kTile;
    const uint64_t T1 = min(n, (uint64_t)tb1 * kTile);

    int4_t acc[2] = {int4_t{0, 0, 0, 0}, int4_t{0, 0, 0, 0}};
    Chunk k = chunk_of((m.p0 + T0 * m.dp) >> 32, span, m.p0, m.dp, n);
    if (T0 > 0 && k.sa < T0) k = chunk_of(k.ce, span, m.p0, m.dp, n);
    bool seen_first = k.first;  // this wave holds the dump from its first chunk
    bool open = false;          // acc holds part of dump k.m
    // replica operand of a chunk (chips from cmod), loaded one chunk ahead
    auto load_b = [&](uint32_t cmod, int4_t (&b)[2]) {
        uint32_t o = cmod + b_off;
        if (o >= kCodeLen) o -= kCodeLen;
        b[0] = *reinterpret_cast<const int4_t*>(cpl + o);
        b[1] = *reinterpret_cast<const int4_t*>(cpl + o + 16);
    };
    int4_t bop[2];
    if (active) load_b(k.cmod, bop);

    for (uint32_t tile = tb0; tile < tb1; ++tile) {
        const uint64_t t0 = (uint64_t)tile * kTile;
        const uint64_t t1 = min(n, t0 + kTile);
        __syncthreads();
        stage_tile<FMT>(samples, n, t0, s_lds, nthreads);
        __syncthreads();
        if (!active) continue;
        while (k.sa < t1 && k.sa < k.sb) {
            // stage 1: clear S (32 rows of 32 cells), scatter the chunk's samples
            {
                uint2* z = reinterpret_cast<uint2*>(s_lds + s_base + (lane >> 1) * kRowBytes +
                                                    64 * (lane & 1));
#pragma unroll
                for (int c = 0; c < 8; ++c) z[c] = uint2{0u, 0u};
            }
            wave_fence();
            const uint64_t n0 = k.sa + lane;
            uint64_t U = m.p0 + n0 * m.dp;
            uint32_t ph = m.phi0 + (uint32_t)n0 * m.dphi;
            uint32_t xaddr = kOffX + (uint32_t)(n0 - t0) * 8u;
            const uint64_t dU = 64ull * m.dp;
            const uint32_t dph = 64u * m.dphi;
            const uint32_t cbase = s_base - 4u * (uint32_t)k.cs;
            const uint32_t cnt = __builtin_amdgcn_readfirstlane((uint32_t)(k.sb - k.sa));
            const uint32_t full = cnt / 64;
            for (uint32_t j = 0; j < full; ++j) {
                scatter_step<false>(s_lds, xaddr, ph, lut_base, U, cbase, true);
                U += dU;
                ph += dph;
                xaddr += 512u;
            }
            if (cnt % 64)
                scatter_step<true>(s_lds, xaddr, ph, lut_base, U, cbase, lane < cnt % 64);
            wave_fence();
            // stage 2: two 16-row tiles x two 16-chip K steps x 16 columns
            {
                const uint32_t j = lane & 15, g = lane >> 4;
                const int4_t b_cur[2] = {bop[0], bop[1]};
                // the next chunk starts at chip offset cmod + 32, or at a
                // code epoch (offset 0) after the last chunk of a dump
                uint32_t cnext = k.cmod + kChunkChips;
                if (cnext >= kCodeLen) cnext -= kCodeLen;
                load_b(k.last ? 0u : cnext, bop);
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        const uint8_t* ap = s_lds + s_base + (16 * t + j) * kRowBytes + 64 * ks + 16 * g;
                        const int2_t a0 = *reinterpret_cast<const int2_t*>(ap);
                        const int2_t a1 = *reinterpret_cast<const int2_t*>(ap + 8);
                        const int4_t a = int4_t{a0.x, a0.y, a1.x, a1.y};
                        acc[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b_cur[ks], acc[t], 0, 0, 0);
                    }
                }
            }
            open = true;
            if (k.last) {
                finish_dump(acc, s_lds, s_base, lane, ch, jmin, k.m, seen_first && k.m > 0, d);
                open = false;
            }
            const bool was_last = k.last;
            chunk_next(k, span, m.dp, inv_dp, n);
            if (was_last) seen_first = true;
        }
    }
    // the dump still open at the end of this block's range
    if (active && open) finish_dump(acc, s_lds, s_base, lane, ch, jmin, k.m, false, d);
}

template <int FMT>
void launch_one(const uint8_t* samples, uint64_t n, const DevChan* chans, const DevMeta* meta,
                gc_chan_state* state, int n_chan, int32_t* out, int tap_stride, uint32_t max_dumps,
                const uint32_t* tables, int grid, hipStream_t s) {
    const uint32_t n_tiles = (uint32_t)((n + kTile - 1) / kTile);
    const int g = (int)min((uint32_t)grid, n_tiles);
    const int waves = min(n_chan, kWaves);
    const int groups = (n_chan + kWaves - 1) / kWaves;
    hipLaunchKernelGGL((k_mtap<FMT>), dim3(g, groups), dim3(64 * waves), 0, s, samples, n, chans,
                       meta, state, out, tap_stride, max_dumps, tables, n_chan, n_tiles);
}

}  // namespace

hipError_t launch_mtap(const uint8_t* samples, uint64_t n, int fmt, const DevChan* chans,
                       const DevMeta* meta, gc_chan_state* state, int n_chan, int32_t* out,
                       int tap_stride, uint32_t max_dumps, const uint32_t* tables, int grid,
                       hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (fmt == GC_I8_IQ)
        launch_one<GC_I8_IQ>(samples, n, chans, meta, state, n_chan, out, tap_stride, max_dumps,
                             tables, grid, s);
    else if (fmt == GC_I8_REAL)
        launch_one<GC_I8_REAL>(samples, n, chans, meta, state, n_chan, out, tap_stride, max_dumps,
                               tables, grid, s);
    else if (fmt == GC_I2_REAL)
        launch_one<GC_I2_REAL>(samples, n, chans, meta, state, n_chan, out, tap_stride, max_dumps,
                               tables, grid, s);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace gc
