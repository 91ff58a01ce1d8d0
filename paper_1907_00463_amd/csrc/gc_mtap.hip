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
// Stage 1 scatters the samples into S, one window of 32 chips at a time, in
// LDS.  Windows are aligned to multiples of 32 chips, so a cell's address is
// a bit field of U: (U >> 25) & 0xFFC = 128 * (c mod 32) + 4 * q.  A window
// that holds the end of a dump is taken twice, once for each dump.
// A cell holds four int8: the wiped-off I and Q (|w| <= 128*34) each split
// as w = lo + 256*hi with lo in [-128, 127]: the 16-bit (w + 128) XOR 0x80
// holds lo in its low and hi in its high byte, so the pack is one XOR (the
// +128 rides in the wipe-off's multiply-add).  The contraction index runs
// over (chip, byte of the cell) and the 32 columns are (byte b, shift j):
// the replica operand of column (b, j) holds C in byte b of each chip word.
// One v_mfma_i32_32x32x32_i8 per 8 chips (each lane half taking every
// other chip) gives exact int32 T for the four
// bytes of 8 shifts; at the dump's end I = T_0 + 256 T_1, Q = T_2 + 256 T_3,
// prefix sums over q turn every tap into two range sums (stage 3), and the
// dump is stored.
//
// One wave per channel (16 per block), blocks take contiguous chunks of
// sample tiles; the tile (4 B per sample: (xI, xQ) as int16) and a 4-copy
// carrier table of (c, s, s, -s) entries are shared by the block's waves.
// The complex wipe-off is two packed int16 multiply-adds per sample (the
// (xQ, xI) operand by a half swap of the sample word); lanes take
// consecutive samples.  The window walk runs on uniform (scalar) values.
#include "gc_device.h"

namespace gc {

namespace {

constexpr int kWaves = 16;
constexpr int kChunkChips = 32;                   // chips per window (4 MFMA K steps of 8)
constexpr int kRows = 32;                         // q
constexpr int kSBytes = kChunkChips * kRows * 4;  // 4096 per wave, cell (p, q) at 128 p + 4 q
constexpr int kLutCopies = 4;
constexpr int kLutStride = 514;                   // words between copies (256 two-word entries + 2)
constexpr int kLutBytes = kLutCopies * kLutStride * 4;
constexpr int kTile = 20704;                      // samples per tile (what the LDS leaves)
constexpr int kMargin = kChunkChips * 32 + 64 + 128;  // <= 32 chips of <= 32 samples, + one pair read ahead
constexpr int kXSamples = kTile + kMargin;
constexpr int kOffS = 0;                          // S areas first: bases are multiples of 4096
constexpr int kOffLut = kOffS + kWaves * kSBytes;
constexpr int kOffX = kOffLut + kLutBytes;
constexpr int kOffList = kOffX + kXSamples * 4;
// 256 zero entries: the carrier table of direct-form lanes whose row holds no
// sample (their cells come out 0 with no branch); offset by 32 banks from
// the first table copy, so that the same entry of both is in different banks
constexpr int kOffZero = ((kOffList + 4 * (kWaves + 1) + 255) & ~255) + (((kOffLut / 4 + 32) % 64) * 4);
constexpr int kLdsBytes = kOffZero + 256 * 8;
static_assert(kLdsBytes <= 160 * 1024, "LDS per block");
static_assert(kOffS % 4096 == 0 && kSBytes == 4096, "cell offset = (U >> 25) & 0xFFC | wave base");
static_assert((kOffZero / 4 - kOffLut / 4) % 64 == 32, "zero table 32 banks from the first copy");
static_assert(kTile % 16 == 0 && kXSamples % 16 == 0, "staging granule");
static_assert(16 * 33 * 4 <= kSBytes, "stage-3 prefix sums fit the wave's S area");
static_assert(2 * kMtapHalfWords >= 1022 + 1022 + 1 + 24 + 8, "replica operand reads stay in the table");

typedef short short2_t __attribute__((ext_vector_type(2)));
typedef int int4_t __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ short2_t as_s2(uint32_t v) { return __builtin_bit_cast(short2_t, v); }

__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// a uniform value computed on the VALU, moved to an SGPR: the empty asm
// keeps the conversion before the read-first-lane (the compiler otherwise
// hoists the read above it and leaves the rest of the window walk in VGPRs)
__device__ __forceinline__ uint32_t to_sgpr(uint32_t v) {
    asm("" : "+v"(v));
    return __builtin_amdgcn_readfirstlane(v);
}

// ceil(num / d), d in [2^27, 2^31): a double estimate (within one of the
// quotient) made exact by a bounded correction.
__device__ __forceinline__ uint64_t ceil_div(uint64_t num, uint64_t d) {
    uint64_t q = (uint64_t)((double)num / (double)d);
    for (int i = 0; i < 4 && q * d < num; ++i) ++q;
    for (int i = 0; i < 4 && q > 0 && (q - 1) * d >= num; ++i) --q;
    return q;
}

// One chunk: the chips [cs, ce) of dump m inside the aligned window
// [w0, w0 + 32), samples [sa, sb).  Chunks are walked in order; the first
// sample of the next chunk follows from the overshoot of this one
// (e = sb*dp - (ce*2^32 - p0), in [0, dp)) without a division by the code step.
struct Chunk {
    uint64_t cs, ce;   // chips [cs, ce)
    uint64_t w0;       // window start, a multiple of 32
    uint64_t d0;       // first chip of the dump (span * m)
    uint64_t sa, sb;   // samples [sa, sb), clipped to [0, n]
    uint64_t fb;       // first sample of chip ce (unclipped)
    uint64_t eb;       // its overshoot
    uint32_t m;        // dump (window) index
    uint32_t wmod;     // w0 mod 1023: the code chip of window position 0
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

// The chunk of chip c.  A dump spans a whole number of code periods, so the
// code chip of chip c is c mod 1023 whatever the dump.
__device__ __forceinline__ Chunk chunk_of(uint64_t c, uint64_t span, uint64_t p0, uint64_t dp,
                                          uint64_t n) {
    Chunk k;
    k.m = (uint32_t)(c / span);
    k.d0 = (uint64_t)k.m * span;
    k.w0 = c & ~(uint64_t)(kChunkChips - 1);
    k.cs = max(k.d0, k.w0);
    k.ce = min(k.w0 + kChunkChips, k.d0 + span);
    k.first = k.cs == k.d0;
    k.last = k.ce == k.d0 + span;
    k.wmod = (uint32_t)(k.w0 % kCodeLen);
    uint64_t fa, ea;
    chip_first(k.cs, p0, dp, fa, ea);
    chip_first(k.ce, p0, dp, k.fb, k.eb);
    k.sa = min(n, fa);
    k.sb = min(n, k.fb);
    // every field is uniform (the arguments are); keep them in scalar
    // registers so that the walk stays on the scalar unit
    k.fb = uni64(k.fb);
    k.eb = uni64(k.eb);
    k.sa = uni64(k.sa);
    k.sb = uni64(k.sb);
    return k;
}

// The chunk after k: its first sample is k's end; its end advances by
// ceil(((ce' - ce)*2^32 - eb) / dp) samples (one or two candidates around a
// float estimate two below the quotient, stepped up exactly; the float
// error is far below one sample, so a few steps always suffice).
// For a full 32-chip chunk after a full one the sample count is
// ceil((32*2^32 - eb)/dp) with eb in [0, dp): qhi = ceil(32*2^32/dp) or
// qhi - 1, the latter exactly when the numerator is at most (qhi - 1)*dp.
struct FullStep {
    uint64_t qhi, p1, pq;  // qhi, (qhi - 1)*dp, qhi*dp
};

__device__ __forceinline__ void chunk_next(Chunk& k, uint64_t span, uint64_t dp, float inv_dp,
                                           uint64_t n, const FullStep& fs) {
    if (!k.last && k.ce + kChunkChips <= k.d0 + span) {  // a full window after a full window
        k.cs = k.ce;
        k.w0 = k.ce;
        k.wmod += kChunkChips;
        if (k.wmod >= kCodeLen) k.wmod -= kCodeLen;
        k.ce += kChunkChips;
        k.first = false;
        k.last = k.ce == k.d0 + span;
        k.sa = k.sb;
        const uint64_t num = ((uint64_t)kChunkChips << 32) - k.eb;
        const bool hiq = num > fs.p1;
        k.fb += hiq ? fs.qhi : fs.qhi - 1;
        k.eb = (hiq ? fs.pq : fs.p1) - num;
        k.sb = min(n, k.fb);
        return;
    }
    if (k.last) {
        k.m += 1;
        k.d0 += span;
    }
    const uint64_t w0 = k.ce & ~(uint64_t)(kChunkChips - 1);
    if (w0 != k.w0) {
        k.wmod += kChunkChips;
        if (k.wmod >= kCodeLen) k.wmod -= kCodeLen;
        k.w0 = w0;
    }
    k.cs = k.ce;
    k.ce = min(k.w0 + kChunkChips, k.d0 + span);
    k.first = k.cs == k.d0;
    k.last = k.ce == k.d0 + span;
    k.sa = k.sb;
    const uint32_t nch = (uint32_t)(k.ce - k.cs);          // 1 .. 32
    const uint64_t num = ((uint64_t)nch << 32) - k.eb;      // > 0
    const float est = ((float)nch * 4294967296.0f - (float)(uint32_t)k.eb) * inv_dp;
    uint64_t q = to_sgpr((uint32_t)max(0.0f, est - 2.0f));
    for (int i = 0; i < 8 && q * dp < num; ++i) ++q;
    k.fb += q;
    k.eb = q * dp - num;
    k.sb = min(n, k.fb);
}

// Tile samples [t0, t0 + count) as two int16 pairs each: (xI, xQ) and
// (xQ, -xI) (real input: (x, 0) and (0, -x)); zero past the block.  Each
// thread takes units of 8 samples: one 16-byte (complex int8), 8-byte (real
// int8), 4-byte (2-bit complex) or 2-byte (2-bit real) load, four 16-byte
// LDS stores.
template <int FMT>
__device__ __forceinline__ void stage_tile(const uint8_t* __restrict__ samples, uint64_t n,
                                           uint64_t t0, uint8_t* lds, int nthreads,
                                           uint32_t count) {
    static_assert(kXSamples % 8 == 0, "staging unit");
    uint4* dst = reinterpret_cast<uint4*>(lds + kOffX);
    const uint32_t avail = (uint32_t)min(n - t0, (uint64_t)count);
    for (int u = threadIdx.x; u < (int)count / 8; u += nthreads) {
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
        } else if constexpr (FMT == GC_I2_IQ) {
            // two samples per byte, I then Q code in each nibble
            const uint8_t* src = samples + (t0 + s0) / 2;
            uint32_t w = 0;
            if (whole) {
                w = *reinterpret_cast<const uint32_t*>(src);
            } else {
                for (uint32_t b = 0; b < 4; ++b)
                    if (s0 + 2 * b < avail) w |= (uint32_t)src[b] << (8 * b);
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint32_t nib = (w >> (4 * k)) & 15u;
                xi[k] = 2 * (int)(nib & 3u) - 3;
                xq[k] = 2 * (int)(nib >> 2) - 3;
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
        for (int k = 0; k < 8; k += 4) {
            uint32_t o[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                o[j] = (uint32_t)(uint16_t)xi[k + j] | ((uint32_t)(uint16_t)xq[k + j] << 16);
            dst[(s0 + k) / 4] = uint4{o[0], o[1], o[2], o[3]};
        }
    }
}

// Stage 1 for one sample: the wiped-off (wI, wQ) + 128 as int16 pairs,
// (xI, xQ) c + ((xQ, xI) (s, -s) + 128), the swapped sample pair and the
// table entry's second word (s, -s): every product and sum stays below 2^15
// in magnitude (|x c| <= 3072, |w| <= 4352), so the 16-bit lanes hold the
// exact values; XOR 0x80 per half gives the cell bytes (lo, hi).  The empty
// asm keeps the +128 inside the first packed multiply-add (the compiler
// would otherwise add it separately after both products).
__device__ __forceinline__ uint32_t cell_of(uint32_t xw, uint2 cs, short2_t k128) {
    const short2_t x = as_s2(xw);
    const short2_t c2 = as_s2(cs.x);
    const short2_t cc = __builtin_shufflevector(c2, c2, 0, 0);
    short2_t p = __builtin_shufflevector(x, x, 1, 0) * as_s2(cs.y) + k128;
    asm("" : "+v"(p));
    const short2_t w2 = x * cc + p;
    return __builtin_bit_cast(uint32_t, w2) ^ 0x00800080u;
}

// offset of the cell of code phase U in the wave's S area; s_base_v (a
// multiple of 4096 from the start of the block's LDS) is a value whose bits
// the compiler does not see, so the OR stays one v_and_or_b32
__device__ __forceinline__ uint32_t cell_addr(uint64_t U, uint32_t s_base_v) {
    return ((uint32_t)(U >> 25) & 0xFFCu) | s_base_v;
}

struct Dest {
    int32_t* out;
    gc_chan_state* st;
    uint64_t row0;
    int tap_stride;
    uint32_t m_close;
};

// Stage 3 for the dump held in acc (column l32 = 8 b + j: byte b of shift
// jmin + j; element e is row q = 8 (e / 4) + 4 h + e % 4): I and Q of each
// (q, j) from the lo and hi bytes (lane + 8 holds the hi byte), prefix sums
// over q in the wave's S area, two range sums per tap, stored (plain or
// atomic).
__device__ __forceinline__ void finish_dump(i32x16& acc, uint8_t* lds, uint32_t s_base,
                                            uint32_t lane, const DevChan& ch, int jmin,
                                            uint32_t m, bool plain, const Dest& d) {
    int32_t* P = reinterpret_cast<int32_t*>(lds + s_base);  // [plane * 8 + j][33]
    const uint32_t l32 = lane & 31, h = lane >> 5;
    const uint32_t seq = (l32 >> 4) * 8 + (l32 & 7);
    const bool lo_lane = (l32 & 8) == 0;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int hi = __builtin_amdgcn_update_dpp(0, acc[e], 0x108, 0xf, 0xf, false);  // row_shl:8
        const int v = acc[e] + 256 * hi;
        if (lo_lane) P[seq * 33 + 8 * (e / 4) + 4 * h + (e % 4)] = v;
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
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = 0;
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
                                                      int n_chan, uint32_t n_tiles,
                                                      uint32_t tile_len) {
    __shared__ __attribute__((aligned(16))) uint8_t s_lds[kLdsBytes];
    int* s_list = reinterpret_cast<int*>(s_lds + kOffList);
    const int tid = threadIdx.x;
    const int nthreads = blockDim.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
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
    const int nlist = __builtin_amdgcn_readfirstlane(s_list[kWaves]);
    if (nlist == 0) return;
    {
        // entry e of a copy: (c, s) of the table, then (s, -s)
        uint32_t* lut = reinterpret_cast<uint32_t*>(s_lds + kOffLut);
        for (int i = tid; i < kLutCopies * kLutStride; i += nthreads) {
            const int w = i % kLutStride, e = w / 2;
            uint32_t v = 0u;
            if (e < 256) {
                const uint32_t cs = tables[kTabLut + e];
                const uint32_t sn = cs >> 16;
                v = (w & 1) ? sn | ((uint32_t)(uint16_t)(-(int16_t)sn) << 16) : cs;
            }
            lut[i] = v;
        }
        uint32_t* zero = reinterpret_cast<uint32_t*>(s_lds + kOffZero);
        for (int i = tid; i < 512; i += nthreads) zero[i] = 0u;
    }

    const bool active = wave < nlist;
    const int chn = __builtin_amdgcn_readfirstlane(active ? s_list[wave] : 0);
    const DevChan& ch = chans[chn];
    const DevMeta m = metas[chn];
    const Dest d{out, state + chn, (uint64_t)chn * max_dumps, tap_stride, m.m_close};
    const uint64_t span = m.window >> 32;
    const uint32_t s_base = kOffS + (uint32_t)wave * kSBytes;  // offset from s_lds
    uint32_t s_base_v = s_base;
    asm("" : "+v"(s_base_v));
    const short2_t k128 = {128, 128};
    // carrier table reads: a slow carrier (the 64 lanes of a step span fewer
    // than 32 consecutive entries, e.g. complex baseband with Doppler) reads
    // one copy, where lanes on one entry are a broadcast and distinct entries
    // fall in distinct banks; a fast one (IF input) spreads the lanes over
    // the 4 copies so that entries a multiple of 32 apart collide less (16
    // copies measured no faster on IF input and cost a fifth of the tile)
    const uint32_t adphi = (int32_t)m.dphi < 0 ? 0u - m.dphi : m.dphi;
    const bool one_copy = (uint64_t)adphi * 64 <= (31ull << 24);
    const uint32_t lut_base = kOffLut + (one_copy ? 0u : (lane & (kLutCopies - 1)) * kLutStride * 4);
    const int jmin = ch.mt_jmin;
    const float inv_dp = 1.0f / (float)m.dp;
    FullStep fs;
    fs.qhi = uni64(ceil_div((uint64_t)kChunkChips << 32, m.dp));
    fs.p1 = (fs.qhi - 1) * m.dp;
    fs.pq = fs.qhi * m.dp;
    const uint32_t l32 = lane & 31, h = lane >> 5;
    // replica operand: column l32 = 8 b + j takes the byte-b table of the
    // PRN at chip (window chip + shift jmin + j); in K step ks lane half h
    // covers window positions 8 ks + h + 2 i (i = 0..3), four chips two
    // apart: one 16-byte read from the table of their parity
    const int jsh = (int)(((int64_t)jmin + (int64_t)(l32 & 7)) % kCodeLen);
    const uint32_t b_lane = (uint32_t)(jsh < 0 ? jsh + kCodeLen : jsh) + h;
    const uint32_t* btab = tables + kTabMtapCode + ((ch.prn - 1) * 4 + (int)(l32 >> 3)) * kMtapCodeWords;
    // word offsets of the lane's first chip in the parity tables, for an even
    // and an odd window code chip wmod (the chip is wmod + b_lane: parity
    // (wmod + b_lane) & 1, word (wmod + b_lane) >> 1)
    const uint32_t boff_e = (b_lane & 1u) * kMtapHalfWords + (b_lane >> 1);
    const uint32_t boff_o = ((b_lane + 1u) & 1u) * kMtapHalfWords + ((b_lane + 1u) >> 1);
    // per-lane parts of the sample walk
    const uint64_t lane_dU = (uint64_t)lane * m.dp;
    const uint32_t lane_dph = lane * m.dphi;
    const uint64_t dU = 64ull * m.dp;
    const uint32_t dph = 64u * m.dphi;
    // the step increments as VGPR values: the compiler then adds them
    // directly instead of keeping scalar running offsets
    uint64_t dUv = dU, dU2v = 2 * dU;
    uint32_t dph2v = 2 * dph;
    asm("" : "+v"(dUv));
    asm("" : "+v"(dU2v));
    asm("" : "+v"(dph2v));
    // A fragment of K step ks: window positions 8 ks + h + 2 i, row l32
    // (the two lane halves read chips one apart: distinct banks)
    const uint32_t a_base = s_base + 128u * h + 4u * l32;
    // Direct-cell form (rates where two chips span close to a whole number
    // D2 of samples): the sample of cell (q, c) is n = ceil(N / dp) with
    // N = c 2^32 + q 2^27 - P, present when r = n dp - N < 2^27.  Two chips
    // on, N grows by 2^33, so n grows by D2 and r by d2 = D2 dp - 2^33 as
    // long as r stays in [0, dp); while it also stays on its side of 2^27
    // for all 16 positions of a lane's half, the lane's cells are a fixed
    // sample stride apart and the lane forms its MFMA operand in registers.
    // (code steps below 2^30, so that r and its drift over a window stay in
    // int32)
    const uint64_t D2 = uni64((uint64_t)(8589934592.0 / (double)m.dp + 0.5));
    const int64_t d2l = (int64_t)(D2 * m.dp) - (int64_t)(1ull << 33);
    const bool direct_ok = m.dp < (1ull << 30) && d2l >= -(1ll << 18) && d2l <= (1ll << 18);
    const int32_t d2 = (int32_t)d2l;
    const uint32_t dp32 = (uint32_t)m.dp;
    const uint32_t X2 = 4u * (uint32_t)D2;          // tile bytes per two chips
    const uint32_t F2 = (uint32_t)D2 * m.dphi;      // carrier phase per two chips
    const uint32_t X2s = __builtin_amdgcn_readfirstlane(X2);
    const uint32_t F2s = __builtin_amdgcn_readfirstlane(F2);
    const uint64_t Z2s = ((uint64_t)F2s << 32) | X2s;  // both strides in one word

    // contiguous chunk of tiles for this block; chunks belong to the tile
    // holding their first sample
    const uint32_t tb0 = (uint32_t)(((uint64_t)blockIdx.x * n_tiles) / gridDim.x);
    const uint32_t tb1 = (uint32_t)(((uint64_t)(blockIdx.x + 1) * n_tiles) / gridDim.x);
    const uint64_t T0 = (uint64_t)tb0 * tile_len;
    const uint32_t staged = tile_len + kMargin;  // samples staged per tile

    i32x16 acc0;
#pragma unroll
    for (int e = 0; e < 16; ++e) acc0[e] = 0;
    Chunk k = chunk_of((m.p0 + T0 * m.dp) >> 32, span, m.p0, m.dp, n);
    if (T0 > 0 && k.sa < T0) k = chunk_of(k.ce, span, m.p0, m.dp, n);
    bool seen_first = k.first;  // this wave holds the dump from its first chunk
    bool open = false;          // acc0 holds part of dump k.m
    // sample sa of the current chunk (uniform): code phase, carrier phase,
    // and tile address (relative to the tile being worked on); each chunk
    // advances them by its sample count
    uint64_t Ua;
    uint32_t pha, xsa;
    {
        const uint64_t sa = uni64(k.sa);
        Ua = m.p0 + sa * m.dp;
        pha = m.phi0 + (uint32_t)sa * m.dphi;
        xsa = kOffX + (uint32_t)(sa - T0) * 4u;
    }
    auto x_at = [&](uint32_t a) { return *reinterpret_cast<const uint32_t*>(s_lds + a); };
    auto lut_at = [&](uint32_t phase) {
        return *reinterpret_cast<const uint2*>(s_lds + lut_base + ((phase >> 24) << 3));
    };
    auto cell_store = [&](uint32_t a, uint32_t v) { *reinterpret_cast<uint32_t*>(s_lds + a) = v; };

    // direct-form state of the lane's cell (l32, dw0 + h): its sample's tile
    // address and carrier phase, and r; advanced by one window after every
    // window, recomputed when the next window is not the one it refers to
    uint32_t dx = 0, df = 0;
    int32_t dr = 0;
    uint64_t dw0 = ~0ull;
    for (uint32_t tile = tb0; tile < tb1; ++tile) {
        const uint64_t t0 = (uint64_t)tile * tile_len;
        const uint64_t t1 = min(n, t0 + tile_len);
        __syncthreads();
        stage_tile<FMT>(samples, n, t0, s_lds, nthreads, staged);
        __syncthreads();
        if (!active) continue;
        if (tile > tb0) {
            xsa -= 4u * tile_len;
            dx -= 4u * tile_len;
        }
        while (k.sa < t1 && k.sa < k.sb) {
            // the window's replica operand, in flight during stage 1
            int4_t bop[4];
            {
                const uint32_t* bp = btab + ((k.wmod & 1u) ? boff_o : boff_e) + (k.wmod >> 1);
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) bop[ks] = *reinterpret_cast<const int4_t*>(bp + 4 * ks);
            }
            const uint32_t adv = __builtin_amdgcn_readfirstlane((uint32_t)(k.sb - k.sa));
            // direct-cell form: a whole window inside the block, every lane's
            // cells on one side of their row boundaries (decided per lane,
            // taken only when every lane agrees)
            bool direct = false;
            uint32_t lutb = lut_base;
            if (direct_ok && k.cs == k.w0 && k.ce == k.w0 + kChunkChips && k.fb <= n &&
                (k.cs << 32) >= m.p0) {
                if (dw0 != k.w0) {
                    // exact: cell (l32, w0 + h) relative to sample sa, the
                    // first sample of chip w0 (uniform: lane 0's walk values):
                    // N = h 2^32 + l32 2^27 - (U_sa mod 2^32), n = ceil(N / dp)
                    const uint32_t fsa = (uint32_t)Ua;
                    const int64_t N0 = ((int64_t)h << 32) + ((int64_t)l32 << 27) - (int64_t)fsa;
                    const float est =
                        ((float)h * 4294967296.0f + (float)(l32 << 27) - (float)fsa) * inv_dp;
                    int32_t n0 = (int32_t)ceilf(est);
                    int64_t r = (int64_t)n0 * (int64_t)m.dp - N0;
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        if (r < 0) { r += (int64_t)m.dp; ++n0; }
                        if (r >= (int64_t)m.dp) { r -= (int64_t)m.dp; --n0; }
                    }
                    dr = (int32_t)r;
                    dx = xsa + 4u * (uint32_t)n0;
                    df = pha + (uint32_t)n0 * m.dphi;
                    dw0 = k.w0;
                }
                // r at the lane's last position; the cells of the window
                // follow the first one's pattern when r stays in [0, dp) on
                // one side of 2^27 (r is linear in the position)
                const int32_t rhi = dr + 15 * d2;
                const bool occ = dr < (1 << 27);
                const bool ok = (uint32_t)dr < dp32 && (uint32_t)rhi < dp32 && (rhi < (1 << 27)) == occ;
                direct = __all(ok);
                lutb = occ ? lut_base : (uint32_t)kOffZero;
            }
            if (!direct) dw0 = ~0ull;
            // opaque, so that each cell is one add from these (not a
            // multiply of its sample index)
            uint32_t x0 = dx, f0 = df;
            asm("" : "+v"(x0));
            asm("" : "+v"(f0));
            // the window's four MFMA operands (either form), then one MFMA
            // chain for both: the accumulator stays in one register set
            int4_t aop[4];
            if (direct) {
                // stage 1 in registers: dword i of K step ks is the cell of
                // window position 8 ks + h + 2 i, row l32
                // (one K step at a time, the next step's reads issued before
                // this step's arithmetic; a lane whose row holds no sample
                // reads the zero table and forms 0 cells)
                uint32_t xv[4];
                uint2 cv[4];
                // running sample address (low word) and carrier phase (high
                // word), stepped by the uniform two-chip strides with one
                // 64-bit add: the address stays far below 2^32, so no carry
                // reaches the phase, and the phase wraps as a 32-bit word
                uint64_t zc = ((uint64_t)f0 << 32) | x0;
                auto load_step = [&](uint32_t* xs, uint2* cs) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        cs[i] = *reinterpret_cast<const uint2*>(s_lds + lutb + ((uint32_t)(zc >> 56) << 3));
                        xs[i] = x_at((uint32_t)zc);
                        zc += Z2s;
                    }
                };
                load_step(xv, cv);
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    uint32_t xn[4];
                    uint2 cn[4];
                    if (ks < 3) load_step(xn, cn);
                    // cell_of for four cells, the +128 kept inside the first
                    // multiply-add of each
                    short2_t pp[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const short2_t x = as_s2(xv[i]);
                        pp[i] = __builtin_shufflevector(x, x, 1, 0) * as_s2(cv[i].y) + k128;
                    }
                    asm("" : "+v"(pp[0]), "+v"(pp[1]), "+v"(pp[2]), "+v"(pp[3]));
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const short2_t c2 = as_s2(cv[i].x);
                        const short2_t w2 = as_s2(xv[i]) * __builtin_shufflevector(c2, c2, 0, 0) + pp[i];
                        aop[ks][i] = (int)(__builtin_bit_cast(uint32_t, w2) ^ 0x00800080u);
                    }
                    if (ks < 3) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            xv[i] = xn[i];
                            cv[i] = cn[i];
                        }
                    }
                }
            } else {
                // stage 1: clear S (32 x 32 cells), scatter the chunk's samples
                {
                    uint4* z = reinterpret_cast<uint4*>(s_lds + s_base) + lane;
#pragma unroll
                    for (int c = 0; c < 4; ++c) z[64 * c] = uint4{0u, 0u, 0u, 0u};
                }
                wave_fence();
                // at most 32 chips of at most 32 samples, inside the staged tile
                const uint32_t cnt = min(adv, (uint32_t)(staged - (uint32_t)(k.sa - t0)));
                uint64_t U = Ua + lane_dU;
                uint32_t ph = pha + lane_dph, xa = xsa + lane * 4u;
                // pairs of full steps, software-pipelined over two register
                // sets: the reads of the next pair (unconditional: the staged
                // tile extends one pair past any chunk) are issued before the
                // stores of the current one
                uint32_t pairs = __builtin_amdgcn_readfirstlane(cnt / 128);
                if (pairs > 0) {
                    uint32_t xa0 = x_at(xa), xa1 = x_at(xa + 256u);
                    uint2 ca0 = lut_at(ph), ca1 = lut_at(ph + dph);
                    uint32_t xb0, xb1;
                    uint2 cb0, cb1;
                    for (;;) {
                        {
                            const uint32_t v0 = cell_of(xa0, ca0, k128), v1 = cell_of(xa1, ca1, k128);
                            const uint32_t a0 = cell_addr(U, s_base_v), a1 = cell_addr(U + dUv, s_base_v);
                            U += dU2v;
                            ph += dph2v;
                            xa += 512u;
                            xb0 = x_at(xa);
                            xb1 = x_at(xa + 256u);
                            cb0 = lut_at(ph);
                            cb1 = lut_at(ph + dph);
                            cell_store(a0, v0);
                            cell_store(a1, v1);
                            if (--pairs == 0) break;
                        }
                        {
                            const uint32_t v0 = cell_of(xb0, cb0, k128), v1 = cell_of(xb1, cb1, k128);
                            const uint32_t a0 = cell_addr(U, s_base_v), a1 = cell_addr(U + dUv, s_base_v);
                            U += dU2v;
                            ph += dph2v;
                            xa += 512u;
                            xa0 = x_at(xa);
                            xa1 = x_at(xa + 256u);
                            ca0 = lut_at(ph);
                            ca1 = lut_at(ph + dph);
                            cell_store(a0, v0);
                            cell_store(a1, v1);
                            if (--pairs == 0) break;
                        }
                    }
                }
                // the last 0 .. 127 samples: one pair with masked stores
                const uint32_t rest = cnt % 128;
                if (rest > 0) {
                    const uint32_t v0 = cell_of(x_at(xa), lut_at(ph), k128);
                    const uint32_t v1 = cell_of(x_at(xa + 256u), lut_at(ph + dph), k128);
                    const uint32_t a0 = cell_addr(U, s_base_v), a1 = cell_addr(U + dUv, s_base_v);
                    if (lane < rest) cell_store(a0, v0);
                    if (lane + 64 < rest) cell_store(a1, v1);
                }
                wave_fence();
                // stage 2 operands: four K steps of 8 chips, 32 rows q
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const uint8_t* ap = s_lds + a_base + 1024u * ks;
                    aop[ks] = int4_t{*reinterpret_cast<const int*>(ap),
                                     *reinterpret_cast<const int*>(ap + 256),
                                     *reinterpret_cast<const int*>(ap + 512),
                                     *reinterpret_cast<const int*>(ap + 768)};
                }
            }
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                acc0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(aop[ks], bop[ks], acc0, 0, 0, 0);
            dx += 16u * X2;
            df += 16u * F2;
            dr += 16 * d2;
            dw0 += kChunkChips;
            open = true;
            if (k.last) {
                finish_dump(acc0, s_lds, s_base, lane, ch, jmin, k.m, seen_first && k.m > 0, d);
                open = false;
            }
            Ua += (uint64_t)adv * m.dp;
            pha += adv * m.dphi;
            xsa += 4u * adv;
            const bool was_last = k.last;
            chunk_next(k, span, m.dp, inv_dp, n, fs);
            if (was_last) seen_first = true;
        }
    }
    // the dump still open at the end of this block's range
    if (active && open) {
        finish_dump(acc0, s_lds, s_base, lane, ch, jmin, k.m, false, d);
    }
}

template <int FMT>
void launch_one(const uint8_t* samples, uint64_t n, const DevChan* chans, const DevMeta* meta,
                gc_chan_state* state, int n_chan, int32_t* out, int tap_stride, uint32_t max_dumps,
                const uint32_t* tables, int grid, hipStream_t s) {
    // every block takes the same number of tiles: k = ceil(n / (kTile grid))
    // each, of ceil(n / (k grid)) samples rounded up to 16 (at most kTile, at
    // least kMinTile)
    constexpr uint64_t kMinTile = 2048;
    const uint64_t G = (uint64_t)max(grid, 1);
    const uint64_t per = (n + (uint64_t)kTile * G - 1) / ((uint64_t)kTile * G);
    uint64_t tl = (n + per * G - 1) / (per * G);
    tl = min((uint64_t)kTile, max(kMinTile, (tl + 15) & ~15ull));
    const uint32_t tile_len = (uint32_t)tl;
    const uint32_t n_tiles = (uint32_t)((n + tl - 1) / tl);
    const int g = (int)min((uint32_t)grid, n_tiles);
    const int waves = min(n_chan, kWaves);
    const int groups = (n_chan + kWaves - 1) / kWaves;
    hipLaunchKernelGGL((k_mtap<FMT>), dim3(g, groups), dim3(64 * waves), 0, s, samples, n, chans,
                       meta, state, out, tap_stride, max_dumps, tables, n_chan, n_tiles,
                       tile_len);
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
    else if (fmt == GC_I2_IQ)
        launch_one<GC_I2_IQ>(samples, n, chans, meta, state, n_chan, out, tap_stride, max_dumps,
                             tables, grid, s);
    else if (fmt == GC_I2_REAL)
        launch_one<GC_I2_REAL>(samples, n, chans, meta, state, n_chan, out, tap_stride, max_dumps,
                               tables, grid, s);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace gc
