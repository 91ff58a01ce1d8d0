// gc_pbin.hip -- early/prompt/late correlator for channels whose half-chip
// bins are periodic in the sample stream (integer carrier path, real int8
// and 2-bit samples).
//
// When fs is close to an integer multiple L of twice the code rate (L = 2 at
// 4.092 MHz, 4 at 8.184, 8 at 16.368, 10 at 20.46), every half chip of code
// phase covers exactly
// L samples, give or take one sample every |dp / (L*dp - 2^31)| bins (the
// code Doppler "slip").  Bin k of a run then starts at sample s_0 + k*L, so
// consecutive lanes can take consecutive bins with fixed per-lane offsets:
//
//   * a block streams through a contiguous chunk of tiles (of at most kTile
//     samples, sized per launch so that the blocks get equal shares),
//     staged once in LDS as int16 in two copies (aligned, and shifted by one
//     sample) so that every bin starts on a dword of one of them; each wave
//     owns one channel and keeps its E/P/L sums in registers across tiles,
//     reducing across lanes only when a dump closes;
//   * lane l of a wave takes bins k0 + 64j + l, j = 0, 1, ...: per sample one
//     phase add, one v_perm (address of the lane's own copy of the carrier
//     table), one table read and one packed int16 multiply-add; per pair of
//     samples one dword read; per bin two packed multiply-adds with the
//     early and late code signs of its chip (two consecutive entries of a
//     sign table, fetched two steps ahead) -- the prompt sign of a bin is its
//     early or its late sign, fixed for a lane over a run;
//   * with L = 8, bins start 4 dwords apart, so the lanes of each 8-lane
//     group read the dwords of their bin in a rotated order and one read
//     instruction touches 64 distinct LDS banks; with L = 4 (2 dwords apart)
//     lanes 16-47 read their second dword first; with L = 2 or 10 (1 or 5
//     dwords apart) the banks are distinct already;
//   * short bins take more steps per loop iteration (8 at L = 2, 4 at L = 4,
//     2 otherwise), their code signs fetched one iteration ahead;
//   * the step at which a dump closes is found per wave in advance; only that
//     step (and the ragged last step of a run) carries per-lane checks;
//   * a tile in which the bin grid slips by one sample is split into two
//     periodic runs, and the one sample at the seam is corrected with one
//     atomic update per output word.
// The result equals the per-sample definition exactly (integer sums
// regrouped).  Channels whose bins are not periodic use the chip-by-chip
// binned kernel or the direct path.
#include "gc_device.h"

namespace gc {

namespace {

constexpr int kTile = kPbinTileSamples;        // samples per tile
constexpr int kMarginS = 64;                   // bins that start in a tile end within this
constexpr int kXSamples = kTile + kMarginS;    // int16 samples per staged copy
constexpr int kXBytes = kXSamples * 2;
constexpr int kLutWords = 256 * 64;            // per-lane copies of the carrier table
constexpr int kXA = kLutWords * 4;             // LDS byte offset of copy A: A[i] = x[t0 + i]
constexpr int kXB = kXA + kXBytes;             // copy B: B[i] = x[t0 + i + 1]
constexpr int kLdsBytes = kXB + kXBytes;
constexpr int kMaxWaves = 16;                  // one channel per wave
constexpr uint32_t kPermSel = 0x0C0C0700u;     // byte1 = phase[31:24], byte0 = lane*4
// most 64-bin steps of one lane in a tile, and steps per loop iteration
constexpr int max_steps(int L) { return (kTile / L + 2 + 63) / 64; }
constexpr int unroll(int L) { return L <= 2 ? 8 : (L <= 4 ? 4 : 2); }
static_assert(max_steps(2) * 3 * GC_LUT_AMP * 2 <= 32767, "2-bit int16 sums, L = 2");
static_assert(max_steps(4) * 3 * GC_LUT_AMP * 4 <= 32767, "2-bit int16 sums, L = 4");
static_assert(max_steps(8) * 3 * GC_LUT_AMP * 8 <= 32767, "2-bit int16 sums, L = 8");
static_assert(max_steps(10) * 3 * GC_LUT_AMP * 10 <= 32767, "2-bit int16 sums, L = 10");
static_assert(max_steps(kPbinMinBinLen) <= kPbinMaxSteps && unroll(2) <= kPbinMaxAhead,
              "sign table sizes");
// sign words read: start chip <= 1022, then up to 32*(steps + ahead - 1) + 1 more
static_assert(kCodeLen - 1 + 32 * (kPbinMaxSteps + kPbinMaxAhead - 1) + 2 <= kSignLen,
              "sign table padding");
static_assert(kLdsBytes + 4 * (kMaxWaves + 1) <= 160 * 1024, "LDS per block");
static_assert((kTile / kPbinMinBinLen + 2) * kMaxWaves < (1 << 30), "32-bit bin shares");

typedef short short2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ short2_t as_s2(uint32_t v) { return __builtin_bit_cast(short2_t, v); }

__device__ __forceinline__ uint32_t lds_u32(const uint8_t* lds, uint32_t off) {
    return *reinterpret_cast<const uint32_t*>(lds + off);
}

struct Dest {
    int32_t* out;
    gc_chan_state* st;
    uint64_t row0;
    int tap_stride;
    uint32_t m_close;
    __device__ __forceinline__ int32_t* at(uint32_t w, int slot, int comp) const {
        if (w < m_close) return out + ((row0 + w) * tap_stride + slot) * 2 + comp;
        return &st->acc[slot][comp];
    }
};

// Persistent per-wave state of its channel: the E, P, L sums of the open
// dump (I, Q each; Q holds +x*s) as int32, and the sums of the current run.
// Within a run every bin of a lane lies in the same half of its chip, so
// its prompt sign equals its early sign (first half) or its late sign
// (second half): a run accumulates only E and L, and fold() adds the one of
// them that matches the lane's half to P.  For 2-bit input the run sums are
// packed int16 (at most max_steps(L) bins of |sum| <= 3*24*L per lane).
struct Slot {
    int v[6];              // E I, E Q, P I, P Q, L I, L Q
    short2_t e16, l16;     // run sums, 2-bit input
    int r[4];              // run sums, int8 input: E I, E Q, L I, L Q
    uint32_t w;            // dump of the open sums (wave-uniform)
    uint32_t wnext;        // first chip of dump w + 1
    bool init;
};

template <int FMT>
__device__ __forceinline__ void fold(Slot& s, uint32_t par) {
    if constexpr (FMT == GC_I2_REAL) {
        const short2_t p = par ? s.l16 : s.e16;
        s.v[0] += s.e16.x; s.v[1] += s.e16.y;
        s.v[2] += p.x;     s.v[3] += p.y;
        s.v[4] += s.l16.x; s.v[5] += s.l16.y;
        s.e16 = s.l16 = short2_t{0, 0};
    } else {
        s.v[0] += s.r[0]; s.v[1] += s.r[1];
        s.v[2] += par ? s.r[2] : s.r[0];
        s.v[3] += par ? s.r[3] : s.r[1];
        s.v[4] += s.r[2]; s.v[5] += s.r[3];
        s.r[0] = s.r[1] = s.r[2] = s.r[3] = 0;
    }
}

// Sum of the open dump over the wave's 64 lanes (all lanes active): lanes
// 0-5 receive the six totals (E I, E Q, P I, P Q, L I, L Q) and one atomic
// instruction adds them to their output words; Q is negated here (wipe-off
// Q = -x*s).
__device__ __forceinline__ void wave_flush(const Slot& s, const Dest& d, const DevChan& ch) {
    const uint32_t lane = threadIdx.x & 63;
    const int t = wave_total6(s.v);
    if (lane < 6 && t != 0) {
        const int slot = lane < 2 ? ch.slot_e : (lane < 4 ? ch.slot_p : ch.slot_l);
        atomicAdd(d.at(s.w, slot, (int)(lane & 1)), (lane & 1) ? -t : t);
    }
}

// Bin sum a with the code signs sg = (sL, sE) of chips (c + par - 1,
// c + par), each a packed (s, s) int16 word, into the run's E and L sums.
template <int FMT>
__device__ __forceinline__ void add_bin(Slot& s, short2_t a, uint2 sg) {
    if constexpr (FMT == GC_I2_REAL) {
        s.e16 = a * as_s2(sg.y) + s.e16;
        s.l16 = a * as_s2(sg.x) + s.l16;
    } else {
        const int ai = a.x, aq = a.y;
        const int e = (int)(short)(sg.y & 0xFFFF), l = (int)(short)(sg.x & 0xFFFF);
        s.r[0] += ai * e; s.r[1] += aq * e;
        s.r[2] += ai * l; s.r[3] += aq * l;
    }
}

// Sum over one bin of x * (c, s): dword j of the bin (samples 2j, 2j+1) is
// read at xaddr + roff[j]; sample i takes carrier phase ph + poff[i].
template <int L>
__device__ __forceinline__ short2_t bin_sum(const uint8_t* lds, uint32_t xaddr, uint32_t ph,
                                           const uint32_t (&roff)[L / 2], const uint32_t (&poff)[L],
                                           uint32_t lane4) {
    // all reads first, then the multiply-adds
    uint32_t xw[L / 2], cs[L];
#pragma unroll
    for (int j = 0; j < L / 2; ++j) xw[j] = lds_u32(lds, xaddr + roff[j]);
#pragma unroll
    for (int i = 0; i < L; ++i) cs[i] = lds_u32(lds, __builtin_amdgcn_perm(ph + poff[i], lane4, kPermSel));
    short2_t a = {0, 0}, b = {0, 0};  // even and odd samples: two independent chains
#pragma unroll
    for (int j = 0; j < L / 2; ++j) {
        const short2_t w = as_s2(xw[j]);
        const short2_t x0 = {w.x, w.x};
        const short2_t x1 = {w.y, w.y};
        a = x0 * as_s2(cs[2 * j]) + a;
        b = x1 * as_s2(cs[2 * j + 1]) + b;
    }
    return a + b;
}

// Bins [kb, ke) of the current tile, bin k starting at tile sample
// base + k*L, bin index h_a + k.  Lane l takes bins kb + 64j + l.
template <int FMT, int L>
__device__ __forceinline__ void periodic_run(Slot& S, const uint8_t* lds, uint32_t lane,
                                             uint32_t lane4, int64_t base, uint32_t h_a,
                                             uint32_t kb, uint32_t ke, uint64_t t0,
                                             const DevMeta& m, const DevChan& ch,
                                             const uint32_t* __restrict__ sgn_prn, uint32_t span,
                                             const Dest& d) {
    if (ke <= kb) return;
    constexpr int B = L / 2;               // dwords per bin
    constexpr int U = unroll(L);           // steps per loop iteration
    static_assert(L % 2 == 0 && (B % 2 == 1 || B == 2 || B == 4), "bank layout");
    // rotation of the dword order so that one read instruction of the wave
    // hits distinct banks (bins 2 or 4 dwords apart share bank classes)
    uint32_t g = 0;
    if constexpr (B == 4) {
        const uint32_t c8 = lane >> 3;
        g = (c8 ^ (c8 >> 2)) & 3u;
    } else if constexpr (B == 2) {
        g = ((lane >> 4) ^ (lane >> 5)) & 1u;
    }
    uint32_t roff[B];
    uint32_t poff[L];
#pragma unroll
    for (int j = 0; j < B; ++j) {
        const uint32_t jr = (B == 4 || B == 2) ? ((j + g) & (uint32_t)(B - 1)) : (uint32_t)j;
        roff[j] = 4u * jr;
        poff[2 * j] = 2u * jr * m.dphi;
        poff[2 * j + 1] = (2u * jr + 1u) * m.dphi;
    }
    // bins of one run all start on the same parity; pick the copy on which
    // they start on a dword
    const uint32_t par_s = (uint32_t)base & 1u;
    const uint32_t xbase = par_s ? (uint32_t)((int64_t)kXB + 2 * (base - 1))
                                 : (uint32_t)((int64_t)kXA + 2 * base);
    const uint32_t k0 = kb + lane;
    uint32_t xaddr = xbase + (uint32_t)(2 * L) * k0;
    uint32_t ph = m.phi0 + (uint32_t)(t0 + (uint64_t)(base + (int64_t)k0 * L)) * m.dphi;
    const uint32_t hk0 = h_a + k0;
    const uint32_t par = hk0 & 1u;
    // byte offset of the sign pair (chip c + par - 1, chip c + par); the
    // table repeats the code so that the offset only grows within a run
    uint32_t soff = 4u * (((hk0 >> 1) + par + kCodeLen - 1) % kCodeLen);
    const uint8_t* sgb = reinterpret_cast<const uint8_t*>(sgn_prn);
    // signs of steps j .. j + U - 1 (fetched one iteration ahead of their use)
    uint2 sg[U];
#pragma unroll
    for (int u = 0; u < U; ++u) sg[u] = *reinterpret_cast<const uint2*>(sgb + soff + 128u * u);

    constexpr uint32_t dx = 64u * 2u * L;
    const uint32_t dph = (uint32_t)(64 * L) * m.dphi;
    const uint32_t steps = (ke - kb + 63) / 64;
    const uint32_t full = (ke - kb) / 64;
    const uint32_t hfirst = h_a + kb;      // bin of lane 0 at step 0
    uint32_t j = 0;
    while (j < steps) {
        // first step at which lane 63's bin reaches chip wnext
        const uint32_t h_cross = 2u * S.wnext;
        const uint32_t jx = h_cross > hfirst + 63u ? (h_cross - hfirst - 63u + 63u) / 64u : 0u;
        const uint32_t jend = min(max(jx, j), full);
        for (; j + U <= jend; j += U) {
            short2_t a[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                a[u] = bin_sum<L>(lds, xaddr + u * dx, ph + (uint32_t)u * dph, roff, poff, lane4);
#pragma unroll
            for (int u = 0; u < U; ++u) add_bin<FMT>(S, a[u], sg[u]);
#pragma unroll
            for (int u = 0; u < U; ++u)
                sg[u] = *reinterpret_cast<const uint2*>(sgb + soff + 128u * (U + u));
            soff += 128u * U;
            xaddr += U * dx;
            ph += (uint32_t)U * dph;
        }
        for (; j < jend; ++j) {
            const short2_t a0 = bin_sum<L>(lds, xaddr, ph, roff, poff, lane4);
            add_bin<FMT>(S, a0, sg[0]);
#pragma unroll
            for (int u = 0; u + 1 < U; ++u) sg[u] = sg[u + 1];
            sg[U - 1] = *reinterpret_cast<const uint2*>(sgb + soff + 128u * U);
            soff += 128u;
            xaddr += dx;
            ph += dph;
        }
        if (j >= steps) break;
        // a step with a dump boundary, or the ragged last step
        {
            const uint32_t k = k0 + 64u * j;
            const bool valid = k < ke;
            const uint32_t c = (hk0 + 64u * j) >> 1;
            const bool ahead = valid && c >= S.wnext;
            short2_t a = bin_sum<L>(lds, valid ? xaddr : (uint32_t)kXA, ph, roff, poff, lane4);
            if (!valid) a = short2_t{0, 0};
            if (valid && !ahead) add_bin<FMT>(S, a, sg[0]);
            if (__ballot(ahead) != 0) {
                fold<FMT>(S, par);
                wave_flush(S, d, ch);
#pragma unroll
                for (int q = 0; q < 6; ++q) S.v[q] = 0;
                S.w += 1;
                S.wnext += span;
                if (ahead) add_bin<FMT>(S, a, sg[0]);
            }
#pragma unroll
            for (int u = 0; u + 1 < U; ++u) sg[u] = sg[u + 1];
            sg[U - 1] = *reinterpret_cast<const uint2*>(sgb + soff + 128u * U);
            soff += 128u;
            xaddr += dx;
            ph += dph;
            ++j;
        }
    }
    fold<FMT>(S, par);
}

// Direct per-sample form over tile offsets [lo, hi) for one E/P/L channel
// (samples of chips cut by the ends of the block).
__device__ __forceinline__ void direct_epl(const uint8_t* lds, uint32_t lane4, uint64_t t0,
                                           uint32_t lo, uint32_t hi, const DevMeta& m,
                                           const DevChan& ch, const uint32_t* __restrict__ sgn_prn,
                                           const Dest& d) {
    if (lo >= hi) return;
    const short* sx = reinterpret_cast<const short*>(lds + kXA);
    const uint64_t W = m.window;
    const uint64_t wa = (m.p0 + (t0 + lo) * m.dp) / W;
    const uint64_t wb = (m.p0 + (t0 + hi - 1) * m.dp) / W;
    const int64_t tap[3] = {int64_t(1) << 31, 0, -(int64_t(1) << 31)};
    const int slot[3] = {ch.slot_e, ch.slot_p, ch.slot_l};
    for (uint64_t w = wa; w <= wb; ++w) {
        const uint64_t s_lo = window_start(w, W, m.p0, m.dp);
        const uint64_t s_hi = window_start(w + 1, W, m.p0, m.dp);
        const uint32_t a = (uint32_t)max((uint64_t)lo, s_lo > t0 ? s_lo - t0 : 0);
        const uint32_t b = (uint32_t)min((uint64_t)hi, s_hi - t0);
        int acc[6] = {0, 0, 0, 0, 0, 0};
        for (uint32_t i = a + (threadIdx.x & 63); i < b; i += 64) {
            const uint64_t n = t0 + i;
            const uint32_t phi = m.phi0 + (uint32_t)n * m.dphi;
            int cc, ss;
            lut_cs(lds_u32(lds, __builtin_amdgcn_perm(phi, lane4, kPermSel)), cc, ss);
            const int x = sx[i];
            const uint64_t u = m.p0 + n * m.dp;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int64_t v = (int64_t)u + tap[k];
                int32_t chip = (int32_t)(v >> 32) % kCodeLen;
                if (chip < 0) chip += kCodeLen;
                const int r = (int)(short)(sgn_prn[chip] & 0xFFFF);
                acc[2 * k] += x * cc * r;
                acc[2 * k + 1] -= x * ss * r;
            }
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int t = wave_total_dpp(acc[k]);
            if ((threadIdx.x & 63) == 0 && t != 0) atomicAdd(d.at((uint32_t)w, slot[k >> 1], k & 1), t);
        }
    }
}

// One sample added to (sign = +1) or removed from (-1) bin h's E/P/L
// outputs, by one lane (the seam of a one-sample slip of the bin grid).
__device__ __forceinline__ void seam_sample(const uint8_t* lds, uint32_t lane4, uint64_t t0,
                                            int64_t off, uint64_t h, int sign, const DevMeta& m,
                                            const DevChan& ch, const uint32_t* __restrict__ sgn_prn,
                                            uint32_t span, const Dest& d) {
    const short* sx = reinterpret_cast<const short*>(lds + kXA);
    const uint32_t phi = m.phi0 + (uint32_t)(t0 + (uint64_t)off) * m.dphi;
    int cc, ss;
    lut_cs(lds_u32(lds, __builtin_amdgcn_perm(phi, lane4, kPermSel)), cc, ss);
    const int x = sx[off];
    const uint32_t c = (uint32_t)(h >> 1), par = (uint32_t)(h & 1);
    const uint32_t si = (c + par + kCodeLen - 1) % kCodeLen;
    const int sl = (int)(short)(sgn_prn[si] & 0xFFFF), se = (int)(short)(sgn_prn[si + 1] & 0xFFFF);
    const int sp = par ? sl : se;
    const uint32_t w = c / span;
    const int s3[3] = {se, sp, sl};
    const int slot[3] = {ch.slot_e, ch.slot_p, ch.slot_l};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        atomicAdd(d.at(w, slot[k], 0), sign * x * cc * s3[k]);
        atomicAdd(d.at(w, slot[k], 1), -sign * x * ss * s3[k]);
    }
}

// Two 2-bit codes (bits 0-1 and 2-3 of nib) -> packed int16 samples 2c - 3.
__device__ __forceinline__ uint32_t expand2(uint32_t nib) {
    const short2_t c = as_s2((nib * 0x4001u) & 0x00030003u);
    const short2_t two = {2, 2}, m3 = {-3, -3};
    return __builtin_bit_cast(uint32_t, c * two + m3);
}

// Tile samples [t0, t0 + count) into copies A and B (int16; zero past the
// end of the block); count is at most kXSamples and a multiple of 16.
template <int FMT>
__device__ __forceinline__ void stage_tile(const uint8_t* __restrict__ samples, uint64_t n,
                                           uint64_t t0, uint8_t* lds, int nthreads,
                                           uint32_t count) {
    static_assert(kXSamples % 16 == 0, "staging granule");
    uint4* dA = reinterpret_cast<uint4*>(lds + kXA);
    uint4* dB = reinterpret_cast<uint4*>(lds + kXB);
    if constexpr (FMT == GC_I2_REAL) {
        // one input dword (16 samples) per thread and pass
        const uint8_t* src = samples + t0 / 4;
        const uint32_t avail = (uint32_t)min((n - t0 + 3) / 4, (uint64_t)count / 4);  // bytes
        for (int i = threadIdx.x; i < (int)count / 16; i += nthreads) {
            const uint32_t b = 4u * i;
            uint32_t v = 0, nx = 0;
            if (b + 4 <= avail) {
                v = *reinterpret_cast<const uint32_t*>(src + b);
            } else {
                for (uint32_t q = 0; q < 4; ++q)
                    if (b + q < avail) v |= (uint32_t)src[b + q] << (8 * q);
            }
            if (b + 4 < avail) nx = src[b + 4];
            uint32_t w[9];
#pragma unroll
            for (int k = 0; k < 8; ++k) w[k] = expand2((v >> (4 * k)) & 15u);
            w[8] = expand2(nx & 15u);
            if (b + 4 > avail) {  // samples past the block read as zero
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (b + k / 2 >= avail) w[k] = 0;
            }
            if (b + 4 >= avail) w[8] = 0;
            dA[2 * i] = uint4{w[0], w[1], w[2], w[3]};
            dA[2 * i + 1] = uint4{w[4], w[5], w[6], w[7]};
            uint32_t u[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) u[k] = __builtin_amdgcn_alignbit(w[k + 1], w[k], 16);
            dB[2 * i] = uint4{u[0], u[1], u[2], u[3]};
            dB[2 * i + 1] = uint4{u[4], u[5], u[6], u[7]};
        }
    } else {
        // 16 int8 samples per thread and pass
        const uint8_t* src = samples + t0;
        const uint32_t avail = (uint32_t)min(n - t0, (uint64_t)count);
        for (int i = threadIdx.x; i < (int)count / 16; i += nthreads) {
            const uint32_t b = 16u * i;
            uint32_t v[5] = {0, 0, 0, 0, 0};
            if (b + 16 <= avail) {
                const uint4 q = *reinterpret_cast<const uint4*>(src + b);
                v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
            } else {
                for (uint32_t q = 0; q < 16; ++q)
                    if (b + q < avail) v[q / 4] |= (uint32_t)src[b + q] << (8 * (q % 4));
            }
            if (b + 16 < avail) v[4] = src[b + 16];
            uint32_t w[9];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint32_t d = v[k / 2] >> (16 * (k % 2));
                w[k] = (uint32_t)(uint16_t)(int16_t)(int8_t)(d & 0xFF) |
                       ((uint32_t)(uint16_t)(int16_t)(int8_t)((d >> 8) & 0xFF) << 16);
            }
            w[8] = (uint32_t)(uint16_t)(int16_t)(int8_t)(v[4] & 0xFF);
            dA[2 * i] = uint4{w[0], w[1], w[2], w[3]};
            dA[2 * i + 1] = uint4{w[4], w[5], w[6], w[7]};
            uint32_t u[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) u[k] = __builtin_amdgcn_alignbit(w[k + 1], w[k], 16);
            dB[2 * i] = uint4{u[0], u[1], u[2], u[3]};
            dB[2 * i + 1] = uint4{u[4], u[5], u[6], u[7]};
        }
    }
}

// First sample (tile offset) of bin h with its overshoot: smallest n with
// (t0 + n)*dp >= h*2^31 - p0, given u0 = p0 + t0*dp <= h*2^31.
__device__ __forceinline__ void bin_start(uint64_t h, uint64_t u0, uint32_t dp, float inv_dp,
                                          uint64_t& n_out, uint64_t& e_out) {
    const uint64_t D = (h << 31) - u0;
    const float df = (float)(uint32_t)(D >> 32) * 4294967296.0f + (float)(uint32_t)D;
    uint64_t nr = (uint64_t)(uint32_t)max(0.0f, df * inv_dp - 2.0f);
    while (nr * dp < D) ++nr;
    n_out = nr;
    e_out = nr * dp - D;
}

// Bins [kb, ke) of a run clipped to this wave's share [pb, pe).
template <int FMT, int L>
__device__ __forceinline__ void clipped_run(Slot& S, const uint8_t* lds, uint32_t lane,
                                            uint32_t lane4, int64_t base, uint32_t h_a,
                                            uint32_t kb, uint32_t ke, uint32_t pb, uint32_t pe,
                                            uint64_t t0, const DevMeta& m, const DevChan& ch,
                                            const uint32_t* __restrict__ sgn_prn, uint32_t span,
                                            const Dest& d) {
    periodic_run<FMT, L>(S, lds, lane, lane4, base, h_a, max(kb, pb), min(ke, pe), t0, m, ch,
                         sgn_prn, span, d);
}

// One channel on the staged tile [t0, t1), share [n0, n1) of W: the tile's
// whole-chip bins are cut at multiples of 64 bins near nb*n/W and the wave
// takes the bins between the cuts at n0 and n1; the share starting at 0
// also takes the direct samples at the block ends and the slip seam.
template <int FMT, int L>
__device__ __forceinline__ void channel_tile(Slot& S, const uint8_t* lds, uint32_t lane,
                                             uint32_t lane4, uint64_t t0, uint64_t t1,
                                             const DevMeta& m, const DevChan& ch,
                                             const uint32_t* __restrict__ sgn_prn, const Dest& d,
                                             uint32_t n0, uint32_t n1, uint32_t W) {
    const uint32_t span = (uint32_t)(m.window >> 32);
    const uint32_t tl = (uint32_t)(t1 - t0);
    // samples of chips cut by the ends of the block
    const bool lead = n0 == 0;
    if (lead && m.head_end > t0)
        direct_epl(lds, lane4, t0, 0, (uint32_t)(min((uint64_t)m.head_end, t1) - t0), m, ch,
                   sgn_prn, d);
    if (lead && t1 > m.tail_beg)
        direct_epl(lds, lane4, t0, (uint32_t)(max((uint64_t)m.tail_beg, t0) - t0), tl, m, ch,
                   sgn_prn, d);
    // bins of whole chips whose code phase starts in [u(t0), u(t1))
    const uint64_t u0 = m.p0 + t0 * m.dp;
    const uint64_t u1 = m.p0 + t1 * m.dp;
    uint64_t ha = (u0 + 0x7FFFFFFFull) >> 31;
    uint64_t hb = (u1 + 0x7FFFFFFFull) >> 31;
    if (ha < 2 * m.c_full0) ha = 2 * m.c_full0;
    if (hb > 2 * m.c_full1) hb = 2 * m.c_full1;
    if (hb <= ha) return;
    const uint32_t nb = (uint32_t)(hb - ha);
    // this wave's share of the bins (nb < 2^15, so 32-bit products)
    const uint32_t pb = n0 == 0 ? 0u : min(nb, ((nb * n0) / W + 63u) & ~63u);
    const uint32_t pe = n1 == W ? nb : min(nb, ((nb * n1) / W + 63u) & ~63u);
    // the open dump becomes the one of the share's first bin (the shares of
    // the other waves lie in between): flush what is open if that is later
    if (pb < pe) {
        const uint32_t c_first = (uint32_t)((ha + pb) >> 1);
        if (!S.init || c_first >= S.wnext) {
            const uint32_t w_first = c_first / span;
            if (S.init) {
                wave_flush(S, d, ch);
#pragma unroll
                for (int q = 0; q < 6; ++q) S.v[q] = 0;
            }
            S.init = true;
            S.w = w_first;
            S.wnext = (w_first + 1) * span;
        }
    }
    const uint32_t dp = (uint32_t)m.dp;
    uint64_t na, ea;
    bin_start(ha, u0, dp, 1.0f / (float)dp, na, ea);
    // bin k starts at na + k*L while e_k = ea + k*D stays in [0, dp); bins
    // 0 .. nb-1 all hold L samples when that holds up to k = nb (the start of
    // the first bin of the next tile)
    const int64_t D = (int64_t)L * (int64_t)dp - (int64_t(1) << 31);
    const int64_t elast = (int64_t)ea + (int64_t)nb * D;
    if (elast >= 0 && elast < (int64_t)dp) {
        clipped_run<FMT, L>(S, lds, lane, lane4, (int64_t)na, (uint32_t)ha, 0, nb, pb, pe, t0, m,
                            ch, sgn_prn, span, d);
        return;
    }
    // one slip: first k (1 <= ks <= nb) whose bin starts one sample earlier
    // (D > 0) or later (D < 0) than the grid of bin 0
    uint32_t ks;
    int sigma;
    if (D > 0) {
        ks = (uint32_t)(((int64_t)dp - (int64_t)ea + D - 1) / D);
        sigma = -1;
    } else {
        ks = (uint32_t)((int64_t)ea / (-D) + 1);
        sigma = 1;
    }
    clipped_run<FMT, L>(S, lds, lane, lane4, (int64_t)na, (uint32_t)ha, 0, ks, pb, pe, t0, m, ch,
                        sgn_prn, span, d);
    clipped_run<FMT, L>(S, lds, lane, lane4, (int64_t)na + sigma, (uint32_t)ha, ks, nb, pb, pe, t0,
                        m, ch, sgn_prn, span, d);
    // bin ks-1 really ends at na + ks*L + sigma: the sample between the two
    // grids was counted twice (sigma = -1) or not at all (sigma = +1)
    if (lead && lane == 0) {
        const int64_t off = (int64_t)na + (int64_t)ks * L + (sigma < 0 ? -1 : 0);
        seam_sample(lds, lane4, t0, off, ha + ks - 1, sigma < 0 ? -1 : 1, m, ch, sgn_prn, span, d);
    }
}

// Tiles [tb0, tb1) of tile_len samples (at most kTile, a multiple of 16) of
// one sample block for the block's channel list
// s_list[0 .. nlist), nlist <= blockDim.x / 64.  The channels' bins are
// shared evenly among W waves (W below): wave w takes positions [w*nlist,
// (w+1)*nlist) of nlist*W, channel c holding [c*W, (c+1)*W), so each wave
// has one channel piece (when nlist divides W) or at most two.  A wave with
// one piece keeps its channel's sums in registers across the tiles and
// flushes the dump still open at the end; a wave with two flushes each
// piece after every tile.
template <int FMT>
__device__ __forceinline__ void pbin_chunk(uint8_t* s_lds, const int* s_list, int nlist,
                                           const uint8_t* __restrict__ samples, uint64_t n,
                                           uint32_t tb0, uint32_t tb1, uint32_t tile_len,
                                           const DevChan* __restrict__ chans,
                                           const DevMeta* __restrict__ metas,
                                           gc_chan_state* __restrict__ state,
                                           int32_t* __restrict__ out, int tap_stride,
                                           uint32_t max_dumps,
                                           const uint32_t* __restrict__ tables) {
    const int tid = threadIdx.x;
    const int nthreads = blockDim.x;
    // waves used: all of the block's, unless the channels already fill three
    // quarters of them; then one wave per channel (sharing a channel between
    // waves costs a cut of its bins and a flush per tile, more than the
    // remaining idle waves would gain)
    const uint32_t Wb = __builtin_amdgcn_readfirstlane((uint32_t)nthreads / 64);
    const uint32_t W = 4u * (uint32_t)nlist >= 3u * Wb ? (uint32_t)nlist : Wb;
    const uint32_t wave = __builtin_amdgcn_readfirstlane((uint32_t)tid / 64);
    const bool busy = wave < W;
    const uint32_t lane = tid & 63;
    const uint32_t lane4 = lane * 4;
    Slot S;
    auto reset = [&]() {
#pragma unroll
        for (int q = 0; q < 6; ++q) S.v[q] = 0;
        S.e16 = S.l16 = short2_t{0, 0};
        S.r[0] = S.r[1] = S.r[2] = S.r[3] = 0;
        S.w = 0;
        S.wnext = 0;
        S.init = false;
    };
    reset();
    // this wave's pieces: positions [x0, x1) of nlist * W
    const uint32_t x0 = (busy ? wave : 0u) * (uint32_t)nlist, x1 = x0 + (uint32_t)nlist;
    const uint32_t cA = x0 / W, cB = (x1 - 1) / W;
    const bool two = cB != cA;
    const uint32_t aN0 = x0 - cA * W, aN1 = two ? W : x1 - cA * W;
    const uint32_t bN1 = x1 - cB * W;
    auto piece = [&](uint32_t slot, uint32_t p0, uint32_t p1, uint64_t t0, uint64_t t1) {
        const int chn = __builtin_amdgcn_readfirstlane(s_list[slot]);
        const DevChan& ch = chans[chn];
        const uint32_t* sgn_prn = tables + kTabSign + (ch.prn - 1) * kSignLen;
        const DevMeta m = metas[chn];
        const Dest d{out, state + chn, (uint64_t)chn * max_dumps, tap_stride, m.m_close};
        switch (m.bin_len) {
            case 2: channel_tile<FMT, 2>(S, s_lds, lane, lane4, t0, t1, m, ch, sgn_prn, d, p0, p1, W); break;
            case 4: channel_tile<FMT, 4>(S, s_lds, lane, lane4, t0, t1, m, ch, sgn_prn, d, p0, p1, W); break;
            case 8: channel_tile<FMT, 8>(S, s_lds, lane, lane4, t0, t1, m, ch, sgn_prn, d, p0, p1, W); break;
            default: channel_tile<FMT, 10>(S, s_lds, lane, lane4, t0, t1, m, ch, sgn_prn, d, p0, p1, W); break;
        }
    };
    auto flush = [&](uint32_t slot) {
        if (S.init) {
            const int chn = __builtin_amdgcn_readfirstlane(s_list[slot]);
            const Dest d{out, state + chn, (uint64_t)chn * max_dumps, tap_stride,
                         metas[chn].m_close};
            wave_flush(S, d, chans[chn]);
        }
        reset();
    };
    for (uint32_t tile = tb0; tile < tb1; ++tile) {
        const uint64_t t0 = (uint64_t)tile * tile_len;
        const uint64_t t1 = min(n, t0 + tile_len);
        __syncthreads();
        stage_tile<FMT>(samples, n, t0, s_lds, nthreads, tile_len + kMarginS);
        __syncthreads();
        for (uint32_t j = 0; j < (busy ? (two ? 2u : 1u) : 0u); ++j) {
            const uint32_t slot = j ? cB : cA;
            piece(slot, j ? 0u : aN0, j ? bN1 : aN1, t0, t1);
            if (two) flush(slot);
        }
    }
    // the dump still open at the end of the chunk
    if (busy && !two) flush(cA);
}

// Periodic channels first .. of [c_begin, c_end) into s_list (at most
// `cap`), their number into s_list[kMaxWaves]; by thread 0.
__device__ __forceinline__ void list_periodic(int* s_list, const DevMeta* __restrict__ metas,
                                              int c_begin, int c_end, int first, int cap) {
    if (threadIdx.x == 0) {
        int k = 0, seen = 0;
        for (int c = c_begin; c < c_end && k < cap; ++c) {
            const DevMeta& m = metas[c];
            if (m.status == GC_OK && m.path == kPathPeriodic) {
                if (seen >= first) s_list[k++] = c;
                ++seen;
            }
        }
        s_list[kMaxWaves] = k;
    }
}

// FIXED: tiles of kTile samples (tile_len unused), the common case, where a
// compile-time tile length keeps the walk's scalar state out of spill slots
template <int FMT, bool FIXED>
__global__ __launch_bounds__(kMaxWaves * 64) void k_pbin(const uint8_t* __restrict__ samples,
                                                         uint64_t n,
                                                         const DevChan* __restrict__ chans,
                                                         const DevMeta* __restrict__ metas,
                                                         gc_chan_state* __restrict__ state,
                                                         int32_t* __restrict__ out, int tap_stride,
                                                         uint32_t max_dumps,
                                                         const uint32_t* __restrict__ tables,
                                                         int n_chan, uint32_t n_tiles,
                                                         uint32_t tile_len, int per_block) {
    // one LDS block: the per-lane carrier tables at offset 0 (the v_perm
    // result is the address itself), the two staged copies, the channel list
    __shared__ __attribute__((aligned(16))) uint8_t s_lds[kLdsBytes + 4 * (kMaxWaves + 1)];
    uint32_t* s_lut = reinterpret_cast<uint32_t*>(s_lds);
    int* s_list = reinterpret_cast<int*>(s_lds + kLdsBytes);
    // this block's channel group: periodic channels of ranks
    // per_block*blockIdx.y ..; with fewer channels than kMaxWaves, several
    // waves share a channel (R per channel, nlist*R <= blockDim.x/64)
    list_periodic(s_list, metas, 0, n_chan, (int)blockIdx.y * per_block, per_block);
    __syncthreads();
    const int nlist = s_list[kMaxWaves];
    if (nlist == 0) return;
    for (int i = threadIdx.x; i < kLutWords; i += blockDim.x) s_lut[i] = tables[kTabLut + (i >> 6)];
    // contiguous chunk of tiles for this block
    const uint32_t tb0 = (uint32_t)(((uint64_t)blockIdx.x * n_tiles) / gridDim.x);
    const uint32_t tb1 = (uint32_t)(((uint64_t)(blockIdx.x + 1) * n_tiles) / gridDim.x);
    pbin_chunk<FMT>(s_lds, s_list, nlist, samples, n, tb0, tb1, FIXED ? (uint32_t)kTile : tile_len,
                    chans, metas, state, out, tap_stride, max_dumps, tables);
}

// Many receivers in one persistent launch: item i is a chunk of tiles of
// one receiver for a group of at most kMaxWaves of its channels; the block
// lists the group's periodic channels and shares their bins evenly among
// its kMaxWaves waves.  Blocks take items from a queue (an atomic counter,
// zero when the kernel starts), so that items of unequal cost (channel
// count, samples per chip) even out across the compute units.

__global__ __launch_bounds__(kMaxWaves * 64) void k_pbin_batch(
    const DevRx* __restrict__ rx, const PbinItem* __restrict__ items, uint32_t n_items,
    uint32_t* __restrict__ counter, const DevChan* __restrict__ chans,
    const DevMeta* __restrict__ metas, gc_chan_state* __restrict__ state,
    int32_t* __restrict__ out, int tap_stride, uint32_t max_dumps,
    const uint32_t* __restrict__ tables) {
    __shared__ __attribute__((aligned(16))) uint8_t s_lds[kLdsBytes + 4 * (kMaxWaves + 2)];
    uint32_t* s_lut = reinterpret_cast<uint32_t*>(s_lds);
    int* s_list = reinterpret_cast<int*>(s_lds + kLdsBytes);
    uint32_t* s_item = reinterpret_cast<uint32_t*>(s_lds + kLdsBytes) + kMaxWaves + 1;
    for (int i = threadIdx.x; i < kLutWords; i += blockDim.x) s_lut[i] = tables[kTabLut + (i >> 6)];
    for (;;) {
        __syncthreads();   // the previous item is done with s_list, s_item and the tile
        if (threadIdx.x == 0) *s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t it = *s_item;
        if (it >= n_items) break;   // every block ends on its first ticket past the end
        const PbinItem I = items[it];
        list_periodic(s_list, metas, I.chan_begin, I.chan_begin + I.n_chan, 0, kMaxWaves);
        __syncthreads();
        const int nlist = s_list[kMaxWaves];
        if (nlist == 0) continue;
        const DevRx& X = rx[I.rx];
        if (X.fmt == GC_I2_REAL)
            pbin_chunk<GC_I2_REAL>(s_lds, s_list, nlist, X.samples, X.n, I.tile_begin,
                                   I.tile_end, kTile, chans, metas, state, out, tap_stride, max_dumps,
                                   tables);
        else
            pbin_chunk<GC_I8_REAL>(s_lds, s_list, nlist, X.samples, X.n, I.tile_begin,
                                   I.tile_end, kTile, chans, metas, state, out, tap_stride, max_dumps,
                                   tables);
    }
}

template <int FMT>
void launch_one(const uint8_t* samples, uint64_t n, const DevChan* chans, const DevMeta* meta,
                gc_chan_state* state, int n_chan, int32_t* out, int tap_stride, uint32_t max_dumps,
                const uint32_t* tables, int grid, hipStream_t s) {
    // Balanced tiles: every block takes k = ceil(n / (kTile grid)) tiles, of
    // n / (k grid) samples rounded up to 512 (whole 64-lane steps of the 2-,
    // 4- and 8-sample bins, as kTile is), so that the last round does not
    // leave blocks idle; taken only when that shortens the largest block's
    // share by more than 1/16 (below that it measured no faster).
    constexpr uint64_t kMinTile = 2048;
    const uint64_t G = (uint64_t)max(grid, 1);
    const uint64_t per = (n + (uint64_t)kTile * G - 1) / ((uint64_t)kTile * G);
    const uint64_t cand = max(kMinTile, ((n + per * G - 1) / (per * G) + 511) & ~511ull);
    const uint64_t tl = 16 * cand < 15 * (uint64_t)kTile ? cand : (uint64_t)kTile;
    const uint32_t tile_len = (uint32_t)tl;
    const uint32_t n_tiles = (uint32_t)((n + tl - 1) / tl);
    const int g = (int)min((uint32_t)grid, n_tiles);
    // up to kMaxWaves channels per block, one wave each; a plan with fewer
    // channels lets R = kMaxWaves / n_chan waves share each channel (more
    // waves for a small plan; with many channels sharing costs more than
    // it gains)
    const int per_block = min(n_chan, kMaxWaves);
    const int R = kMaxWaves / per_block;
    const int groups = (n_chan + per_block - 1) / per_block;
    if (tile_len == (uint32_t)kTile)
        hipLaunchKernelGGL((k_pbin<FMT, true>), dim3(g, groups), dim3(64 * per_block * R), 0, s,
                           samples, n, chans, meta, state, out, tap_stride, max_dumps, tables,
                           n_chan, n_tiles, tile_len, per_block);
    else
        hipLaunchKernelGGL((k_pbin<FMT, false>), dim3(g, groups), dim3(64 * per_block * R), 0, s,
                           samples, n, chans, meta, state, out, tap_stride, max_dumps, tables,
                           n_chan, n_tiles, tile_len, per_block);
}

}  // namespace

int pbin_tile_samples() { return kTile; }

hipError_t launch_pbin_batch(int grid, const DevRx* rx, const PbinItem* items, uint32_t n_items,
                             uint32_t* counter, const DevChan* chans, const DevMeta* meta,
                             gc_chan_state* state, int32_t* out, int tap_stride,
                             uint32_t max_dumps, const uint32_t* tables, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    const int g = (int)min((uint32_t)grid, n_items);
    hipLaunchKernelGGL(k_pbin_batch, dim3(g), dim3(64 * kMaxWaves), 0, s, rx, items, n_items,
                       counter, chans, meta, state, out, tap_stride, max_dumps, tables);
    return hipGetLastError();
}

hipError_t launch_pbin(const uint8_t* samples, uint64_t n, int fmt, const DevChan* chans,
                       const DevMeta* meta, gc_chan_state* state, int n_chan, int32_t* out,
                       int tap_stride, uint32_t max_dumps, const uint32_t* tables, int grid,
                       hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (fmt == GC_I2_REAL)
        launch_one<GC_I2_REAL>(samples, n, chans, meta, state, n_chan, out, tap_stride, max_dumps,
                               tables, grid, s);
    else if (fmt == GC_I8_REAL)
        launch_one<GC_I8_REAL>(samples, n, chans, meta, state, n_chan, out, tap_stride, max_dumps,
                               tables, grid, s);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace gc
