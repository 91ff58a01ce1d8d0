// gc_epl.hip -- binned early/prompt/late correlator for real int8, 2-bit and
// complex int8 (I then Q) sample streams (integer carrier path).
//
// The replicas of E, P and L (offsets +1/2, 0, -1/2 chip) are constant over
// each half chip of code phase, so the kernel first sums the wiped-off
// samples of every half chip (a "bin"), then applies the three taps' code
// signs once per bin:
//   bin 0 of chip c (phase in [c, c+1/2)):   E, P use C[c],   L uses C[c-1]
//   bin 1 of chip c (phase in [c+1/2, c+1)): E uses C[c+1],   P, L use C[c]
// This is the same sum as the per-sample definition, regrouped; all
// arithmetic is integer, so the result is identical bit for bit.
//
// Work layout (one persistent block per CU):
//   * a tile of kTile samples is staged once in LDS as int16 (2-bit codes
//     expanded) and read by every channel of the plan; a packed multiply
//     picks either sample of a dword through its operand select, so samples
//     need no unpacking.  Complex samples are staged as (xI, xQ) int16 pairs,
//     one dword each, in two half tiles; per sample two packed multiply-adds
//     form the planes (xI, xQ)*c and (xQ, xI)*s, and the bin's wiped-off
//     sum is (xI c + xQ s, xQ c - xI s) from their halves;
//   * the block's lanes (1024 in a plan, 256 or 512 in the batch shapes)
//     form G groups of whole waves (G a power of two, at most the number of
//     channels with work, at least 128 lanes a group), and the groups take
//     different channels at once; within a group the chips whose first
//     sample lies in the tile are split into one run of consecutive whole
//     chips per lane (tile / group lanes samples, e.g. 46 * G in a plan;
//     neighbouring runs start an odd number of LDS dwords apart, so lanes
//     hit different banks).  Longer runs amortise the per-run set-up
//     (Bresenham start, code signs, flush) over more samples;
//   * a lane walks its run sample by sample: the carrier phase advances by
//     one add, the sin/cos entry comes from a per-lane copy of the table in
//     LDS (address = one v_perm, no bank conflicts), and one packed int16
//     multiply-add folds x*(c, s) into the bin sum; bin lengths come from an
//     exact integer Bresenham step on the code phase (q or q+1 samples);
//   * lanes keep E/P/L sums in registers, flush them with atomics at a dump
//     boundary inside their run (rare), and at the end of the run the wave
//     sums lanes of the same dump with DPP and adds once per dump.
// Chips cut by the ends of the block, and channels whose steps do not fit
// the binned form, go through a direct per-sample path on the same tile.
#include "gc_device.h"

namespace gc {

namespace {

constexpr int kMargin = kEplMarginSamples;    // chips that start in a tile end within this
constexpr int kLutWords = 256 * 64;           // entry l of lane L at word l*64 + L
constexpr uint32_t kPermSel = 0x0C0C0700u;    // byte1 = phase[31:24], byte0 = lane*4

// Complex samples in LDS: one dword each, either plain (sample i at dword
// i) or blocked: blocks of kIqBlk samples, each followed by copies of the
// next block's first kIqPad samples, so sample i sits at dword iq_at(i)
// and the samples of a bin of up to kIqPad + 1 are consecutive dwords from
// iq_at of its first.  The lanes of a wave walk runs a whole number of
// chips apart; at a whole number of samples per chip that is a multiple of
// 8 (8.184, 16.368 MHz) their starts fall on 8 or fewer of the banks, and
// the odd shift of kIqPad per block spreads them.  Elsewhere the plain
// layout spreads them already and saves the per-bin address arithmetic.
constexpr uint32_t kIqBlk = 256;
constexpr uint32_t kIqPad = 5;
__device__ __forceinline__ uint32_t iq_at(uint32_t i) { return i + kIqPad * (i >> 8); }
template <bool PAD>
__device__ __forceinline__ uint32_t iq_idx(uint32_t i) { return PAD ? iq_at(i) : i; }
static_assert(kIqBlk == 256, "iq_at shifts by 8");
constexpr int iq_words(int samples) {
    return (samples + (int)kIqBlk - 1) / (int)kIqBlk * (int)(kIqBlk + kIqPad);
}

// Block shape: THREADS lanes, each walking a run of about RUN samples per
// channel (RUN/2 LDS dwords, odd, so that lanes start in different banks).
template <int THREADS, int RUN>
struct Shape {
    static constexpr int kThreads = THREADS;
    static constexpr int kRun = RUN;
    static constexpr int kTile = THREADS * RUN;                 // samples per tile
    static constexpr int kXSamples = kTile + kMargin;           // staged as int16
    // complex input: half tiles of kTile / 2 samples (+ margin), one dword
    // each, plain or blocked (iq_at; sized for the blocked one)
    static constexpr int kHalf = kTile / 2;
    static constexpr int kXSamplesIQ = kHalf + kMargin;
    static constexpr int kXBytes = kXSamples * 2 > iq_words(kXSamplesIQ) * 4
                                       ? kXSamples * 2
                                       : iq_words(kXSamplesIQ) * 4;
    static constexpr int kLdsBytes = kLutWords * 4 + kXBytes;   // table at LDS offset 0
    static_assert((RUN / 2) % 2 == 1, "odd dword stride between lanes");
    static_assert(kTile % 8 == 0, "half tiles start on a multiple of 4 samples");
    static_assert(kLdsBytes <= 160 * 1024, "LDS per block");
};
using ShapePlan = Shape<1024, 46>;            // single-receiver plans: 47104-sample tiles

typedef short short2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ short2_t as_s2(uint32_t v) { return __builtin_bit_cast(short2_t, v); }
__device__ __forceinline__ uint32_t as_u32(short2_t v) { return __builtin_bit_cast(uint32_t, v); }

// One sample: x * (c, s) accumulated into the packed bin sum (I = x*c, Q = x*s;
// the Q sign of the wipe-off is applied when the bin is folded).
__device__ __forceinline__ short2_t mac_sample(short2_t a, short x, uint32_t phi, uint32_t lane4,
                                               const uint8_t* lut_bytes) {
    const uint32_t off = __builtin_amdgcn_perm(phi, lane4, kPermSel);
    const short2_t cs = as_s2(*reinterpret_cast<const uint32_t*>(lut_bytes + off));
    const short2_t xx = {x, x};
    return xx * cs + a;
}

// Sum over one bin of len samples starting at phase phi, len in {Q, Q+1}
// (Q > 0: straight-line code, the last sample weighted by 0 or 1 so that no
// branch splits the chip body), or any len (Q == 0).  The bin's phase advance
// is len*dphi, applied by the caller.
template <int Q>
__device__ __forceinline__ short2_t bin_sum(const short* __restrict__ xs, uint32_t phi,
                                            uint32_t dphi, uint32_t lane4, const uint8_t* lut,
                                            uint32_t len) {
    short2_t a = {0, 0};
    if constexpr (Q > 0) {
#pragma unroll
        for (int j = 0; j < Q; ++j) a = mac_sample(a, xs[j], phi + j * dphi, lane4, lut);
        const short x2 = len > (uint32_t)Q ? xs[Q] : (short)0;
        a = mac_sample(a, x2, phi + Q * dphi, lane4, lut);
    } else {
        for (uint32_t j = 0; j < len; ++j) a = mac_sample(a, xs[j], phi + j * dphi, lane4, lut);
    }
    return a;
}

// Complex sample (xI, xQ) at phase phi: a += (xI, xQ)*c, b += (xQ, xI)*s
// (operand selects swap and broadcast the halves).
__device__ __forceinline__ void mac_iq(short2_t& a, short2_t& b, uint32_t xw, uint32_t phi,
                                       uint32_t lane4, const uint8_t* lut_bytes) {
    const uint32_t off = __builtin_amdgcn_perm(phi, lane4, kPermSel);
    const short2_t cs = as_s2(*reinterpret_cast<const uint32_t*>(lut_bytes + off));
    const short2_t x = as_s2(xw);
    const short2_t xs = __builtin_shufflevector(x, x, 1, 0);
    a = x * __builtin_shufflevector(cs, cs, 0, 0) + a;
    b = xs * __builtin_shufflevector(cs, cs, 1, 1) + b;
}

// Complex bin of len samples from tile sample nb (as bin_sum): the planes
// a = sum (xI, xQ)*c and b = sum (xQ, xI)*s, each within int16
// (len * 128 * 24 <= 32767).  In the blocked layout bins of at most
// kIqPad + 1 samples read consecutive dwords and longer ones map each
// sample.
template <int Q, bool PAD>
__device__ __forceinline__ void bin_sum_iq(const uint32_t* __restrict__ sx, uint32_t nb,
                                           uint32_t phi, uint32_t dphi, uint32_t lane4,
                                           const uint8_t* lut, uint32_t len, short2_t& a,
                                           short2_t& b) {
    a = short2_t{0, 0};
    b = short2_t{0, 0};
    if constexpr (Q > 0 && (!PAD || Q <= (int)kIqPad)) {
        const uint32_t* xs = sx + iq_idx<PAD>(nb);
#pragma unroll
        for (int j = 0; j < Q; ++j) mac_iq(a, b, xs[j], phi + j * dphi, lane4, lut);
        const uint32_t x2 = len > (uint32_t)Q ? xs[Q] : 0u;
        mac_iq(a, b, x2, phi + Q * dphi, lane4, lut);
    } else if constexpr (Q > 0) {
#pragma unroll
        for (int j = 0; j < Q; ++j) mac_iq(a, b, sx[iq_at(nb + j)], phi + j * dphi, lane4, lut);
        const uint32_t x2 = len > (uint32_t)Q ? sx[iq_at(nb + Q)] : 0u;
        mac_iq(a, b, x2, phi + Q * dphi, lane4, lut);
    } else {
        for (uint32_t j = 0; j < len; ++j)
            mac_iq(a, b, sx[iq_idx<PAD>(nb + j)], phi + j * dphi, lane4, lut);
    }
}

struct Dest {
    int32_t* out;
    gc_chan_state* st;
    uint64_t row0;        // ch * max_dumps
    int tap_stride;
    uint32_t m_close;
    __device__ __forceinline__ int32_t* at(uint32_t w, int slot, int comp) const {
        if (w < m_close) return out + ((row0 + w) * tap_stride + slot) * 2 + comp;
        return &st->acc[slot][comp];
    }
};

// E/P/L sums of one lane (I, Q for each).  For 2-bit input they live as
// packed int16 (|sum| <= run length * 72 < 2^15); for int8 as int32.
template <int FMT>
struct EplAcc;

template <>
struct EplAcc<GC_I2_REAL> {
    short2_t e, p, l;
    __device__ __forceinline__ void zero() { e = p = l = short2_t{0, 0}; }
    __device__ __forceinline__ void fold0(short2_t a, uint32_t mp, uint32_t mc, uint32_t) {
        e = a * as_s2(mc) + e;
        p = a * as_s2(mc) + p;
        l = a * as_s2(mp) + l;
    }
    __device__ __forceinline__ void fold1(short2_t a, uint32_t, uint32_t mc, uint32_t mn) {
        e = a * as_s2(mn) + e;
        p = a * as_s2(mc) + p;
        l = a * as_s2(mc) + l;
    }
    __device__ __forceinline__ void get(int v[6]) const {
        v[0] = e.x; v[1] = e.y; v[2] = p.x; v[3] = p.y; v[4] = l.x; v[5] = l.y;
    }
};

// int32 sums folded a chip at a time: the chip's two bins paired per
// component, (b0, b1), against the sign pairs of the taps, E (s_c, s_c+1),
// P (s_c, s_c) and L (s_c-1, s_c), by a two-term int16 dot product into
// int32 each.
__device__ __forceinline__ uint32_t lo_pair(uint32_t x0, uint32_t x1) {
    return __builtin_amdgcn_perm(x1, x0, 0x05040100u);   // (x0.lo, x1.lo)
}
__device__ __forceinline__ uint32_t hi_pair(uint32_t x0, uint32_t x1) {
    return __builtin_amdgcn_perm(x1, x0, 0x07060302u);   // (x0.hi, x1.hi)
}
__device__ __forceinline__ int dot2(uint32_t x, uint32_t s, int acc) {
    return __builtin_amdgcn_sdot2(as_s2(x), as_s2(s), acc, false);
}

struct EplAcc32 {
    int ei, eq, pi, pq, li, lq;
    __device__ __forceinline__ void zero() { ei = eq = pi = pq = li = lq = 0; }
    // I of the two bins in xi, the kept (negated) Q in xq
    __device__ __forceinline__ void fold_chip(uint32_t xi, uint32_t xq, uint32_t se, uint32_t sc,
                                              uint32_t sl) {
        ei = dot2(xi, se, ei); eq = dot2(xq, se, eq);
        pi = dot2(xi, sc, pi); pq = dot2(xq, sc, pq);
        li = dot2(xi, sl, li); lq = dot2(xq, sl, lq);
    }
    __device__ __forceinline__ void get(int v[6]) const {
        v[0] = ei; v[1] = eq; v[2] = pi; v[3] = pq; v[4] = li; v[5] = lq;
    }
};

// int8 real input: a bin is (sum x c, sum x s).
template <>
struct EplAcc<GC_I8_REAL> : EplAcc32 {};

// Complex input: a bin's wiped-off sums are wi = aI + bI and nq = bQ - aQ
// (Q kept negated like the real forms' +x*s), formed as the packed
// a * (1, -1) + b while they fit int16 (bins of at most Q + 1 samples, each
// |xI c + xQ s| <= max|x| * 34), else dotted plane by plane.
template <>
struct EplAcc<GC_I8_IQ> : EplAcc32 {};
template <>
struct EplAcc<GC_I2_IQ> : EplAcc32 {};

template <int FMT, int Q>
__device__ __forceinline__ constexpr bool iq_packed_w() {
    return Q > 0 && (uint64_t)(Q + 1) * (FMT == GC_I2_IQ ? 3u : 128u) * kLutAbsSumMax <= 32767u;
}

// Lane-private atomics of one run's sums (dump boundary inside a run).
template <int FMT>
__device__ __forceinline__ void flush_lane(const EplAcc<FMT>& acc, const Dest& d, uint32_t w,
                                           const DevChan& c) {
    int v[6];
    acc.get(v);
    const int slot[3] = {c.slot_e, c.slot_p, c.slot_l};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        atomicAdd(d.at(w, slot[k], 0), v[2 * k]);
        atomicAdd(d.at(w, slot[k], 1), -v[2 * k + 1]);  // wipe-off Q = -x*s
    }
}

// Binned run of one lane over chips [c, c + K) whose samples start at tile
// offset nb with code-phase overshoot e past the chip start.
template <int FMT, int Q, bool PAD>
__device__ __forceinline__ void epl_run(const void* __restrict__ sx, const uint8_t* lut,
                                     uint32_t lane4, uint32_t nb, uint32_t phi, uint32_t dphi,
                                     uint32_t e, uint32_t dp, uint32_t q, uint32_t r, uint32_t c,
                                     uint32_t K, uint32_t Kmax, uint32_t span,
                                     const uint32_t* __restrict__ sgn, const Dest d,
                                     const DevChan& ch) {
    EplAcc<FMT> acc;
    acc.zero();
    // window of chip c: floor(c / span), float estimate corrected exactly
    uint32_t w = (uint32_t)max(0.0f, (float)c * (1.0f / (float)span) - 1.0f);
    while ((w + 1) * span <= c) ++w;
    uint32_t wnext = (w + 1) * span;
    uint32_t mp = sgn[0], mc = sgn[1], mn = sgn[2];
    uint32_t sl = lo_pair(mp, mc);   // (s_c-1, s_c) of the chip
    const bool active = K > 0;
    for (uint32_t k = 0; k < Kmax; ++k) {
        if (k < K) {
            if (c == wnext) {  // a dump closes before this chip
                flush_lane<FMT>(acc, d, w, ch);
                acc.zero();
                w += 1;
                wnext += span;
            }
            const uint32_t mnn = sgn[k + 3];
            // bin 0: phase [c, c + 1/2)
            bool lt = e < r;
            uint32_t len = q + (lt ? 1u : 0u);
            e = lt ? e + dp - r : e - r;
            short2_t a0, b0, a1, b1;
            if constexpr (fmt_complex(FMT)) {
                bin_sum_iq<Q, PAD>(static_cast<const uint32_t*>(sx), nb, phi, dphi, lane4, lut, len,
                              a0, b0);
            } else {
                a0 = bin_sum<Q>(static_cast<const short*>(sx) + nb, phi, dphi, lane4, lut, len);
                if constexpr (FMT == GC_I2_REAL) acc.fold0(a0, mp, mc, mn);
            }
            nb += len;
            phi += len * dphi;
            // bin 1: phase [c + 1/2, c + 1)
            lt = e < r;
            len = q + (lt ? 1u : 0u);
            e = lt ? e + dp - r : e - r;
            if constexpr (fmt_complex(FMT)) {
                bin_sum_iq<Q, PAD>(static_cast<const uint32_t*>(sx), nb, phi, dphi, lane4, lut, len,
                              a1, b1);
            } else {
                a1 = bin_sum<Q>(static_cast<const short*>(sx) + nb, phi, dphi, lane4, lut, len);
                if constexpr (FMT == GC_I2_REAL) acc.fold1(a1, mp, mc, mn);
            }
            nb += len;
            phi += len * dphi;
            if constexpr (FMT != GC_I2_REAL) {
                const uint32_t se = lo_pair(mc, mn);   // (s_c, s_c+1)
                if constexpr (FMT == GC_I8_REAL) {
                    const uint32_t x0 = as_u32(a0), x1 = as_u32(a1);
                    acc.fold_chip(lo_pair(x0, x1), hi_pair(x0, x1), se, mc, sl);
                } else if constexpr (iq_packed_w<FMT, Q>()) {
                    const short2_t m1 = {1, -1};
                    const uint32_t w0 = as_u32(a0 * m1 + b0), w1 = as_u32(a1 * m1 + b1);
                    acc.fold_chip(lo_pair(w0, w1), hi_pair(w0, w1), se, mc, sl);
                } else {
                    // wi = aI + bI, nq = bQ - aQ: the b planes with the signs,
                    // the a planes with the signs for I and negated for Q
                    const uint32_t xa0 = as_u32(a0), xa1 = as_u32(a1);
                    const uint32_t xb0 = as_u32(b0), xb1 = as_u32(b1);
                    acc.fold_chip(lo_pair(xb0, xb1), hi_pair(xb0, xb1), se, mc, sl);
                    const uint32_t ai = lo_pair(xa0, xa1), aq = hi_pair(xa0, xa1);
                    const uint32_t naq = as_u32(short2_t{0, 0} - as_s2(aq));
                    acc.fold_chip(ai, naq, se, mc, sl);
                }
                sl = se;
            }
            mp = mc;
            mc = mn;
            mn = mnn;
            c += 1;
        }
    }
    // dump of the lane's last chip; lanes of one wave hold consecutive chips,
    // so equal dumps are contiguous: sum each group once
    int v[6];
    acc.get(v);
    const int slot[3] = {ch.slot_e, ch.slot_p, ch.slot_l};
    uint64_t pending = __ballot(active);
    while (pending) {
        const int first = __ffsll((unsigned long long)pending) - 1;
        const uint32_t wsel = __builtin_amdgcn_readlane(w, first);
        const bool mine = active && w == wsel;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int t = wave_total_dpp(mine ? v[k] : 0);
            if ((int)(threadIdx.x & 63) == first)
                atomicAdd(d.at(wsel, slot[k >> 1], k & 1), (k & 1) ? -t : t);
        }
        pending &= ~__ballot(mine);
    }
}

// Direct per-sample form over tile offsets [lo, hi) for up to 4 taps (chips
// cut by the block ends, and channels the binned form does not cover), by
// the nthr threads of a group (gtid = 0 .. nthr - 1, whole waves).
template <int FMT, bool PAD>
__device__ __forceinline__ void direct_range(const void* __restrict__ sx, const uint8_t* lut,
                                             uint32_t gtid, uint32_t nthr,
                                             uint32_t lane4, uint64_t t0, uint32_t lo, uint32_t hi,
                                             const DevMeta& m, const DevChan& ch,
                                             const uint32_t* __restrict__ sgn_prn, const Dest d) {
    if (lo >= hi) return;
    const uint64_t W = m.window;
    const uint64_t wa = (m.p0 + (t0 + lo) * m.dp) / W;
    const uint64_t wb = (m.p0 + (t0 + hi - 1) * m.dp) / W;
    const int nk = ch.n_taps;
    for (uint64_t w = wa; w <= wb; ++w) {
        const uint64_t s_lo = window_start(w, W, m.p0, m.dp);
        const uint64_t s_hi = window_start(w + 1, W, m.p0, m.dp);
        const uint32_t a = (uint32_t)max((uint64_t)lo, s_lo > t0 ? s_lo - t0 : 0);
        const uint32_t b = (uint32_t)min((uint64_t)hi, s_hi - t0);
        int acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (uint32_t i = a + gtid; i < b; i += nthr) {
            const uint64_t n = t0 + i;
            const uint32_t phi = m.phi0 + (uint32_t)n * m.dphi;
            const uint32_t off = __builtin_amdgcn_perm(phi, lane4, kPermSel);
            const uint32_t e = *reinterpret_cast<const uint32_t*>(lut + off);
            int c, s;
            lut_cs(e, c, s);
            int wi, wq;
            if constexpr (fmt_complex(FMT)) {
                const uint32_t xw = static_cast<const uint32_t*>(sx)[iq_idx<PAD>(i)];
                const int xi = (int)(short)(xw & 0xFFFF), xq = (int)(short)(xw >> 16);
                wipe<GC_I8_IQ, int>(xi, xq, c, s, wi, wq);
            } else {
                const int x = static_cast<const short*>(sx)[i];
                wipe<GC_I8_REAL, int>(x, 0, c, s, wi, wq);
            }
            const uint64_t u = m.p0 + n * m.dp;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k < nk) {
                    const int64_t v = (int64_t)u + ch.taps[k];
                    int32_t chip = (int32_t)(v >> 32) % kCodeLen;
                    if (chip < 0) chip += kCodeLen;
                    const int r = (int)(short)(sgn_prn[chip] & 0xFFFF);
                    acc[2 * k] += wi * r;
                    acc[2 * k + 1] += wq * r;
                }
            }
        }
        for (int k = 0; k < 2 * nk; ++k) {
            const int t = wave_total_dpp(acc[k]);
            if ((threadIdx.x & 63) == 0 && t != 0) atomicAdd(d.at((uint32_t)w, k >> 1, k & 1), t);
        }
    }
}

// ---------------------------------------------------------------------------
// Float carrier (GC_CARRIER_F32): the same bins and runs with the carrier
// (cos, sin)(2 pi ph) from carrier_f32 and float sums.  A lane's run starts
// from its first sample's phase in FP64 (reduced to [0, 1)); inside a bin
// sample j takes ph + j * ff in fp32, and the bin's phase advance is added
// and reduced once per bin.  Dumps and the state's open dump are float.
struct DestF {
    float* out;
    gc_chan_state* st;
    uint64_t row0;        // ch * max_dumps
    int tap_stride;
    uint32_t m_close;
    __device__ __forceinline__ float* at(uint32_t w, int slot, int comp) const {
        if (w < m_close) return out + ((row0 + w) * tap_stride + slot) * 2 + comp;
        return &st->acc_f[slot][comp];
    }
};

__device__ __forceinline__ float sign_f(uint32_t word) { return (float)(int)(short)(word & 0xFFFF); }

// Wiped-off (I, Q) of one bin of len samples (Q > 0: q or q + 1 samples,
// the last weighted 0 or 1; Q == 0: any length).
template <int FMT, int Q, bool PAD>
__device__ __forceinline__ void bin_f32(const void* __restrict__ sx, uint32_t nb, float ph, float ff,
                                        uint32_t len, float& bi, float& bq) {
    bi = 0.0f;
    bq = 0.0f;
    auto one = [&](uint32_t j, float wt) {
        float c, s;
        carrier_f32(ph + (float)j * ff, c, s);
        if constexpr (fmt_complex(FMT)) {
            // blocked layout: bins of at most kIqPad + 1 samples are
            // consecutive dwords
            const uint32_t* xp = static_cast<const uint32_t*>(sx);
            const uint32_t xw = (Q > 0 && (!PAD || Q <= (int)kIqPad))
                                    ? xp[iq_idx<PAD>(nb) + j]
                                    : xp[iq_idx<PAD>(nb + j)];
            const float xi = wt * (float)(int)(short)(xw & 0xFFFF);
            const float xq = wt * (float)(int)(short)(xw >> 16);
            bi += xi * c + xq * s;
            bq += xq * c - xi * s;
        } else {
            const float x = wt * (float)static_cast<const short*>(sx)[nb + j];
            bi += x * c;
            bq -= x * s;
        }
    };
    if constexpr (Q > 0) {
#pragma unroll
        for (int j = 0; j < Q; ++j) one((uint32_t)j, 1.0f);
        one((uint32_t)Q, len > (uint32_t)Q ? 1.0f : 0.0f);
    } else {
        for (uint32_t j = 0; j < len; ++j) one(j, 1.0f);
    }
}

// Float run of one lane over chips [c, c + K) (as epl_run): ph0 is the phase
// of its first sample in cycles, reduced to [0, 1).
template <int FMT, int Q, bool PAD>
__device__ __forceinline__ void epl_run_f32(const void* __restrict__ sx, uint32_t nb, float ph,
                                            float ff, uint32_t e, uint32_t dp, uint32_t q,
                                            uint32_t r, uint32_t c, uint32_t K, uint32_t Kmax,
                                            uint32_t span, const uint32_t* __restrict__ sgn,
                                            const DestF d, const DevChan& ch) {
    float v[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};  // E, P, L: I, Q
    uint32_t w = (uint32_t)max(0.0f, (float)c * (1.0f / (float)span) - 1.0f);
    while ((w + 1) * span <= c) ++w;
    uint32_t wnext = (w + 1) * span;
    float sp = sign_f(sgn[0]), sc = sign_f(sgn[1]), sn = sign_f(sgn[2]);
    const int slot[3] = {ch.slot_e, ch.slot_p, ch.slot_l};
    const bool active = K > 0;
    for (uint32_t k = 0; k < Kmax; ++k) {
        if (k < K) {
            if (c == wnext) {  // a dump closes before this chip
#pragma unroll
                for (int t = 0; t < 6; ++t) {
                    atomicAdd(d.at(w, slot[t >> 1], t & 1), v[t]);
                    v[t] = 0.0f;
                }
                w += 1;
                wnext += span;
            }
            const float snn = sign_f(sgn[k + 3]);
            float bi, bq;
            // bin 0: E, P use C[c], L uses C[c-1]
            bool lt = e < r;
            uint32_t len = q + (lt ? 1u : 0u);
            e = lt ? e + dp - r : e - r;
            bin_f32<FMT, Q, PAD>(sx, nb, ph, ff, len, bi, bq);
            v[0] += bi * sc; v[1] += bq * sc;
            v[2] += bi * sc; v[3] += bq * sc;
            v[4] += bi * sp; v[5] += bq * sp;
            nb += len;
            ph += (float)len * ff;
            ph -= floorf(ph);
            // bin 1: E uses C[c+1], P, L use C[c]
            lt = e < r;
            len = q + (lt ? 1u : 0u);
            e = lt ? e + dp - r : e - r;
            bin_f32<FMT, Q, PAD>(sx, nb, ph, ff, len, bi, bq);
            v[0] += bi * sn; v[1] += bq * sn;
            v[2] += bi * sc; v[3] += bq * sc;
            v[4] += bi * sc; v[5] += bq * sc;
            nb += len;
            ph += (float)len * ff;
            ph -= floorf(ph);
            sp = sc;
            sc = sn;
            sn = snn;
            c += 1;
        }
    }
    // dump of the lane's last chip: equal dumps are contiguous lanes, each
    // group summed once
    uint64_t pending = __ballot(active);
    while (pending) {
        const int first = __ffsll((unsigned long long)pending) - 1;
        const uint32_t wsel = __builtin_amdgcn_readlane(w, first);
        const bool mine = active && w == wsel;
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            const float tot = wave_sum(mine ? v[t] : 0.0f);
            if ((int)(threadIdx.x & 63) == first) atomicAdd(d.at(wsel, slot[t >> 1], t & 1), tot);
        }
        pending &= ~__ballot(mine);
    }
}

// Float direct per-sample form over tile offsets [lo, hi) for up to 4 taps
// (as direct_range; each sample's phase in FP64).
template <int FMT, bool PAD>
__device__ __forceinline__ void direct_range_f32(const void* __restrict__ sx, uint32_t gtid,
                                                 uint32_t nthr, uint64_t t0, uint32_t lo,
                                                 uint32_t hi, const DevMeta& m, const DevChan& ch,
                                                 const uint32_t* __restrict__ sgn_prn,
                                                 const DestF d) {
    if (lo >= hi) return;
    const uint64_t W = m.window;
    const uint64_t wa = (m.p0 + (t0 + lo) * m.dp) / W;
    const uint64_t wb = (m.p0 + (t0 + hi - 1) * m.dp) / W;
    const int nk = ch.n_taps;
    for (uint64_t w = wa; w <= wb; ++w) {
        const uint64_t s_lo = window_start(w, W, m.p0, m.dp);
        const uint64_t s_hi = window_start(w + 1, W, m.p0, m.dp);
        const uint32_t a = (uint32_t)max((uint64_t)lo, s_lo > t0 ? s_lo - t0 : 0);
        const uint32_t b = (uint32_t)min((uint64_t)hi, s_hi - t0);
        float acc[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        for (uint32_t i = a + gtid; i < b; i += nthr) {
            const uint64_t n = t0 + i;
            const double p = m.phf0 + (double)n * m.ff;
            float c, s;
            carrier_f32((float)(p - floor(p)), c, s);
            float wi, wq;
            if constexpr (fmt_complex(FMT)) {
                const uint32_t xw = static_cast<const uint32_t*>(sx)[iq_idx<PAD>(i)];
                wipe<GC_I8_IQ, float>((float)(int)(short)(xw & 0xFFFF),
                                      (float)(int)(short)(xw >> 16), c, s, wi, wq);
            } else {
                wipe<GC_I8_REAL, float>((float)static_cast<const short*>(sx)[i], 0.0f, c, s, wi,
                                        wq);
            }
            const uint64_t u = m.p0 + n * m.dp;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k < nk) {
                    const int64_t v = (int64_t)u + ch.taps[k];
                    int32_t chip = (int32_t)(v >> 32) % kCodeLen;
                    if (chip < 0) chip += kCodeLen;
                    const float r = sign_f(sgn_prn[chip]);
                    acc[2 * k] += wi * r;
                    acc[2 * k + 1] += wq * r;
                }
            }
        }
        for (int k = 0; k < 2 * nk; ++k) {
            const float t = wave_sum(acc[k]);
            if ((threadIdx.x & 63) == 0 && t != 0.0f) atomicAdd(d.at((uint32_t)w, k >> 1, k & 1), t);
        }
    }
}

// A nibble of two 2-bit codes (sample j in bits [2j, 2j+1], code c -> 2c - 3)
// as an int16 pair.
__device__ __forceinline__ uint32_t codes_to_pair(uint32_t nib) {
    const short2_t c = as_s2((nib * 0x4001u) & 0x00030003u);
    const short2_t two = {2, 2}, m3 = {-3, -3};
    return as_u32(c * two + m3);
}

// Two int8 samples (bytes 0 and 1 of v) as an int16 pair.
__device__ __forceinline__ uint32_t bytes_to_pair(uint32_t v) {
    return ((uint32_t)(uint16_t)(int16_t)(int8_t)(v & 0xFF)) |
           ((uint32_t)(uint16_t)(int16_t)(int8_t)((v >> 8) & 0xFF) << 16);
}

// Complex tile samples s and s + 1 (s even) at their dwords: plain, or
// blocked (iq_at) and then again among the copies ending the previous
// block when they are among the first kIqPad of theirs.
template <bool PAD>
__device__ __forceinline__ void put_iq_pair(uint32_t* __restrict__ x, uint32_t s, uint32_t lo,
                                            uint32_t hi) {
    if constexpr (!PAD) {
        *reinterpret_cast<uint2*>(x + s) = uint2{lo, hi};
        return;
    }
    const uint32_t p = iq_at(s);
    x[p] = lo;
    x[p + 1] = hi;
    const uint32_t o = s & (kIqBlk - 1);
    if (s >= kIqBlk && o < kIqPad) {
        x[p - kIqPad] = lo;
        if (o + 1 < kIqPad) x[p + 1 - kIqPad] = hi;
    }
}

// Samples [t0, t0 + count) of the block into LDS (zero past its end); count
// is at most kXSamples and a multiple of 8 (complex) or 16 (real input).
// Complex samples take the plain or (PAD) the blocked layout.
template <int FMT, int kThreads, int kXSamples, bool PAD = false>
__device__ __forceinline__ void stage_tile(const uint8_t* __restrict__ samples, uint64_t n,
                                           uint64_t t0, void* sx, const uint32_t* tables,
                                           uint32_t count) {
    uint2* dst = reinterpret_cast<uint2*>(sx);  // real input: 4 samples per 8 bytes
    uint32_t* dx = reinterpret_cast<uint32_t*>(sx);  // complex input: see iq_at
    // A staged range inside the block (every one but the block's last):
    // units of 8 complex or 16 real samples (8, 4, 4 or 16 input bytes, 32
    // bytes out), four per thread and pass with all four loads issued before
    // any is decoded, so that the pass waits for memory once (a unit past
    // the end loads the last one and is not stored; the empty asm takes
    // every loaded value, so no load is left for after the first wait).
    constexpr int kPer = fmt_complex(FMT) ? 8 : 16;
    constexpr int kMaxPasses = (kXSamples / kPer + kThreads - 1) / kThreads;
    constexpr int kP = kMaxPasses < 4 ? kMaxPasses : 4;
    if (count % kPer == 0 && t0 + count <= n) {
        const int units = (int)(count / kPer);
        auto raw = [&](int u) {
            uint4 r = uint4{0u, 0u, 0u, 0u};
            if constexpr (FMT == GC_I8_IQ) {
                const uint2* src = reinterpret_cast<const uint2*>(samples + 2 * (t0 + 8ull * u));
                const uint2 a = src[0], b = src[1];
                r = uint4{a.x, a.y, b.x, b.y};
            } else if constexpr (FMT == GC_I2_IQ) {
                r.x = *reinterpret_cast<const uint32_t*>(samples + (t0 + 8ull * u) / 2);
            } else if constexpr (FMT == GC_I2_REAL) {
                r.x = *reinterpret_cast<const uint32_t*>(samples + (t0 + 16ull * u) / 4);
            } else {
                const uint2* src = reinterpret_cast<const uint2*>(samples + t0 + 16ull * u);
                const uint2 a = src[0], b = src[1];
                r = uint4{a.x, a.y, b.x, b.y};
            }
            return r;
        };
        auto put = [&](int u, const uint4 r) {
            const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                uint2 o;
                if constexpr (FMT == GC_I8_IQ || FMT == GC_I8_REAL) {
                    // two samples (complex) or four (real) per input dword
                    o.x = bytes_to_pair(w[k]);
                    o.y = bytes_to_pair(w[k] >> 16);
                } else if constexpr (FMT == GC_I2_IQ) {
                    // one byte: two complex samples, a nibble each
                    const uint32_t v = (w[0] >> (8 * k)) & 0xFFu;
                    o.x = codes_to_pair(v & 15u);
                    o.y = codes_to_pair(v >> 4);
                } else {
                    // one byte: four real samples
                    const uint32_t v = (w[0] >> (8 * k)) & 0xFFu;
                    o.x = codes_to_pair(v & 15u);
                    o.y = codes_to_pair(v >> 4);
                }
                if constexpr (fmt_complex(FMT))
                    put_iq_pair<PAD>(dx, 8u * u + 2u * k, o.x, o.y);
                else
                    dst[4 * u + k] = o;
            }
        };
        for (int u0 = threadIdx.x; u0 < units; u0 += kP * kThreads) {
            uint4 r[4] = {};
#pragma unroll
            for (int p = 0; p < kP; ++p) r[p] = raw(min(u0 + p * kThreads, units - 1));
            asm volatile(""
                         : "+v"(r[0].x), "+v"(r[0].y), "+v"(r[0].z), "+v"(r[0].w),
                           "+v"(r[1].x), "+v"(r[1].y), "+v"(r[1].z), "+v"(r[1].w),
                           "+v"(r[2].x), "+v"(r[2].y), "+v"(r[2].z), "+v"(r[2].w),
                           "+v"(r[3].x), "+v"(r[3].y), "+v"(r[3].z), "+v"(r[3].w));
#pragma unroll
            for (int p = 0; p < kP; ++p) {
                const int u = u0 + p * kThreads;
                if (u < units) put(u, r[p]);
            }
        }
        return;
    }
    if constexpr (FMT == GC_I8_IQ) {
        // count complex samples from t0 (a multiple of 4): the 4 bytes of
        // two samples give two (xI, xQ) int16 dwords
        for (int i = threadIdx.x; i < (int)count / 2; i += kThreads) {
            const uint64_t smp = t0 + 2ull * i;
            uint32_t v = 0;
            if (smp + 2 <= n) {
                v = *reinterpret_cast<const uint32_t*>(samples + 2 * smp);
            } else if (smp < n) {
                v = *reinterpret_cast<const uint16_t*>(samples + 2 * smp);
            }
            uint2 o;
            o.x = ((uint32_t)(uint16_t)(int16_t)(int8_t)(v & 0xFF)) |
                  ((uint32_t)(uint16_t)(int16_t)(int8_t)((v >> 8) & 0xFF) << 16);
            o.y = ((uint32_t)(uint16_t)(int16_t)(int8_t)((v >> 16) & 0xFF)) |
                  ((uint32_t)(uint16_t)(int16_t)(int8_t)(v >> 24) << 16);
            put_iq_pair<PAD>(dx, 2u * i, o.x, o.y);
        }
    } else if constexpr (FMT == GC_I2_IQ) {
        // t0 is even: byte t0/2 + i holds tile samples 2i and 2i+1, each a
        // nibble of I then Q codes; samples past the block read as zero
        for (int i = threadIdx.x; i < (int)count / 2; i += kThreads) {
            const uint64_t smp = t0 + 2ull * i;
            const uint32_t v = smp < n ? samples[smp >> 1] : 0u;
            const auto iq = [](uint32_t nib) {
                return (uint32_t)(uint16_t)(int16_t)(2 * (int)(nib & 3u) - 3) |
                       ((uint32_t)(uint16_t)(int16_t)(2 * (int)((nib >> 2) & 3u) - 3) << 16);
            };
            uint2 o;
            o.x = smp < n ? iq(v & 15u) : 0u;
            o.y = smp + 1 < n ? iq(v >> 4) : 0u;
            put_iq_pair<PAD>(dx, 2u * i, o.x, o.y);
        }
    } else if constexpr (FMT == GC_I2_REAL) {
        // t0 is a multiple of 4: byte t0/4 + i holds tile samples 4i .. 4i+3
        const uint64_t nbytes = (n + 3) / 4;
        const uint64_t b0 = t0 / 4;
        for (int i = threadIdx.x; i < (int)count / 4; i += kThreads) {
            const uint64_t b = b0 + i;
            uint2 o = {0u, 0u};
            if (b < nbytes) {
                const uint32_t* e = tables + kTabExpand + 2 * samples[b];  // 4 x int16
                o.x = e[0];
                o.y = e[1];
            }
            dst[i] = o;
        }
    } else {
        for (int i = threadIdx.x; i < (int)count / 4; i += kThreads) {
            const uint64_t b = t0 + 4ull * i;
            uint32_t v = 0;
            if (b + 4 <= n) {
                v = *reinterpret_cast<const uint32_t*>(samples + b);  // t0 % 4 == 0
            } else {
                for (int j = 0; j < 4; ++j)
                    if (b + j < n) v |= (uint32_t)samples[b + j] << (8 * j);
            }
            uint2 o;
            o.x = ((uint32_t)(uint16_t)(int16_t)(int8_t)(v & 0xFF)) |
                  ((uint32_t)(uint16_t)(int16_t)(int8_t)((v >> 8) & 0xFF) << 16);
            o.y = ((uint32_t)(uint16_t)(int16_t)(int8_t)((v >> 16) & 0xFF)) |
                  ((uint32_t)(uint16_t)(int16_t)(int8_t)(v >> 24) << 16);
            dst[i] = o;
        }
    }
}

// Channels [c_begin, c_end) of one receiver on its staged tile [t0, t1);
// n_act of them are left to this kernel (not refused, not periodic).
template <int FMT, class SH, int CARR = GC_CARRIER_LUT, bool PAD = false>
__device__ __forceinline__ void epl_tile(const void* __restrict__ s_x, const uint8_t* lut,
                                         uint64_t t0, uint64_t t1, int c_begin, int c_end,
                                         int n_act,
                                         const DevChan* __restrict__ chans,
                                         const DevMeta* __restrict__ metas,
                                         gc_chan_state* __restrict__ state,
                                         int32_t* __restrict__ out, int tap_stride,
                                         uint32_t max_dumps, const uint32_t* __restrict__ tables) {
    // Groups of whole waves take different channels at once: G groups of
    // kThreads / G threads, G the largest power of two up to the number of
    // channels left to this kernel with at least 128 threads per group.  A
    // lane's run of whole chips is then G times longer than with every
    // thread on one channel, so the per-run set-up and the closing wave sums
    // weigh less (at 5 MHz complex input, about 5 chips per run otherwise).
    static_assert((SH::kThreads & (SH::kThreads - 1)) == 0, "power-of-two block");
    int G = 1;
    while (2 * G <= n_act && SH::kThreads / (2 * G) >= 128) G *= 2;
    const uint32_t lg = (uint32_t)__builtin_ctz((uint32_t)(SH::kThreads / G));  // log2 group size
    const uint32_t kGroup = 1u << lg;
    const int tid = threadIdx.x;
    const uint32_t gtid = (uint32_t)tid & (kGroup - 1);
    const int grp = __builtin_amdgcn_readfirstlane(tid >> lg);
    const uint32_t lane4 = (tid & 63) * 4;
    // the group's channels: every G-th of those left to this kernel (when
    // that is all of them, every G-th channel, without reading the others)
    const bool all = n_act == c_end - c_begin;
    int seq = 0;   // rank of the channel among those left to this kernel
    for (int chn = c_begin + (all ? grp : 0); chn < c_end; chn += all ? G : 1) {
        if (!all) {
            if (metas[chn].status != GC_OK || metas[chn].path == kPathPeriodic) continue;
            if ((seq++ & (G - 1)) != grp) continue;
        }
        const DevMeta m = metas[chn];
        const DevChan& ch = chans[chn];
        const Dest d{out, state + chn, (uint64_t)chn * max_dumps, tap_stride, m.m_close};
        const DestF df{reinterpret_cast<float*>(out), state + chn, (uint64_t)chn * max_dumps,
                       tap_stride, m.m_close};
        const uint32_t* sgn_prn = tables + kTabSign + (ch.prn - 1) * kSignLen;
        const uint32_t tl = (uint32_t)(t1 - t0);
        auto direct = [&](uint32_t lo, uint32_t hi) {
            if constexpr (CARR == GC_CARRIER_F32)
                direct_range_f32<FMT, PAD>(s_x, gtid, kGroup, t0, lo, hi, m, ch, sgn_prn, df);
            else
                direct_range<FMT, PAD>(s_x, lut, gtid, kGroup, lane4, t0, lo, hi, m, ch, sgn_prn, d);
        };
        if (m.path != kPathBinned) {
            direct(0, tl);
            continue;
        }
        // block-edge samples outside whole chips
        {
            const uint64_t he = m.head_end, tb = m.tail_beg;
            if (he > t0) direct(0, (uint32_t)min(he, t1) - (uint32_t)t0);
            if (t1 > tb) direct((uint32_t)(max(tb, t0) - t0), tl);
        }
        // whole chips whose first sample lies in [t0, t1)
        const uint64_t u0 = m.p0 + t0 * m.dp;
        const uint64_t u1 = m.p0 + t1 * m.dp;
        uint64_t ca = (u0 + 0xFFFFFFFFull) >> 32;
        uint64_t cb = (u1 + 0xFFFFFFFFull) >> 32;
        if (ca < m.c_full0) ca = m.c_full0;
        if (cb > m.c_full1) cb = m.c_full1;
        if (cb <= ca) continue;
        const uint32_t N = (uint32_t)(cb - ca);
        const uint32_t k0 = (uint32_t)(((uint64_t)gtid * N) >> lg);
        const uint32_t k1 = (uint32_t)(((uint64_t)(gtid + 1) * N) >> lg);
        const uint32_t K = k1 - k0;
        const uint32_t Kmax = (N + kGroup - 1) >> lg;
        const uint32_t c = (uint32_t)(ca + k0);
        const uint32_t dp = (uint32_t)m.dp;
        const float inv_dp = 1.0f / (float)dp;
        uint32_t nrel = 0, e = 0, phi = 0;
        float phf = 0.0f;
        if (K > 0) {
            // first sample of chip c: ceil((c*2^32 - u0) / dp), estimated with
            // a float reciprocal (D < 2^47, so the estimate is within a few
            // samples) and made exact with integer checks
            const uint64_t D = ((uint64_t)c << 32) - u0;
            const float df = (float)(uint32_t)(D >> 32) * 4294967296.0f + (float)(uint32_t)D;
            uint64_t nr = (uint64_t)(uint32_t)max(0.0f, df * inv_dp - 2.0f);
            while (nr * dp < D) ++nr;
            nrel = (uint32_t)nr;
            e = (uint32_t)(nr * dp - D);
            phi = m.phi0 + (uint32_t)(t0 + nrel) * m.dphi;
            if constexpr (CARR == GC_CARRIER_F32) {
                const double p = m.phf0 + (double)(t0 + nrel) * m.ff;
                phf = (float)(p - floor(p));
            }
        }
        const uint32_t q = (uint32_t)((1ull << 31) / dp);
        const uint32_t r = (uint32_t)((1ull << 31) - (uint64_t)q * dp);
        const uint32_t span = (uint32_t)(m.window >> 32);
        const uint32_t* sgn = sgn_prn + (c + kCodeLen - 1) % kCodeLen;
#define GC_RUN(QQ)                                                                           \
    if constexpr (CARR == GC_CARRIER_F32)                                                     \
        epl_run_f32<FMT, QQ, PAD>(s_x, nrel, phf, (float)m.ff, e, dp, q, r, c, K, Kmax, span, sgn, \
                             df, ch);                                                         \
    else                                                                                      \
        epl_run<FMT, QQ, PAD>(s_x, lut, lane4, nrel, phi, m.dphi, e, dp, q, r, c, K, Kmax, span, sgn, \
                         d, ch)
        switch (q) {  // bins of q or q + 1 samples
            case 1: GC_RUN(1); break;
            case 2: GC_RUN(2); break;
            case 3: GC_RUN(3); break;
            case 4: GC_RUN(4); break;
            case 7: GC_RUN(7); break;
            case 8: GC_RUN(8); break;
            case 9: GC_RUN(9); break;
            case 10: GC_RUN(10); break;
            default: GC_RUN(0); break;
        }
#undef GC_RUN
    }
}

// One tile [t0, t0 + tile_len) of a block of n samples for channels
// [c_begin, c_end): staged and correlated whole (real input) or as two half
// tiles (complex input, one dword per sample).  tile_len is at most SH::kTile
// and a multiple of 16.
template <int FMT, class SH, int CARR = GC_CARRIER_LUT, bool PAD = false>
__device__ __forceinline__ void tile_pass(const uint8_t* __restrict__ samples, uint64_t n,
                                          uint64_t t0, uint32_t tile_len, void* s_x,
                                          const uint8_t* lut,
                                          int c_begin, int c_end, int n_act,
                                          const DevChan* __restrict__ chans,
                                          const DevMeta* __restrict__ metas,
                                          gc_chan_state* __restrict__ state,
                                          int32_t* __restrict__ out, int tap_stride,
                                          uint32_t max_dumps, const uint32_t* __restrict__ tables) {
    constexpr int kParts = fmt_complex(FMT) ? 2 : 1;
    constexpr int kStaged = fmt_complex(FMT) ? SH::kXSamplesIQ : SH::kXSamples;
    const uint32_t part = tile_len / kParts;
#pragma unroll
    for (int h = 0; h < kParts; ++h) {
        const uint64_t a = t0 + (uint64_t)h * part;
        if (a >= n) break;
        const uint64_t b = min(n, a + part);
        __syncthreads();
        stage_tile<FMT, SH::kThreads, kStaged, PAD>(samples, n, a, s_x, tables, part + kMargin);
        __syncthreads();
        epl_tile<FMT, SH, CARR, PAD>(s_x, lut, a, b, c_begin, c_end, n_act, chans, metas, state, out,
                                tap_stride, max_dumps, tables);
    }
}

// Whether complex tiles take the blocked layout: some binned channel's
// samples per chip (2^32 / dp) lie within 1/256 of a nonzero multiple of 8,
// so that its lanes' runs would start on a few banks.  The same for every
// block of a launch (it reads only the call's metas).
__device__ __forceinline__ bool iq_blocked(const DevMeta* __restrict__ metas, int n_chan) {
    bool pad = false;
    for (int c = 0; c < n_chan; ++c) {
        const DevMeta& m = metas[c];
        if (m.status != GC_OK || m.path != kPathBinned || m.dp == 0) continue;
        const float spc = 4294967296.0f / (float)m.dp;
        const float k = rintf(spc * 0.125f);
        pad = pad || (k >= 1.0f && fabsf(spc - 8.0f * k) < 1.0f / 256.0f);
    }
    return __builtin_amdgcn_readfirstlane((int)pad) != 0;
}

// FIXED: tiles of ShapePlan::kTile samples (tile_len unused), where a
// compile-time tile length keeps scalar state out of spill slots
template <int FMT, int CARR, bool FIXED>
__global__ __launch_bounds__(ShapePlan::kThreads) void k_epl(
    const uint8_t* __restrict__ samples, uint64_t n, const DevChan* __restrict__ chans,
    const DevMeta* __restrict__ metas, gc_chan_state* __restrict__ state,
    int32_t* __restrict__ out, int tap_stride, uint32_t max_dumps,
    const uint32_t* __restrict__ tables, int n_chan, uint32_t n_tiles, uint32_t tile_len) {
    using SH = ShapePlan;
    // one LDS block: the per-lane carrier tables at offset 0 (so the v_perm
    // result is the address itself), then the staged samples
    __shared__ __attribute__((aligned(16))) uint8_t s_lds[SH::kLdsBytes];
    uint32_t* s_lut = reinterpret_cast<uint32_t*>(s_lds);
    void* s_x = s_lds + kLutWords * 4;
    const int tid = threadIdx.x;
    // channels left to this kernel: not refused and not on the periodic path
    int n_act = 0;
    for (int c = 0; c < n_chan; ++c)
        n_act += metas[c].status == GC_OK && metas[c].path != kPathPeriodic;
    if (n_act == 0) return;
    if constexpr (CARR == GC_CARRIER_LUT)
        for (int i = tid; i < kLutWords; i += SH::kThreads) s_lut[i] = tables[kTabLut + (i >> 6)];

    const uint32_t tl = FIXED ? (uint32_t)SH::kTile : tile_len;
    const bool pad = fmt_complex(FMT) && iq_blocked(metas, n_chan);
    for (uint32_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const uint64_t t0 = (uint64_t)tile * tl;
        if (pad)
            tile_pass<FMT, SH, CARR, fmt_complex(FMT)>(samples, n, t0, tl, s_x, s_lds, 0, n_chan,
                                                       n_act, chans, metas, state, out,
                                                       tap_stride, max_dumps, tables);
        else
            tile_pass<FMT, SH, CARR>(samples, n, t0, tl, s_x, s_lds, 0, n_chan, n_act, chans,
                                     metas, state, out, tap_stride, max_dumps, tables);
    }
}

// Many receivers in one persistent launch: work item i is tile
// i - tile_begin[r] of the receiver r with tile_begin[r] <= i < tile_begin[r+1]
// (items taken in the order given by `order` when it is not null); the tile
// is staged in the receiver's format and correlated for its channels.
template <class SH>
__global__ __launch_bounds__(SH::kThreads) void k_epl_batch(
    const DevRx* __restrict__ rx, int n_rx, const uint32_t* __restrict__ order,
    uint32_t n_items, const uint32_t* __restrict__ n_items_dev,
    const DevChan* __restrict__ chans, const DevMeta* __restrict__ metas,
    gc_chan_state* __restrict__ state, int32_t* __restrict__ out, int tap_stride,
    uint32_t max_dumps, const uint32_t* __restrict__ tables) {
    __shared__ __attribute__((aligned(16))) uint8_t s_lds[SH::kLdsBytes];
    uint32_t* s_lut = reinterpret_cast<uint32_t*>(s_lds);
    void* s_x = s_lds + kLutWords * 4;
    const int tid = threadIdx.x;
    // the item count written by the set-up's item selection, when given
    if (n_items_dev) n_items = min(n_items, *n_items_dev);
    if (blockIdx.x >= n_items) return;
    for (int i = tid; i < kLutWords; i += SH::kThreads) s_lut[i] = tables[kTabLut + (i >> 6)];
    for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const uint32_t item = order ? order[it] : it;
        // receiver of this item: last r with tile_begin[r] <= item
        int lo = 0, hi = n_rx - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (rx[mid].tile_begin <= item) lo = mid; else hi = mid - 1;
        }
        const DevRx& R = rx[lo];
        // nothing to do when every channel of the receiver is refused or on
        // the periodic path (uniform over the block)
        int n_act = 0;
        for (int c = R.chan_begin; c < R.chan_end; ++c)
            n_act += metas[c].status == GC_OK && metas[c].path != kPathPeriodic;
        if (n_act == 0) continue;
        const uint64_t t0 = (uint64_t)(item - R.tile_begin) * SH::kTile;
        if (R.fmt == GC_I2_REAL)
            tile_pass<GC_I2_REAL, SH>(R.samples, R.n, t0, SH::kTile, s_x, s_lds, R.chan_begin, R.chan_end, n_act,
                                      chans, metas, state, out, tap_stride, max_dumps, tables);
        else if (R.fmt == GC_I8_IQ)
            tile_pass<GC_I8_IQ, SH>(R.samples, R.n, t0, SH::kTile, s_x, s_lds, R.chan_begin, R.chan_end, n_act,
                                    chans, metas, state, out, tap_stride, max_dumps, tables);
        else if (R.fmt == GC_I2_IQ)
            tile_pass<GC_I2_IQ, SH>(R.samples, R.n, t0, SH::kTile, s_x, s_lds, R.chan_begin, R.chan_end, n_act,
                                    chans, metas, state, out, tap_stride, max_dumps, tables);
        else
            tile_pass<GC_I8_REAL, SH>(R.samples, R.n, t0, SH::kTile, s_x, s_lds, R.chan_begin, R.chan_end, n_act,
                                      chans, metas, state, out, tap_stride, max_dumps, tables);
    }
}

}  // namespace

int epl_blocks_per_device(int device) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        cus = 256;
    return cus > 0 ? cus : 256;
}

hipError_t launch_epl(const uint8_t* samples, uint64_t n, int fmt, int carrier,
                      const DevChan* chans, const DevMeta* meta, gc_chan_state* state, int n_chan,
                      int32_t* out, int tap_stride, uint32_t max_dumps, const uint32_t* tables,
                      int grid, hipStream_t s) {
    if (n == 0) return hipSuccess;
    using SH = ShapePlan;
    // Balanced tiles: every block takes k = ceil(n / (kTile grid)) tiles, of
    // 256 m samples with m the smallest odd number reaching n / (k grid), so
    // that the last round does not leave blocks idle.  256 m keeps a group's
    // lane runs an odd or half-odd number of LDS dwords apart (few bank
    // conflicts for complex samples, one dword each); taken only when it
    // shortens the largest block's share by more than 1/16, as other
    // lengths can split the chips of a periodic-rate tile unevenly over the
    // lanes.
    constexpr uint64_t kMinTile = 2048;
    const uint64_t G = (uint64_t)max(grid, 1);
    const uint64_t per = (n + (uint64_t)SH::kTile * G - 1) / ((uint64_t)SH::kTile * G);
    uint64_t m = ((n + per * G - 1) / (per * G) + 255) / 256;
    m |= 1;
    const uint64_t cand = max(kMinTile, 256 * m);
    const uint64_t tl = 16 * cand < 15 * (uint64_t)SH::kTile ? cand : (uint64_t)SH::kTile;
    const uint32_t tile_len = (uint32_t)tl;
    const uint32_t n_tiles = (uint32_t)((n + tl - 1) / tl);
    const int g = (int)min((uint32_t)grid, n_tiles);
    const bool fixed = tile_len == (uint32_t)SH::kTile;
#define GC_EPL(F, C)                                                                            \
    do {                                                                                        \
        if (fixed)                                                                              \
            hipLaunchKernelGGL((k_epl<F, C, true>), dim3(g), dim3(SH::kThreads), 0, s, samples, \
                               n, chans, meta, state, out, tap_stride, max_dumps, tables,       \
                               n_chan, n_tiles, tile_len);                                      \
        else                                                                                    \
            hipLaunchKernelGGL((k_epl<F, C, false>), dim3(g), dim3(SH::kThreads), 0, s,         \
                               samples, n, chans, meta, state, out, tap_stride, max_dumps,      \
                               tables, n_chan, n_tiles, tile_len);                              \
    } while (0)
    const bool f32 = carrier == GC_CARRIER_F32;
    if (fmt == GC_I2_REAL) {
        if (f32) {
            GC_EPL(GC_I2_REAL, GC_CARRIER_F32);
        } else {
            GC_EPL(GC_I2_REAL, GC_CARRIER_LUT);
        }
    } else if (fmt == GC_I8_REAL) {
        if (f32) {
            GC_EPL(GC_I8_REAL, GC_CARRIER_F32);
        } else {
            GC_EPL(GC_I8_REAL, GC_CARRIER_LUT);
        }
    } else if (fmt == GC_I2_IQ) {
        if (f32) {
            GC_EPL(GC_I2_IQ, GC_CARRIER_F32);
        } else {
            GC_EPL(GC_I2_IQ, GC_CARRIER_LUT);
        }
    } else if (fmt == GC_I8_IQ) {
        if (f32) {
            GC_EPL(GC_I8_IQ, GC_CARRIER_F32);
        } else {
            GC_EPL(GC_I8_IQ, GC_CARRIER_LUT);
        }
    } else {
        return hipErrorInvalidValue;
    }
#undef GC_EPL
    return hipGetLastError();
}

// Batch shapes the tuner chooses from (threads per block, samples per lane run).
namespace {
using ShapeB0 = Shape<512, 90>;   // 46080-sample tiles
using ShapeB1 = Shape<256, 90>;   // 23040
using ShapeB2 = Shape<512, 46>;   // 23552
using ShapeB3 = Shape<256, 182>;  // 46592
template <class SH>
uint32_t tiles_of(uint64_t n) { return (uint32_t)((n + SH::kTile - 1) / SH::kTile); }
}  // namespace

int epl_batch_shapes() { return 4; }

uint32_t epl_batch_tile(int shape) {
    switch (shape) {
        case 0: return ShapeB0::kTile;
        case 1: return ShapeB1::kTile;
        case 2: return ShapeB2::kTile;
        case 3: return ShapeB3::kTile;
    }
    return 0;
}

hipError_t launch_epl_batch(int shape, int grid, const DevRx* rx, int n_rx,
                            const uint32_t* order, uint32_t n_items, const uint32_t* n_items_dev,
                            const DevChan* chans, const DevMeta* meta, gc_chan_state* state,
                            int32_t* out, int tap_stride, uint32_t max_dumps,
                            const uint32_t* tables, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    const int g = (int)min((uint32_t)grid, n_items);
#define GC_B(SH)                                                                              \
    hipLaunchKernelGGL((k_epl_batch<SH>), dim3(g), dim3(SH::kThreads), 0, s, rx, n_rx, order, \
                       n_items, n_items_dev, chans, meta, state, out, tap_stride, max_dumps,   \
                       tables)
    switch (shape) {
        case 0: GC_B(ShapeB0); break;
        case 1: GC_B(ShapeB1); break;
        case 2: GC_B(ShapeB2); break;
        case 3: GC_B(ShapeB3); break;
        default: return hipErrorInvalidValue;
    }
#undef GC_B
    return hipGetLastError();
}

}  // namespace gc
