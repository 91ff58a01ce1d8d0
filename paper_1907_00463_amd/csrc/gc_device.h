// gc_device.h -- device helpers shared by the libgnsscorr kernels.
#pragma once

#include "gc_internal.h"

namespace gc {

// Layout of the context's device table block (uint32 words).
constexpr int kTabG1 = 0;     // 32 words: G1 sequence, bit i of word i/32
constexpr int kTabG2 = 32;    // 32 words: G2 sequence
constexpr int kTabLut = 64;   // 256 words: (cos low 16 | sin high 16), int16 each
constexpr int kTabExpand = 320;  // 512 words: packed 2-bit byte -> its 4 samples as int16 (2 words)
constexpr int kTabSign = 832;    // 32 PRNs x kSignLen words: chip i -> (s, s) int16, s = +-1

// Periodic form (half chips of exactly L = 2, 4, 8 or 10 samples): tile
// length, the most 64-bin steps one lane makes in a tile (at most tile/L + 2
// bins), and the most steps whose code signs are fetched ahead of use.
constexpr int kPbinTileSamples = 23552;
constexpr int kPbinMinBinLen = 2;
constexpr int kPbinMaxSteps = (kPbinTileSamples / kPbinMinBinLen + 2 + 63) / 64;
constexpr int kPbinMaxAhead = 8;
// chip index 0..1022 followed by a wrapped copy long enough for a run of
// periodic steps (32 chips per step, read up to kPbinMaxAhead steps ahead)
// from any chip
constexpr int kSignLen = 1023 + 32 * (kPbinMaxSteps + kPbinMaxAhead + 1);
// Multi-tap replica operand: 32 PRNs x 4 byte positions x 2 parities x
// kMtapHalfWords words; word y of parity r of byte position b holds chip
// (2y + r) mod 1023 of the PRN as an int8 in byte b and zeros in the other
// bytes (so four chips two apart are one 16-byte read).
constexpr int kMtapHalfWords = 1040;
constexpr int kMtapCodeWords = 2 * kMtapHalfWords;
constexpr int kTabMtapCode = kTabSign + 32 * kSignLen;
constexpr int kTabWords = kTabMtapCode + 32 * 4 * kMtapCodeWords;
constexpr int kLutAbsSumMax = 34;  // max over l of |cos_l| + |sin_l| at amplitude 24

// Chip i of the C/A code whose G2 delay is d: G1[i] XOR G2[(i - d) mod 1023],
// logic 0 -> +1, logic 1 -> -1.
__device__ __forceinline__ int8_t ca_chip(const uint32_t* tables, int d, int i) {
    int j = i - d;
    if (j < 0) j += kCodeLen;
    uint32_t b1 = (tables[kTabG1 + (i >> 5)] >> (i & 31)) & 1u;
    uint32_t b2 = (tables[kTabG2 + (j >> 5)] >> (j & 31)) & 1u;
    return (b1 ^ b2) ? (int8_t)-1 : (int8_t)1;
}

// Complex sample formats (the wipe-off multiplies xI + j xQ by exp(-j*theta)).
constexpr bool fmt_complex(int fmt) { return fmt == GC_I8_IQ || fmt == GC_I2_IQ; }

// Unpacked sample: real formats leave q = 0.
template <int FMT>
__device__ __forceinline__ void load_sample(const uint8_t* __restrict__ s, uint64_t n, int& i, int& q) {
    if constexpr (FMT == GC_I8_REAL) {
        i = (int)(int8_t)s[n];
        q = 0;
    } else if constexpr (FMT == GC_I8_IQ) {
        const uint16_t v = *reinterpret_cast<const uint16_t*>(s + 2 * n);
        i = (int)(int8_t)(v & 0xFF);
        q = (int)(int8_t)(v >> 8);
    } else if constexpr (FMT == GC_I2_REAL) {
        const int code = (s[n >> 2] >> (2 * (n & 3))) & 3;
        i = 2 * code - 3;
        q = 0;
    } else {  // 2-bit complex: I then Q code of sample n in the nibble n & 1
        const int nib = (s[n >> 1] >> (4 * (n & 1))) & 15;
        i = 2 * (nib & 3) - 3;
        q = 2 * (nib >> 2) - 3;
    }
}

// Carrier table entry -> (c, s).
__device__ __forceinline__ void lut_cs(uint32_t e, int& c, int& s) {
    c = (int)(int16_t)(e & 0xFFFF);
    s = (int)(int16_t)(e >> 16);
}

// Float carrier: (cos, sin)(2*pi*ph) for a phase ph in cycles, 0 <= ph < 1,
// by the VALU's sine and cosine instructions (their argument is in
// revolutions).  Every float-carrier kernel calls this one function, and
// gc_carrier_f32_error measures it against double precision.
__device__ __forceinline__ void carrier_f32(float ph, float& c, float& s) {
    c = __builtin_amdgcn_cosf(ph);
    s = __builtin_amdgcn_sinf(ph);
}

// Wipe-off by exp(-j*theta): real (x*c, -x*s); complex (xi*c + xq*s, xq*c - xi*s).
template <int FMT, typename T>
__device__ __forceinline__ void wipe(T xi, T xq, T c, T s, T& wi, T& wq) {
    if constexpr (fmt_complex(FMT)) {
        wi = xi * c + xq * s;
        wq = xq * c - xi * s;
    } else {
        wi = xi * c;
        wq = -(xi * s);
    }
}

// Largest |term| of one sample in a packed int16 bin sum: x*c or x*s (real
// input), and for complex input each of the two planes (xI, xQ)*c and
// (xQ, xI)*s that the kernels sum separately.
__device__ __forceinline__ uint64_t bin_plane_max(int fmt) {
    return (fmt == GC_I2_REAL || fmt == GC_I2_IQ) ? 3ull * GC_LUT_AMP : 128ull * GC_LUT_AMP;
}

// Binned E/P/L form: tile geometry and the per-channel condition on the code
// step.  A chip must fit in the staged margin, and a half-chip bin sum must
// fit int16 (bin length <= q + 1 samples, q = floor(2^31 / dp)).
constexpr int kEplMarginSamples = 128;
__device__ __forceinline__ bool binned_geometry_ok(uint64_t dp) {
    return dp != 0 && dp < (1ull << 31) && dp * (kEplMarginSamples - 1) >= (1ull << 32);
}
__device__ __forceinline__ bool binned_ok(int fmt, uint64_t dp) {
    if (!binned_geometry_ok(dp)) return false;
    const uint64_t q = (1ull << 31) / dp;
    return (q + 1) * bin_plane_max(fmt) <= 32767ull;
}

// Periodic form: half chips of exactly L samples (L = 2, 4, 8 or 10), with
// at most one one-sample slip of the bin grid per tile of kPbinTileSamples
// samples.
__device__ __forceinline__ int periodic_bin_len(int fmt, uint64_t dp) {
    if (dp == 0 || dp >= (1ull << 31)) return 0;
    const uint64_t L = ((1ull << 31) + dp / 2) / dp;  // nearest integer to 2^31 / dp
    if (L != 2 && L != 4 && L != 8 && L != 10) return 0;
    if (L * bin_plane_max(fmt) > 32767ull) return 0;
    const int64_t D = (int64_t)(L * dp) - (int64_t)(1ull << 31);
    const uint64_t drift = (uint64_t)(D < 0 ? -D : D) * (kPbinTileSamples / L + 2);
    return drift < dp ? (int)L : 0;
}

// First sample index of window m (m >= 1): ceil((m*W - p0) / dp).
__device__ __forceinline__ uint64_t window_start(uint64_t m, uint64_t W, uint64_t p0, uint64_t dp) {
    return m == 0 ? 0 : (m * W - p0 + dp - 1) / dp;
}

// Wavefront sum of v over all 64 lanes, returned to every lane: an
// inclusive scan with DPP row shifts (within 16-lane rows) and row
// broadcasts (across rows) leaves the total in lane 63.
__device__ __forceinline__ int wave_total_dpp(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// Six wavefront sums at once (all 64 lanes active).  The six values (two
// zeros pad them to eight) are halved over lane pairs three times, lane
// l ^ 7, then l ^ 2, then l ^ 1: each lane keeps the half its lane bit picks
// and adds the partner's copy of that half, so that afterwards lane l holds
// value l & 7 summed over its group of eight lanes.  That one value is then
// summed over the row (l ^ 8) and over the four rows (l ^ 16, l ^ 32).
// Lanes 0-5 (and 8-13, ...) return the totals of v[0] .. v[5].
__device__ __forceinline__ int wave_total6(const int (&v)[6]) {
    const uint32_t lane = threadIdx.x & 63;
    const bool b2 = (lane & 4) != 0, b1 = (lane & 2) != 0, b0 = (lane & 1) != 0;
    int u[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int lo = v[k], hi = k + 4 < 6 ? v[k + 4] : 0;
        const int send = b2 ? lo : hi;
        u[k] = (b2 ? hi : lo) + __builtin_amdgcn_update_dpp(0, send, 0x141, 0xf, 0xf, false);  // row_half_mirror
    }
    int w[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int send = b1 ? u[k] : u[k + 2];
        w[k] = (b1 ? u[k + 2] : u[k]) + __builtin_amdgcn_update_dpp(0, send, 0x4E, 0xf, 0xf, false);  // quad_perm [2,3,0,1]
    }
    int t = (b0 ? w[1] : w[0]) +
            __builtin_amdgcn_update_dpp(0, b0 ? w[0] : w[1], 0xB1, 0xf, 0xf, false);  // quad_perm [1,0,3,2]
    t += __builtin_amdgcn_update_dpp(0, t, 0x128, 0xf, 0xf, false);  // row_ror:8
    t += __shfl_xor(t, 16, 64);
    t += __shfl_xor(t, 32, 64);
    return t;
}

// Wavefront sum (64 lanes) with DPP-backed cross-lane moves.
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace gc
