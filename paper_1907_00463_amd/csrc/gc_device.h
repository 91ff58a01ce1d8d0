// gc_device.h -- device helpers shared by the libgnsscorr kernels.
#pragma once

#include "gc_internal.h"

namespace gc {

// Layout of the context's device table block (uint32 words).
constexpr int kTabG1 = 0;     // 32 words: G1 sequence, bit i of word i/32
constexpr int kTabG2 = 32;    // 32 words: G2 sequence
constexpr int kTabLut = 64;   // 256 words: (cos low 16 | sin high 16), int16 each
constexpr int kTabWords = 320;
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
    } else {
        const int code = (s[n >> 2] >> (2 * (n & 3))) & 3;
        i = 2 * code - 3;
        q = 0;
    }
}

// Carrier table entry -> (c, s).
__device__ __forceinline__ void lut_cs(uint32_t e, int& c, int& s) {
    c = (int)(int16_t)(e & 0xFFFF);
    s = (int)(int16_t)(e >> 16);
}

// Wipe-off by exp(-j*theta): real (x*c, -x*s); complex (xi*c + xq*s, xq*c - xi*s).
template <int FMT, typename T>
__device__ __forceinline__ void wipe(T xi, T xq, T c, T s, T& wi, T& wq) {
    if constexpr (FMT == GC_I8_IQ) {
        wi = xi * c + xq * s;
        wq = xq * c - xi * s;
    } else {
        wi = xi * c;
        wq = -(xi * s);
    }
}

// First sample index of window m (m >= 1): ceil((m*W - p0) / dp).
__device__ __forceinline__ uint64_t window_start(uint64_t m, uint64_t W, uint64_t p0, uint64_t dp) {
    return m == 0 ? 0 : (m * W - p0 + dp - 1) / dp;
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
