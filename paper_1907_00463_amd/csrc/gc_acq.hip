// gc_acq.hip -- acquisition search (parallel code-phase search over Doppler
// bins and PRNs, Sec. 3.3 and 3.7) as an exact int8 contraction on the
// matrix cores.
//
// The search computes, for Knc blocks of Mc code periods at R samples per
// chip (N = 1023 R samples per period), the power
//     P[p, d, tau] = sum_b |Y_b[p, d, tau]|^2,
//     Y_b[p, d, tau] = sum_{n in block b} w_d[n] C_p[floor((n + tau) / R) mod 1023],
// where w_d is the sample wiped off by the carrier table at bin d's NCO
// phase.  That phase is n * step_d from the first sample of the buffer and
// continues across blocks.  Every value is an integer and is computed exactly.
//
// Grouping by chip: with tau = R j + r (0 <= r < R), floor((n + tau) / R) =
// j + floor((n + r) / R), so
//     S_r[c]       = sum of w over the samples of the block whose
//                    floor((n + r) / R) = c (mod 1023)
//     Y[R j + r]   = sum_c S_r[c] C[(c + j) mod 1023].
// For every (bin, r, I/Q) this is a 1023 x 1023 circulant product with the
// code.  Together they form one dense GEMM per PRN: rows (bin, r, I/Q),
// contraction over chips c and columns j.  It does 1/R of the work of the
// direct sample-by-sample correlation.
//
//   k_acq_sums    forms S exactly in int32 and writes each value as int8
//                 digits in base 128: 2 digits when |S| < 2^14, else 4.
//                 Each digit is one operand row.
//   k_acq_corr    runs v_mfma_i32_32x32x32_i8 over c.  The code operand
//                 (+-1) comes from 16 byte-shifted copies of the doubled
//                 code in LDS, so every lane's 16 consecutive chips are one
//                 aligned 16-byte read.  The kernel recombines the digits in
//                 int64 and adds |Y|^2 over the blocks.
//   k_acq_reduce  per (PRN, bin, chip): the largest power over r (the
//                 lowest r on ties), plus the optional full surface.  Per
//                 (PRN, bin): the largest chip value (the lowest chip on ties).
//   k_acq_detect  per PRN: the peak bin (the lowest on ties), the peak, and
//                 the second peak at least two chips (circularly) from the
//                 peak's chip in that bin; then the ratio and the decision.
#include <math.h>

#include <algorithm>
#include <vector>

#include "gc_device.h"
#include "gc_internal.h"

struct gc_acq {
    int device;
    gc_ctx* ctx;
    int fmt, R, n_bins, n_prn, Mc, Knc, nd;
    double f_lo, f_step;
    int n_x;          // bins * R
    int nt;           // MFMA row blocks per tile (3 or 4)
    int rows_pad;     // operand rows, padded to the row tile
    uint64_t scratch;
    int8_t* d_sd;     // [Knc][rows_pad][1024] digit rows
    int8_t* d_codes;  // [n_prn][16][2064] byte-shifted code copies
    uint32_t* d_steps;
    int32_t* d_prns;
    uint64_t* d_pw;       // [n_prn][n_x][1024] power per (bin, r) row and chip column
    uint64_t* d_chipmax;  // [n_prn][n_bins][1024]
    uint8_t* d_chiparg;   // [n_prn][n_bins][1024]
    uint64_t* d_binmax;   // [n_prn][n_bins]
    uint32_t* d_binarg;   // [n_prn][n_bins]
    // timing slots (empty: off): events before the four kernels and after the last
    std::vector<hipEvent_t> ev;  // [slot][5]
    std::vector<uint8_t> ev_used;
    uint64_t calls = 0;
};

namespace gc {

namespace {

constexpr int kAcqTabStride = 2064;  // bytes per code copy; = 16 mod 128 spreads the copies over banks
constexpr int kAcqCols = 256;        // columns per block (64 per wave)
constexpr int kAcqKc = 128;          // contraction chunk staged per step
constexpr int kAcqARow = 144;        // staged row stride: 8 rows of one read hit distinct banks
constexpr int kAcqK = 1024;          // chips, padded (chip 1023 of every row is 0)
constexpr int kAcqTabBytes = 16 * kAcqTabStride;  // one PRN's code copies
static_assert(kAcqTabStride % 16 == 0 && kAcqTabStride >= 2032, "aligned reads up to chip 2046");
static_assert(kAcqARow % 16 == 0, "aligned row reads");

typedef int int4v __attribute__((ext_vector_type(4)));
typedef int int16v __attribute__((ext_vector_type(16)));

// Operand row of (X = bin * R + r, iq, digit).  Two digits: the four rows
// of X are consecutive (I lo, I hi, Q lo, Q hi), which one lane of a 32x32
// MFMA block holds together.  Four digits: 16-row groups hold X even and
// odd as I(even), I(odd), Q(even), Q(odd), four rows each, so that a lane
// holds all eight rows of one X.
template <int ND>
__device__ __forceinline__ int acq_row(int X, int iq, int k) {
    if constexpr (ND == 2) return 4 * X + 2 * iq + k;
    else return 16 * (X >> 1) + 4 * (X & 1) + 8 * iq + k;
}

constexpr int kSumThreads = 128;

template <int FMT, int ND>
__global__ __launch_bounds__(kSumThreads) void k_acq_sums(const uint8_t* __restrict__ x,
                                                          const uint32_t* __restrict__ tables,
                                                          const uint32_t* __restrict__ steps, int R,
                                                          int Mc, int rows_pad,
                                                          int8_t* __restrict__ sd) {
    extern __shared__ int32_t s_acc[];  // [R][2][kSumThreads]
    __shared__ uint32_t s_lut[256];
    const int tid = threadIdx.x;
    const int c = blockIdx.x * kSumThreads + tid;  // chip 0..1023 (1023: padding)
    const int d = blockIdx.y, b = blockIdx.z;
    for (int i = tid; i < 256; i += kSumThreads) s_lut[i] = tables[kTabLut + i];
    for (int r = 0; r < 2 * R; ++r) s_acc[r * kSumThreads + tid] = 0;
    __syncthreads();
    const uint32_t step = steps[d];
    const int64_t L = (int64_t)Mc * kCodeLen * R;
    const uint64_t g0 = (uint64_t)b * (uint64_t)L;
    // wiped-off sample at block index i, taken modulo the block length
    auto w = [&](int64_t i, int& wi, int& wq) {
        if (i < 0) i += L;
        else if (i >= L) i -= L;
        const uint64_t gi = g0 + (uint64_t)i;
        int xi, xq, cc, ss;
        load_sample<FMT>(x, gi, xi, xq);
        lut_cs(s_lut[((uint32_t)gi * step) >> 24], cc, ss);
        wipe<FMT>(xi, xq, cc, ss, wi, wq);
    };
    if (c < kCodeLen) {
        for (int m = 0; m < Mc; ++m) {
            const int64_t base = ((int64_t)c + (int64_t)kCodeLen * m) * R;
            int si = 0, sq = 0;
            for (int t = 0; t < R; ++t) {
                int a, q;
                w(base + t, a, q);
                si += a;
                sq += q;
            }
            s_acc[tid] += si;
            s_acc[kSumThreads + tid] += sq;
            // window of r: [base - r, base - r + R)
            for (int r = 1; r < R; ++r) {
                int a, q, e, f;
                w(base - r, a, q);
                w(base - r + R, e, f);
                si += a - e;
                sq += q - f;
                s_acc[(2 * r) * kSumThreads + tid] += si;
                s_acc[(2 * r + 1) * kSumThreads + tid] += sq;
            }
        }
    }
    int8_t* out = sd + (uint64_t)b * rows_pad * kAcqK + c;
    for (int r = 0; r < R; ++r) {
        const int X = d * R + r;
#pragma unroll
        for (int iq = 0; iq < 2; ++iq) {
            const int32_t S = c < kCodeLen ? s_acc[(2 * r + iq) * kSumThreads + tid] : 0;
#pragma unroll
            for (int k = 0; k < ND; ++k) {
                const int8_t dig = k == ND - 1 ? (int8_t)(S >> (7 * k)) : (int8_t)((S >> (7 * k)) & 127);
                out[(uint64_t)acq_row<ND>(X, iq, k) * kAcqK] = dig;
            }
        }
    }
}

// Work item of block L when blocks are dealt to the 8 XCDs in turn (block L
// runs on XCD L mod 8): XCD x takes the x-th contiguous range of items in
// (row tile, PRN, column block) order, so the blocks that read one row tile
// of the operand share an L2.
__device__ __forceinline__ int xcd_item(int L, int G) {
    const int x = L & 7, k = L >> 3;
    int start = 0;
    for (int y = 0; y < x; ++y) start += (G - y + 7) >> 3;
    return start + k;
}

// One block: a tile of 32 NT operand rows against 256 columns of one PRN;
// wave w takes columns 64 w .. 64 w + 63 of all the tile's rows (NT x 2
// MFMA blocks).  Row chunks (128 rows x 128 chips) are staged through two LDS
// buffers with the next chunk's global loads in flight during the current
// chunk's MFMAs.
template <int ND, int NT>
__global__ __launch_bounds__(256) void k_acq_corr(const int8_t* __restrict__ sd,
                                                  const int8_t* __restrict__ codes,
                                                  uint64_t* __restrict__ pw, int rows_pad, int n_x,
                                                  int n_prn, int knc) {
    __shared__ __align__(16) int8_t s_tab[kAcqTabBytes];
    constexpr int kRows = 32 * NT;  // operand rows of a tile (NT MFMA row blocks)
    __shared__ __align__(16) int8_t s_a[2][kRows * kAcqARow];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l32 = lane & 31, h = lane >> 5;
    constexpr int kColBlocks = kAcqK / kAcqCols;
    const int item = xcd_item(blockIdx.x, gridDim.x);
    const int cb = item % kColBlocks;
    const int p = (item / kColBlocks) % n_prn;
    const int tile = item / (kColBlocks * n_prn);
    const int row0 = tile * kRows;
    const int colw = cb * kAcqCols + 64 * wave;
    {
        // the PRN's 16 byte-shifted code copies (copy a, byte i = chip
        // (i + a) mod 1023), prepared at plan creation: a lane's chips
        // o .. o + 15 are bytes (o & ~15) .. + 15 of copy (o & 15)
        const int4v* src = reinterpret_cast<const int4v*>(codes + (uint64_t)p * kAcqTabBytes);
        int4v* dst = reinterpret_cast<int4v*>(s_tab);
        constexpr int kPieces = kAcqTabBytes / 16, kPer = (kPieces + 255) / 256;
        int4v v[kPer];
#pragma unroll
        for (int e = 0; e < kPer; ++e)
            if (tid + 256 * e < kPieces) v[e] = src[tid + 256 * e];
#pragma unroll
        for (int e = 0; e < kPer; ++e)
            if (tid + 256 * e < kPieces) dst[tid + 256 * e] = v[e];
    }
    constexpr int NP = ND == 2 ? 4 : 2;  // powers per lane per 32x32 block
    constexpr int kChunks = kAcqK / kAcqKc;
    static_assert(kChunks % 2 == 0, "buffer parity follows the chunk index within a block");
    int64_t pacc[NT][2][NP];  // below 2^63 by the plan's bound
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int q = 0; q < NP; ++q) pacc[t][ct][q] = 0;
    // chunk g = b * kChunks + kc of the row tile: kRows rows x 128 bytes,
    // NT 16-byte pieces per thread
    auto load = [&](int gch, int4v* st) {
        const int b = gch / kChunks, kc = (gch % kChunks) * kAcqKc;
        const int8_t* src = sd + ((uint64_t)b * rows_pad + row0) * kAcqK + kc;
#pragma unroll
        for (int e = 0; e < NT; ++e) {
            const int idx = tid + 256 * e;
            st[e] = *reinterpret_cast<const int4v*>(src + (uint64_t)(idx >> 3) * kAcqK + 16 * (idx & 7));
        }
    };
    int4v stage[NT];
    load(0, stage);
    for (int b = 0; b < knc; ++b) {
        int16v acc[NT][2];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[t][ct][e] = 0;
        for (int kq = 0; kq < kChunks; ++kq) {
            const int kc = kq * kAcqKc;
            int8_t* buf = s_a[kq & 1];
#pragma unroll
            for (int e = 0; e < NT; ++e) {
                const int idx = tid + 256 * e;
                *reinterpret_cast<int4v*>(buf + (idx >> 3) * kAcqARow + 16 * (idx & 7)) = stage[e];
            }
            // one barrier per chunk: the buffer written next was last read
            // two chunks ago, before every wave passed this barrier (the
            // first also publishes the code copies)
            __syncthreads();
            const int gnext = b * kChunks + kq + 1;
            if (gnext < knc * kChunks) load(gnext, stage);
#pragma unroll
            for (int ks = 0; ks < kAcqKc / 32; ++ks) {
                int4v bf[2], af[NT];
#pragma unroll
                for (int ct = 0; ct < 2; ++ct) {
                    const int o = kc + 32 * ks + 16 * h + colw + 32 * ct + l32;
                    bf[ct] = *reinterpret_cast<const int4v*>(s_tab + (o & 15) * kAcqTabStride + (o & ~15));
                }
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    af[t] = *reinterpret_cast<const int4v*>(buf + (32 * t + l32) * kAcqARow + 32 * ks + 16 * h);
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int ct = 0; ct < 2; ++ct)
                        acc[t][ct] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[t], bf[ct], acc[t][ct], 0, 0, 0);
            }
        }
        // block done: recombine digits and add |Y|^2.  Element e of a 32x32
        // block holds row 8 (e / 4) + 4 h + e % 4, column l32.
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                for (int q = 0; q < NP; ++q) {
                    if constexpr (ND == 2) {
                        // |Y| <= 1023 * 2^14: int32, and one 32x32+64 multiply-add per square
                        const int32_t yi = acc[t][ct][4 * q] + 128 * acc[t][ct][4 * q + 1];
                        const int32_t yq = acc[t][ct][4 * q + 2] + 128 * acc[t][ct][4 * q + 3];
                        pacc[t][ct][q] += (int64_t)yi * yi + (int64_t)yq * yq;
                    } else {
                        int64_t yi = 0, yq = 0;
#pragma unroll
                        for (int s = 3; s >= 0; --s) {
                            yi = yi * 128 + (int64_t)acc[t][ct][8 * q + s];
                            yq = yq * 128 + (int64_t)acc[t][ct][8 * q + 4 + s];
                        }
                        pacc[t][ct][q] += yi * yi + yq * yq;
                    }
                }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                // two digits: X = (row0 + 32 t + 8 q + 4 h) / 4; four
                // digits: X = (row0 + 32 t) / 8 + 2 q + h
                const int X = ND == 2 ? (row0 + 32 * t + 8 * q + 4 * h) / 4
                                      : (row0 + 32 * t) / 8 + 2 * q + h;
                const int col = colw + 32 * ct + l32;
                if (X < n_x && col < kCodeLen)
                    pw[((uint64_t)p * n_x + X) * kAcqK + col] = (uint64_t)pacc[t][ct][q];
            }
}

// Largest value and lowest index on ties, over a 256-thread block.
__device__ __forceinline__ void block_argmax(uint64_t& v, uint32_t& i, uint64_t* s_v, uint32_t* s_i) {
    const int tid = threadIdx.x;
    s_v[tid] = v;
    s_i[tid] = i;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            const uint64_t v2 = s_v[tid + s];
            const uint32_t i2 = s_i[tid + s];
            if (v2 > s_v[tid] || (v2 == s_v[tid] && i2 < s_i[tid])) {
                s_v[tid] = v2;
                s_i[tid] = i2;
            }
        }
        __syncthreads();
    }
    v = s_v[0];
    i = s_i[0];
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_acq_reduce(const uint64_t* __restrict__ pw, int R, int n_x,
                                                    int n_bins, uint64_t* __restrict__ chipmax,
                                                    uint8_t* __restrict__ chiparg,
                                                    uint64_t* __restrict__ binmax,
                                                    uint32_t* __restrict__ binarg,
                                                    uint64_t* __restrict__ surface) {
    __shared__ uint64_t s_v[256];
    __shared__ uint32_t s_i[256];
    const int d = blockIdx.x, p = blockIdx.y, tid = threadIdx.x;
    const uint64_t pd = (uint64_t)p * n_bins + d;
    uint64_t best = 0;
    uint32_t bj = 0xFFFFFFFFu;
    for (int j = tid; j < kCodeLen; j += 256) {
        const uint64_t* col = pw + ((uint64_t)p * n_x + (uint64_t)d * R) * kAcqK + j;
        uint64_t* srow = surface ? surface + pd * (uint64_t)(kCodeLen * R) + (uint64_t)R * j : nullptr;
        uint64_t m = col[0];
        int arg = 0;
        if (srow) srow[0] = m;
        for (int r = 1; r < R; ++r) {
            const uint64_t v = col[(uint64_t)r * kAcqK];
            if (srow) srow[r] = v;
            if (v > m) {
                m = v;
                arg = r;
            }
        }
        chipmax[pd * kAcqK + j] = m;
        chiparg[pd * kAcqK + j] = (uint8_t)arg;
        if (bj == 0xFFFFFFFFu || m > best) {  // j rises: the first maximum is kept
            best = m;
            bj = (uint32_t)j;
        }
    }
    block_argmax(best, bj, s_v, s_i);
    if (tid == 0) {
        binmax[pd] = best;
        binarg[pd] = bj;
    }
}

__global__ __launch_bounds__(256) void k_acq_detect(const uint64_t* __restrict__ chipmax,
                                                    const uint8_t* __restrict__ chiparg,
                                                    const uint64_t* __restrict__ binmax,
                                                    const uint32_t* __restrict__ binarg,
                                                    const int32_t* __restrict__ prns, int n_bins,
                                                    int R, double f_lo, double f_step,
                                                    double threshold,
                                                    gc_acq_result* __restrict__ out) {
#pragma clang fp contract(off)
    __shared__ uint64_t s_v[256];
    __shared__ uint32_t s_i[256];
    const int p = blockIdx.x, tid = threadIdx.x;
    uint64_t best = 0;
    uint32_t bd = 0xFFFFFFFFu;
    for (int d = tid; d < n_bins; d += 256) {
        const uint64_t v = binmax[(uint64_t)p * n_bins + d];
        if (bd == 0xFFFFFFFFu || v > best) {
            best = v;
            bd = (uint32_t)d;
        }
    }
    block_argmax(best, bd, s_v, s_i);
    const uint64_t pd = (uint64_t)p * n_bins + bd;
    const int js = (int)binarg[pd];
    uint64_t second = 0;
    uint32_t dummy = 0;
    for (int j = tid; j < kCodeLen; j += 256) {
        int e = j - js;
        if (e < 0) e += kCodeLen;
        const int dist = min(e, kCodeLen - e);
        if (dist >= 2) second = max(second, chipmax[pd * kAcqK + j]);
    }
    block_argmax(second, dummy, s_v, s_i);
    if (tid == 0) {
        const int tau = R * js + (int)chiparg[pd * kAcqK + js];
        gc_acq_result r;
        r.prn = prns[p];
        r.bin = (int32_t)bd;
        r.tau = tau;
        r.peak = best;
        r.second = second;
        r.doppler_hz = f_lo + (double)bd * f_step;
        r.code_phase_chips = (double)tau / (double)R;
        r.metric = second > 0 ? (double)best / (double)second : __builtin_inf();
        r.acquired = r.metric >= threshold ? 1 : 0;
        out[p] = r;
    }
}

// The 16 byte-shifted copies of each searched PRN's code (copy a, byte i =
// chip (i + a) mod 1023 as int8 +-1), from the context's sign table.
__global__ void k_acq_codes(const uint32_t* __restrict__ tables, const int32_t* __restrict__ prns,
                            int8_t* __restrict__ tabs) {
    const int p = blockIdx.x;
    const uint32_t* sign = tables + kTabSign + (uint64_t)(prns[p] - 1) * kSignLen;
    for (int idx = threadIdx.x; idx < kAcqTabBytes; idx += blockDim.x) {
        const int a = idx / kAcqTabStride, i = idx - a * kAcqTabStride;
        tabs[(uint64_t)p * kAcqTabBytes + idx] = (int8_t)(int16_t)(sign[(i + a) % kCodeLen] & 0xFFFF);
    }
}

template <int FMT, int ND>
hipError_t launch_sums(const gc_acq* a, const void* samples, hipStream_t s) {
    hipLaunchKernelGGL((k_acq_sums<FMT, ND>), dim3(kAcqK / kSumThreads, a->n_bins, a->Knc),
                       dim3(kSumThreads), (size_t)a->R * 2 * kSumThreads * sizeof(int32_t), s, (const uint8_t*)samples,
                       a->ctx->d_tables, a->d_steps, a->R, a->Mc, a->rows_pad, a->d_sd);
    return hipGetLastError();
}

template <int ND, int NT>
hipError_t launch_corr(const gc_acq* a, hipStream_t s) {
    const int n_items = a->rows_pad / (32 * NT) * (kAcqK / kAcqCols) * a->n_prn;
    hipLaunchKernelGGL((k_acq_corr<ND, NT>), dim3(n_items), dim3(256), 0, s, a->d_sd, a->d_codes,
                       a->d_pw, a->rows_pad, a->n_x, a->n_prn, a->Knc);
    return hipGetLastError();
}

template <int ND>
hipError_t launch_acq_nd(const gc_acq* a, const void* samples, hipStream_t s, hipEvent_t* ev) {
    hipError_t e;
    switch (a->fmt) {
        case GC_I8_REAL: e = launch_sums<GC_I8_REAL, ND>(a, samples, s); break;
        case GC_I8_IQ: e = launch_sums<GC_I8_IQ, ND>(a, samples, s); break;
        default: e = launch_sums<GC_I2_REAL, ND>(a, samples, s); break;
    }
    if (e == hipSuccess && ev) e = hipEventRecord(ev[1], s);
    if (e != hipSuccess) return e;
    return a->nt == 3 ? launch_corr<ND, 3>(a, s) : launch_corr<ND, 4>(a, s);
}

}  // namespace

}  // namespace gc

using namespace gc;

extern "C" {

gc_status gc_acq_create(gc_ctx* ctx, gc_format fmt, int32_t samples_per_chip, double if_hz,
                        double f_lo_hz, double f_step_hz, int32_t n_bins, const int32_t* prns,
                        int32_t n_prn, int32_t coherent_periods, int32_t blocks, gc_acq** out) {
    if (!ctx || !prns || !out) return GC_EINVAL;
    *out = nullptr;
    const int R = samples_per_chip, Mc = coherent_periods, Knc = blocks;
    if (fmt != GC_I8_REAL && fmt != GC_I8_IQ && fmt != GC_I2_REAL) return GC_EINVAL;
    if (R < 1 || R > GC_ACQ_MAX_SPC || n_bins < 1 || n_bins > GC_ACQ_MAX_BINS || n_prn < 1 ||
        n_prn > GC_ACQ_MAX_PRNS || Mc < 1 || Mc > 1000 || Knc < 1 || Knc > 1000)
        return GC_EINVAL;
    if (!isfinite(if_hz) || !isfinite(f_lo_hz) || !isfinite(f_step_hz)) return GC_EINVAL;
    for (int i = 0; i < n_prn; ++i)
        if (prns[i] < 1 || prns[i] > 32) return GC_EINVAL;
    // bounds: box sums in int8 digits, and the summed power in uint64
    const double maxw = fmt == GC_I2_REAL ? 3.0 * GC_LUT_AMP
                        : fmt == GC_I8_REAL ? 128.0 * GC_LUT_AMP
                                            : 128.0 * kLutAbsSumMax;
    const double smax = (double)Mc * R * maxw;
    int nd;
    if (smax <= 16383.0) nd = 2;
    else if (smax < 268435456.0) nd = 4;
    else return GC_EINVAL;
    const double ymax = (double)Mc * kCodeLen * R * maxw;
    if (2.0 * ymax * ymax * (double)Knc >= 9.0e18) return GC_EINVAL;  // power sums below 2^63

    DeviceGuard g(ctx->device);
    if (!g.ok) return GC_EDEVICE;
    gc_acq* a = new gc_acq();
    a->device = ctx->device;
    a->ctx = ctx;
    a->fmt = fmt;
    a->R = R;
    a->n_bins = n_bins;
    a->n_prn = n_prn;
    a->Mc = Mc;
    a->Knc = Knc;
    a->nd = nd;
    a->f_lo = f_lo_hz;
    a->f_step = f_step_hz;
    a->n_x = n_bins * R;
    const int rows = nd == 2 ? 4 * a->n_x : 16 * ((a->n_x + 1) / 2);
    // row tile of 96 or 128 rows: the one with fewer tile-rows in its last
    // round of blocks (two blocks per compute unit run at once)
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess ||
        cus < 1)
        cus = 256;
    int64_t best = -1;
    for (int nt = 4; nt >= 3; --nt) {
        const int64_t tiles = (rows + 32 * nt - 1) / (32 * nt);
        const int64_t items = tiles * (kAcqK / kAcqCols) * n_prn;
        const int64_t cost = (items + 2 * cus - 1) / (2 * cus) * nt;
        if (best < 0 || cost < best) {
            best = cost;
            a->nt = nt;
        }
    }
    a->rows_pad = (rows + 32 * a->nt - 1) / (32 * a->nt) * (32 * a->nt);

    std::vector<uint32_t> steps((size_t)n_bins);
    const double fs = (double)R * 1.023e6;
    for (int d = 0; d < n_bins; ++d) {
        const double f = if_hz + (f_lo_hz + (double)d * f_step_hz);
        const double cs = nearbyint(f / fs * 4294967296.0);
        if (!(fabs(cs) < 9.0e18)) {
            delete a;
            return GC_EINVAL;
        }
        steps[d] = (uint32_t)(uint64_t)(int64_t)cs;
    }
    const uint64_t sd_bytes = (uint64_t)Knc * a->rows_pad * kAcqK;
    const uint64_t pw_bytes = (uint64_t)n_prn * a->n_x * kAcqK * 8;
    const uint64_t pb = (uint64_t)n_prn * n_bins;
    a->scratch = sd_bytes + pw_bytes + pb * kAcqK * 9 + pb * 12 + (uint64_t)n_prn * (kAcqTabBytes + 4) +
                 4ull * n_bins;
    hipError_t e = hipSuccess;
    auto alloc = [&](void** p, uint64_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, bytes);
    };
    alloc((void**)&a->d_sd, sd_bytes);
    alloc((void**)&a->d_codes, (uint64_t)n_prn * kAcqTabBytes);
    alloc((void**)&a->d_steps, 4ull * n_bins);
    alloc((void**)&a->d_prns, 4ull * n_prn);
    alloc((void**)&a->d_pw, pw_bytes);
    alloc((void**)&a->d_chipmax, pb * kAcqK * 8);
    alloc((void**)&a->d_chiparg, pb * kAcqK);
    alloc((void**)&a->d_binmax, pb * 8);
    alloc((void**)&a->d_binarg, pb * 4);
    // padding rows stay zero: k_acq_sums writes only the rows of real (bin, r)
    if (e == hipSuccess) e = hipMemsetAsync(a->d_sd, 0, sd_bytes, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(a->d_steps, steps.data(), 4ull * n_bins, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(a->d_prns, prns, 4ull * n_prn, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_acq_codes, dim3(n_prn), dim3(256), 0, ctx->stream, ctx->d_tables,
                           a->d_prns, a->d_codes);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        gc_acq_destroy(a);
        return from_hip(e);
    }
    *out = a;
    return GC_OK;
}

gc_status gc_acquire(gc_acq* a, const void* samples, uint64_t n_samples, double threshold,
                     uint64_t* surface, gc_acq_result* results, void* stream) {
    if (!a || !samples || !results) return GC_EINVAL;
    const uint64_t need = (uint64_t)a->Knc * a->Mc * kCodeLen * a->R;
    if (n_samples < need) return GC_EINVAL;
    DeviceGuard g(a->device);
    if (!g.ok) return GC_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    const size_t n_slots = a->ev_used.size();
    hipEvent_t* ev = n_slots ? &a->ev[5 * (size_t)(a->calls % n_slots)] : nullptr;
    if (ev) a->ev_used[(size_t)(a->calls % n_slots)] = 1;
    ++a->calls;
    hipError_t e = ev ? hipEventRecord(ev[0], s) : hipSuccess;
    if (e == hipSuccess)
        e = a->nd == 2 ? launch_acq_nd<2>(a, samples, s, ev) : launch_acq_nd<4>(a, samples, s, ev);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[2], s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_acq_reduce, dim3(a->n_bins, a->n_prn), dim3(256), 0, s, a->d_pw, a->R,
                           a->n_x, a->n_bins, a->d_chipmax, a->d_chiparg, a->d_binmax, a->d_binarg,
                           surface);
        e = hipGetLastError();
    }
    if (e == hipSuccess && ev) e = hipEventRecord(ev[3], s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_acq_detect, dim3(a->n_prn), dim3(256), 0, s, a->d_chipmax, a->d_chiparg,
                           a->d_binmax, a->d_binarg, a->d_prns, a->n_bins, a->R, a->f_lo, a->f_step,
                           threshold, results);
        e = hipGetLastError();
    }
    if (e == hipSuccess && ev) e = hipEventRecord(ev[4], s);
    return from_hip(e);
}

gc_status gc_acq_info(gc_acq* a, int32_t* digits, uint64_t* scratch_bytes, uint64_t* samples_needed,
                      int32_t* row_tile) {
    if (!a) return GC_EINVAL;
    if (digits) *digits = a->nd;
    if (row_tile) *row_tile = 32 * a->nt;
    if (scratch_bytes) *scratch_bytes = a->scratch;
    if (samples_needed) *samples_needed = (uint64_t)a->Knc * a->Mc * kCodeLen * a->R;
    return GC_OK;
}

static void acq_drop_timing(gc_acq* a) {
    for (auto e : a->ev) (void)hipEventDestroy(e);
    a->ev.clear();
    a->ev_used.clear();
}

gc_status gc_acq_timing(gc_acq* a, int32_t n_slots) {
    if (!a || n_slots < 0 || n_slots > 4096) return GC_EINVAL;
    DeviceGuard g(a->device);
    if (!g.ok) return GC_EDEVICE;
    acq_drop_timing(a);
    for (int i = 0; i < 5 * n_slots; ++i) {
        hipEvent_t e;
        const hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
        if (r != hipSuccess) {
            acq_drop_timing(a);
            return from_hip(r);
        }
        a->ev.push_back(e);
    }
    a->ev_used.assign((size_t)n_slots, 0);
    a->calls = 0;
    return GC_OK;
}

gc_status gc_acq_kernel_ms(gc_acq* a, int32_t slot, float* ms) {
    if (!a || !ms || slot < 0 || (size_t)slot >= a->ev_used.size() || !a->ev_used[(size_t)slot])
        return GC_EINVAL;
    DeviceGuard g(a->device);
    if (!g.ok) return GC_EDEVICE;
    const hipEvent_t* ev = &a->ev[5 * (size_t)slot];
    hipError_t e = hipEventSynchronize(ev[4]);
    for (int k = 0; k < 4 && e == hipSuccess; ++k) e = hipEventElapsedTime(&ms[k], ev[k], ev[k + 1]);
    return from_hip(e);
}

gc_status gc_acq_destroy(gc_acq* a) {
    if (!a) return GC_EINVAL;
    DeviceGuard g(a->device);
    acq_drop_timing(a);
    void* ptrs[] = {a->d_sd, a->d_codes, a->d_steps, a->d_prns, a->d_pw,
                    a->d_chipmax, a->d_chiparg, a->d_binmax, a->d_binarg};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete a;
    return GC_OK;
}

}  // extern "C"
