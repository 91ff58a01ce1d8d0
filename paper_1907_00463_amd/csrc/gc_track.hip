// gc_track.hip -- closed tracking loops on the device (Table 3): per channel,
// the E/P/L correlation of one dump, then the DLL / PLL / FLL update that
// sets the NCO steps of the next dump.
//
// One block per channel walks the block of samples dump by dump.  For a dump
// the block's threads take its samples with a stride (carrier phase and code
// phase of sample i are phi + i*dphi and p + i*dp), sum the six products in
// int32 (a code step that keeps the window's sums inside int32 is enforced),
// and reduce them with DPP and LDS; thread 0 adds them to the open dump and,
// when the code phase has reached the window end, emits the dump and runs
// the loop update.  The loop update uses a vectoring CORDIC on the integer
// dumps for the angles and only correctly rounded double operations
// (contraction off) elsewhere, so the loop state is reproducible bit for bit.
#include "gc_internal.h"
#include "gc_device.h"

namespace gc {

namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;
constexpr int kStageBytes = 32768;             // LDS sample window per step
constexpr int kStagePieces = kStageBytes / 16;
static_assert(kStagePieces % kThreads == 0, "whole 16-byte pieces per thread");
typedef int int4v __attribute__((ext_vector_type(4)));
typedef short short2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ short2_t as_s2(uint32_t v) { return __builtin_bit_cast(short2_t, v); }
constexpr double kQ30 = 1073741824.0;

__device__ __forceinline__ int64_t iabs64(int64_t v) { return v < 0 ? -v : v; }

// atan2(y, x), x >= 0, in units of 2^-30 rad: scale the vector into
// [2^39, 2^40), then rotate it towards the x axis by -+atan(2^-i).
__device__ __forceinline__ int bitlen64(uint64_t m) { return m ? 64 - __builtin_clzll(m) : 0; }

__device__ int64_t atan2_q30(int64_t y, int64_t x, const int32_t* tab) {
    if (x == 0 && y == 0) return 0;
    const int64_t hi = int64_t(1) << 40;
    // halving while a magnitude is >= 2^40: one shift that cannot overshoot
    // (arithmetic shifts compose), then the last one or two steps
    {
        const uint64_t m = (uint64_t)max(iabs64(x), iabs64(y));
        const int s = bitlen64(m) - 42;
        if (s > 0) {
            x >>= s;
            y >>= s;
        }
        while (iabs64(x) >= hi || iabs64(y) >= hi) {
            x >>= 1;
            y >>= 1;
        }
    }
    // doubling while both magnitudes are below 2^39 is one exact shift
    {
        const uint64_t m = (uint64_t)max(iabs64(x), iabs64(y));
        const int s = 40 - bitlen64(m);
        if (s > 0) {
            x *= int64_t(1) << s;
            y *= int64_t(1) << s;
        }
    }
    // the rotations, branch-free (two lanes run them side by side); the
    // angle sum stays within the sum of the table, below 2^31
    int32_t z = 0;
#pragma unroll
    for (int i = 0; i < kCordicSteps; ++i) {
        const int64_t xs = x >> i, ys = y >> i;
        const bool pos = y > 0;
        const int32_t t = tab[i];
        x = pos ? x + ys : x - ys;
        y = pos ? y - xs : y + xs;
        z = pos ? z + t : z - t;
    }
    return (int64_t)z;
}

__device__ void loop_coef(double B, double z, double k, double& tau1, double& tau2) {
#pragma clang fp contract(off)
    const double wn = B * 8.0 * z / (4.0 * z * z + 1.0);
    tau1 = k / (wn * wn);
    tau2 = 2.0 * z / wn;
}

// Largest |wipe-off| of one sample of the format.
__device__ __forceinline__ uint64_t max_w(int fmt) {
    return fmt == GC_I8_REAL ? 128ull * GC_LUT_AMP
                             : (fmt == GC_I2_REAL ? 3ull * GC_LUT_AMP : 128ull * kLutAbsSumMax);
}

// The code step keeps a window's sums inside int32.
__device__ __forceinline__ bool step_ok(uint64_t dp, uint64_t W, int fmt) {
    if (dp < 1 || dp >= (1ull << 31)) return false;
    return ((W - 1) / dp + 1) * max_w(fmt) < (1ull << 31);
}

// Loop filter coefficients; new carrier and code steps come from
// loop_update, which is false when the code step leaves 1 .. 2^31-1.
struct Coefs {
    double T, t1c, t2c, t1d, t2d;
};

// The vector whose angle (units of 2^-30 rad) is a discriminator of the
// closing dump: which = 0, the PLL's atan(Q / I) of the prompt; which = 1,
// the FLL's angle between the previous and this prompt, the dot product's
// sign removed.  Two lanes form one vector each and then run the same
// CORDIC side by side.
__device__ __forceinline__ void loop_angle_args(int which, int64_t ip, int64_t qp, int32_t prev_i,
                                                int32_t prev_q, int64_t& y, int64_t& x) {
    if (which == 0) {
        y = ip >= 0 ? qp : -qp;
        x = ip >= 0 ? ip : -ip;
        return;
    }
    int64_t i0 = prev_i, q0 = prev_q, i1 = ip, q1 = qp;
    const int64_t lim = int64_t(1) << 30;
    while (iabs64(i0) >= lim || iabs64(q0) >= lim || iabs64(i1) >= lim || iabs64(q1) >= lim) {
        i0 >>= 1;
        q0 >>= 1;
        i1 >>= 1;
        q1 >>= 1;
    }
    const int64_t dot = i0 * i1 + q0 * q1;
    const int64_t cross = i0 * q1 - q0 * i1;
    y = dot >= 0 ? cross : -cross;
    x = dot >= 0 ? dot : -dot;
}

// Loop update at the close of a dump with sums d (E I, E Q, P I, P Q, L I,
// L Q) and the discriminator angles a (PLL) and f (FLL).
__device__ bool loop_update(const TrackConsts& P, const Coefs& K, const int64_t* d, int64_t a,
                            int64_t f, gc_loop_state& L, uint32_t& carr_step,
                            uint64_t& code_step) {
#pragma clang fp contract(off)
    const double T = K.T, t1c = K.t1c, t2c = K.t2c, t1d = K.t1d, t2d = K.t2d;
    const int64_t ie = d[0], qe = d[1], ip = d[2], qp = d[3], il = d[4], ql = d[5];
    // PLL: atan(Q / I) in cycles
    const double carr_err = ((double)a / kQ30) / (2.0 * M_PI);
    // FLL: angle between consecutive prompts, the dot product's sign removed
    if (L.have_prev) {
        const double f_err = ((double)f / kQ30) / (2.0 * M_PI * T);
        L.fll_basis_hz = L.fll_basis_hz + (4.0 * P.fll_bw * T) * f_err;
    }
    L.prompt_i_prev = (int32_t)ip;
    L.prompt_q_prev = (int32_t)qp;
    L.have_prev = 1;
    {
        const double u1 = (t2c / t1c) * (carr_err - L.pll_err_prev);
        const double u2 = carr_err * (T / t1c);
        L.pll_nco_hz = L.pll_nco_hz + (u1 + u2);
        L.pll_err_prev = carr_err;
    }
    L.carr_hz = L.fll_basis_hz + L.pll_nco_hz;
    {
        const double fe = (double)ie, ge = (double)qe, fl = (double)il, gl = (double)ql;
        const double E = __builtin_sqrt(fe * fe + ge * ge), Lm = __builtin_sqrt(fl * fl + gl * gl);
        const double code_err = (E + Lm) > 0.0 ? (E - Lm) / (E + Lm) : 0.0;
        const double u1 = (t2d / t1d) * (code_err - L.dll_err_prev);
        const double u2 = code_err * (T / t1d);
        L.dll_nco_cps = L.dll_nco_cps + (u1 + u2);
        L.dll_err_prev = code_err;
    }
    L.code_cps = 1.023e6 * (1.0 + (L.carr_hz - P.if_hz) / 1575.42e6) + L.dll_nco_cps;
    const double cs = __builtin_rint(L.carr_hz / P.fs * 4294967296.0);
    carr_step = (uint32_t)(uint64_t)(int64_t)cs;
    const double ks = __builtin_rint(L.code_cps / P.fs * 4294967296.0);
    if (!(ks >= 1.0) || !(ks < 2147483648.0)) return false;
    code_step = (uint64_t)ks;
    return true;
}



// Orders the LDS accesses of one wave's lanes around this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// What every wave needs of a step: the phases and steps at its first
// sample, its sample count, and whether the walk is over.
struct StepCtl {
    uint64_t p, dp, s;
    uint32_t phi, dphi, take;
    int32_t status, done;
};

// ceil(num / d) for num < 2^53, d >= 1: a double estimate made exact.
__device__ __forceinline__ uint64_t ceil_div53(uint64_t num, uint64_t d) {
    uint64_t q = (uint64_t)((double)num / (double)d);
    while (q * d < num) ++q;
    while (q > 0 && (q - 1) * d >= num) --q;
    return q;
}

template <int FMT>
__global__ __launch_bounds__(kThreads) void k_track(const uint8_t* __restrict__ samples,
                                                    uint64_t n, const DevChan* __restrict__ chans,
                                                    gc_chan_state* __restrict__ states,
                                                    gc_loop_state* __restrict__ loops,
                                                    TrackConsts P, int32_t* __restrict__ rows,
                                                    uint32_t* __restrict__ dump_n,
                                                    uint32_t* __restrict__ n_dumps,
                                                    int32_t* __restrict__ status,
                                                    uint32_t max_dumps,
                                                    const uint32_t* __restrict__ tables) {
    __shared__ uint32_t s_lut[256];
    __shared__ uint32_t s_code3[kCodeLen];  // chip c: bytes C[c-1], C[c], C[c+1]
    __shared__ int32_t s_cordic[kCordicSteps];  // round(atan(2^-i) 2^30), all below 2^30
    // 2-bit: (c, -s) int16 pairs of the carrier table, and per chip the
    // sign pairs (C, C) of chips c - 1, c, c + 1
    __shared__ uint32_t s_lut2[FMT == GC_I2_REAL ? 256 : 1];
    // 2-bit: entry 2 c + u for chip c and half u of the chip: the (L, E, P)
    // sign pairs, u = 0 (first half) (C[c-1], C[c], C[c]), u = 1 (second
    // half) (C[c], C[c+1], C[c])
    __shared__ uint4 s_codeh[FMT == GC_I2_REAL ? 2 * kCodeLen : 1];
    __shared__ int32_t s_red[6][kWaves];
    __shared__ StepCtl sc;
    __shared__ gc_loop_state s_loop;  // the loop state and filter coefficients, read and
    __shared__ Coefs s_coef;          // written by wave 0 at each dump close
    __shared__ __align__(16) uint8_t s_stage[kStageBytes];
    const int tid = threadIdx.x;
    const int chn = blockIdx.x;
    const DevChan& ch = chans[chn];
    for (int i = tid; i < 256; i += kThreads) s_lut[i] = tables[kTabLut + i];
    if (tid < kCordicSteps) s_cordic[tid] = (int32_t)P.tab[tid];
    const uint32_t* sgn = tables + kTabSign + (ch.prn - 1) * kSignLen;
    for (int i = tid; i < kCodeLen; i += kThreads) {
        const int im = i == 0 ? kCodeLen - 1 : i - 1, ip = i + 1 == kCodeLen ? 0 : i + 1;
        s_code3[i] = (sgn[im] & 0xFFu) | (sgn[i] & 0xFFu) << 8 | (sgn[ip] & 0xFFu) << 16;
        if constexpr (FMT == GC_I2_REAL) {
            s_codeh[2 * i] = uint4{sgn[im], sgn[i], sgn[i], 0u};
            s_codeh[2 * i + 1] = uint4{sgn[i], sgn[ip], sgn[i], 0u};
        }
    }
    if constexpr (FMT == GC_I2_REAL) {
        for (int i = tid; i < 256; i += kThreads) {
            const uint32_t e = tables[kTabLut + i];
            const uint32_t c = e & 0xFFFFu, sn = e >> 16;
            s_lut2[i] = c | ((uint32_t)(uint16_t)(-(int16_t)sn) << 16);
        }
    }
    const uint64_t W = ch.window;
    gc_chan_state* st = states + chn;
    // The control state lives in wave 0's registers, the same in every lane
    // of the wave: the lanes run the dump close together (the loop update
    // redundantly, on equal inputs), so no control value makes an LDS round
    // trip.  The other waves see each step's phases, steps and sample count
    // in `sc`, written by lane 0 before the step's barrier.
    const bool w0 = tid < 64;
    int64_t acc[6] = {0, 0, 0, 0, 0, 0};
    uint64_t p = 0, dp = 0, s = 0;
    uint32_t phi = 0, dphi = 0, acc_n = 0, nd = 0;
    int32_t status_w = GC_OK;
    int32_t prev_i = 0, prev_q = 0, have_prev = 0;
    // samples whose bytes fit a window from any start (at most 15 bytes of
    // alignment before the first)
    constexpr uint32_t kStageSamples = FMT == GC_I2_REAL ? 4 * (kStageBytes - 17)
                                       : FMT == GC_I8_IQ ? (kStageBytes - 16) / 2
                                                         : kStageBytes - 16;
    // samples of the next step: up to the window end, the block end or the
    // stage size
    auto step_take = [&]() -> uint32_t {
        const uint64_t need = ceil_div53(W - p, dp);     // samples until the phase reaches W
        return (uint32_t)min(min(need, n - s), (uint64_t)kStageSamples);
    };
    if (w0) {
        if (tid == 0) {
            Coefs K;
            K.T = (double)ch.int_periods * 1e-3;
            loop_coef(P.pll_bw, P.pll_zeta, P.pll_k, K.t1c, K.t2c);
            loop_coef(P.dll_bw, P.dll_zeta, P.dll_k, K.t1d, K.t2d);
            s_coef = K;
        }
        p = st->code_phase;
        dp = st->code_step;
        phi = st->carr_phase;
        dphi = st->carr_step;
        acc_n = st->acc_n;
        if (ch.n_taps != 3 || !ch.epl || p >= W) {
            status_w = GC_EINVAL;
        } else if (!step_ok(dp, W, FMT)) {
            status_w = GC_ERANGE;
        } else {
            const int sl[3] = {ch.slot_e, ch.slot_p, ch.slot_l};
            for (int k = 0; k < 3; ++k) {
                acc[2 * k] = st->acc[sl[k]][0];
                acc[2 * k + 1] = st->acc[sl[k]][1];
            }
            const gc_loop_state L = loops[chn];
            if (tid == 0) s_loop = L;
            prev_i = L.prompt_i_prev;
            prev_q = L.prompt_q_prev;
            have_prev = L.have_prev;
        }
        const uint32_t take0 = status_w == GC_OK ? step_take() : 0u;
        if (tid == 0) {
            sc.p = p;
            sc.dp = dp;
            sc.s = s;
            sc.phi = phi;
            sc.dphi = dphi;
            sc.take = take0;
            sc.status = status_w;
            sc.done = status_w != GC_OK;
        }
    }
    __syncthreads();
    if (sc.status != GC_OK) {
        if (tid == 0) {
            status[chn] = sc.status;
            n_dumps[chn] = 0;
        }
        return;
    }
    // The samples pass through LDS in windows of kStageBytes bytes that start
    // at the 16-byte boundary below the first sample of a step.  The window
    // of the next step (which starts where this one ends) is loaded into
    // registers while this step is summed, and stored to LDS once every wave
    // is past this step's sums, while wave 0 closes the step.
    const uint64_t nbytes = FMT == GC_I2_REAL ? (n + 3) / 4 : FMT == GC_I8_IQ ? 2 * n : n;
    auto byte_of = [](uint64_t smp) -> uint64_t {
        return FMT == GC_I2_REAL ? smp >> 2 : FMT == GC_I8_IQ ? 2 * smp : smp;
    };
    int4v pf[kStagePieces / kThreads];
    // A window wholly inside the block is plain 16-byte loads, left in
    // flight until the window is stored (a per-piece choice between these
    // and the byte-wise tail made every load wait at once); only the last
    // window of a block takes the per-piece path.
    auto load_window = [&](uint64_t first) {
        const uint64_t b0 = byte_of(first) & ~(uint64_t)15;
        if (b0 + kStageBytes <= nbytes) {
#pragma unroll
            for (int e = 0; e < kStagePieces / kThreads; ++e)
                pf[e] = *reinterpret_cast<const int4v*>(samples + b0 + 16 * (uint64_t)(tid + kThreads * e));
            return;
        }
#pragma unroll
        for (int e = 0; e < kStagePieces / kThreads; ++e) {
            const uint64_t b = b0 + 16 * (uint64_t)(tid + kThreads * e);
            if (b + 16 <= nbytes) {
                pf[e] = *reinterpret_cast<const int4v*>(samples + b);
            } else {
                uint32_t w[4] = {0, 0, 0, 0};
                for (int k = 0; k < 16 && b + k < nbytes; ++k) w[k >> 2] |= (uint32_t)samples[b + k] << (8 * (k & 3));
                pf[e] = int4v{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
            }
        }
    };
    auto readlane64 = [](int64_t v, int l) -> int64_t {
        const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
        const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
        return (int64_t)(((uint64_t)hi << 32) | lo);
    };
    auto store_window = [&]() {
#pragma unroll
        for (int e = 0; e < kStagePieces / kThreads; ++e)
            reinterpret_cast<int4v*>(s_stage)[tid + kThreads * e] = pf[e];
    };
    load_window(0);
    store_window();
    __syncthreads();
    while (true) {
        const uint64_t p0 = sc.p, dp0 = sc.dp, s0 = sc.s;
        const uint32_t phi0 = sc.phi, dphi0 = sc.dphi, take = sc.take;
        load_window(s0 + take);
        const uint64_t b0 = byte_of(s0) & ~(uint64_t)15;
        int32_t a[6] = {0, 0, 0, 0, 0, 0};
        // this thread's samples i = tid + kThreads k: offsets, carrier and
        // code phases advance by fixed amounts from one to the next
        uint32_t off = (uint32_t)(byte_of(s0 + tid) - b0);
        const uint32_t sh2 = 2u * (uint32_t)((s0 + tid) & 3);   // 2-bit: bit offset in the byte
        uint32_t ph = phi0 + (uint32_t)tid * dphi0;
        uint64_t u = p0 + (uint64_t)tid * dp0;
        const uint32_t dph = (uint32_t)kThreads * dphi0;
        const uint64_t du = (uint64_t)kThreads * dp0;
        constexpr uint32_t doff = FMT == GC_I2_REAL ? kThreads / 4 : FMT == GC_I8_IQ ? 2 * kThreads : kThreads;
        if constexpr (FMT == GC_I2_REAL) {
            // 2-bit samples: x as an (x, x) int16 pair, (wI, wQ) = x (c, -s)
            // in one packed multiply, then E, P and L by packed
            // multiply-adds with the sign pairs of the sample's half-chip.
            // The code phase is kept as its fraction and its chip mod 1023:
            // a thread's phase advances by du = kThreads dp < 2^41 per
            // sample, so the chip moves by under 512 (plus the fraction's
            // carry) and one conditional subtract keeps it below 1023.  A
            // thread's partial sums stay below
            // (kStageSamples / kThreads) * 72 < 2^15.
            short2_t sE = {0, 0}, sP = {0, 0}, sL = {0, 0};
            uint32_t uf = (uint32_t)u;
            uint32_t cp = (uint32_t)((u >> 32) % kCodeLen);
            const uint32_t dfr = (uint32_t)du, dch = (uint32_t)(du >> 32);
            auto one = [&]() {
                const uint32_t v = __builtin_amdgcn_ubfe((uint32_t)s_stage[off], sh2, 2u);
                const uint32_t x16 = (2u * v + 0xFFFDu) & 0xFFFFu;  // 2 v - 3 in the low half
                const short2_t w2 = as_s2(x16 * 0x10001u) * as_s2(s_lut2[ph >> 24]);
                const uint4 c = s_codeh[2 * cp + (uf >> 31)];
                sE = w2 * as_s2(c.y) + sE;
                sP = w2 * as_s2(c.z) + sP;
                sL = w2 * as_s2(c.x) + sL;
                const uint32_t nf = uf + dfr;
                cp += dch + (nf < uf ? 1u : 0u);
                uf = nf;
                cp = min(cp, cp - (uint32_t)kCodeLen);
                off += doff;
                ph += dph;
            };
            // passes in which every thread has a sample run on a uniform
            // count; the last, partial pass is guarded per thread
            const uint32_t nfull = (uint32_t)take / kThreads;
            for (uint32_t k = 0; k < nfull; ++k) one();
            if ((uint32_t)tid < (uint32_t)take - nfull * kThreads) one();
            a[0] = sE.x;
            a[1] = sE.y;
            a[2] = sP.x;
            a[3] = sP.y;
            a[4] = sL.x;
            a[5] = sL.y;
        } else {
            // int8 samples: the same pass split, and the chip carried as in
            // the 2-bit loop
            uint32_t uf = (uint32_t)u;
            uint32_t cp = (uint32_t)((u >> 32) % kCodeLen);
            const uint32_t dfr = (uint32_t)du, dch = (uint32_t)(du >> 32);
            auto one = [&]() {
                int xi, xq;
                if constexpr (FMT == GC_I8_IQ) {
                    xi = (int)(int8_t)s_stage[off];
                    xq = (int)(int8_t)s_stage[off + 1];
                } else {
                    xi = (int)(int8_t)s_stage[off];
                    xq = 0;
                }
                int c, sn;
                lut_cs(s_lut[ph >> 24], c, sn);
                int wi, wq;
                wipe<FMT>(xi, xq, c, sn, wi, wq);
                // prompt chip floor(u / 2^32) mod 1023; the early (late) chip
                // is the next (previous) one when u's fraction is at or above
                // (below) one half chip
                const int sh = uf >= (1u << 31) ? 8 : 0;
                const uint32_t c3 = s_code3[cp];
                const int re = (int)(int8_t)(c3 >> (8 + sh));
                const int rp = (int)(int8_t)(c3 >> 8);
                const int rl = (int)(int8_t)(c3 >> sh);
                a[0] += wi * re;
                a[1] += wq * re;
                a[2] += wi * rp;
                a[3] += wq * rp;
                a[4] += wi * rl;
                a[5] += wq * rl;
                const uint32_t nf = uf + dfr;
                cp += dch + (nf < uf ? 1u : 0u);
                uf = nf;
                cp = min(cp, cp - (uint32_t)kCodeLen);
                off += doff;
                ph += dph;
            };
            const uint32_t nfull = (uint32_t)take / kThreads;
            for (uint32_t k = 0; k < nfull; ++k) one();
            if ((uint32_t)tid < (uint32_t)take - nfull * kThreads) one();
        }
        {  // the wave's six sums land in lanes 0-5, one store
            const int t = wave_total6(a);
            if ((tid & 63) < 6) s_red[tid & 63][tid >> 6] = t;
        }
        __syncthreads();
        if (!w0) store_window();  // every wave is done with this step's window
        if (w0) {  // wave 0 closes the step
            int64_t t = 0;  // the six sums in parallel, one lane each
            if (tid < 6) {
#pragma unroll
                for (int w = 0; w < kWaves; ++w) t += s_red[tid][w];
            }
            store_window();  // after the sums' reads, ahead of the close
#pragma unroll
            for (int k = 0; k < 6; ++k) acc[k] += readlane64(t, k);
            acc_n += take;
            phi = phi0 + take * dphi0;
            p = p0 + (uint64_t)take * dp0;
            s = s0 + take;
            const bool closes = p >= W && nd < max_dumps;
            if (p >= W && nd >= max_dumps) status_w = GC_ENOSPC;
            if (closes) {  // the dump closes: both angles side by side, then the update
                int64_t ang = 0;
                if (tid < 2 && (tid == 0 || have_prev)) {
                    int64_t y, x;
                    loop_angle_args((int)tid, acc[2], acc[3], prev_i, prev_q, y, x);
                    ang = atan2_q30(y, x, s_cordic);
                }
                const int64_t a_pll = readlane64(ang, 0), a_fll = readlane64(ang, 1);
                if (tid < 8) {  // the row: six sums, then the NCO steps of the dump
                    int32_t v = (int32_t)(uint32_t)dp;
                    v = tid == 6 ? (int32_t)dphi : v;
#pragma unroll
                    for (int k = 0; k < 6; ++k) v = tid == (uint32_t)k ? (int32_t)acc[k] : v;
                    rows[((uint64_t)chn * max_dumps + nd) * 8 + tid] = v;
                }
                if (tid == 0) dump_n[(uint64_t)chn * max_dumps + nd] = acc_n;
                nd += 1;
                uint32_t ncs;
                uint64_t nks;
                gc_loop_state L = s_loop;
                const Coefs K = s_coef;
                const bool ok = loop_update(P, K, acc, a_pll, a_fll, L, ncs, nks);
                if (tid == 0) s_loop = L;
                if (!ok || !step_ok(nks, W, FMT)) {
                    status_w = GC_ERANGE;
                } else {
                    dphi = ncs;
                    dp = nks;
                }
                prev_i = L.prompt_i_prev;
                prev_q = L.prompt_q_prev;
                have_prev = L.have_prev;
#pragma unroll
                for (int k = 0; k < 6; ++k) acc[k] = 0;
                acc_n = 0;
                p -= W;
            }
            const bool done = status_w != GC_OK || (s >= n && p < W);
            const uint32_t take_n = done ? 0u : step_take();
            if (tid == 0) {
                sc.p = p;
                sc.dp = dp;
                sc.s = s;
                sc.phi = phi;
                sc.dphi = dphi;
                sc.take = take_n;
                sc.status = status_w;
                sc.done = done;
            }
        }
        __syncthreads();
        if (sc.done) break;
    }
    if (tid == 0) {
        status[chn] = status_w;
        if (status_w == GC_OK) {
            n_dumps[chn] = nd;
            st->code_phase = p;
            st->code_step = dp;
            st->carr_phase = phi;
            st->carr_step = dphi;
            st->acc_n = acc_n;
            const int sl[3] = {ch.slot_e, ch.slot_p, ch.slot_l};
            for (int k = 0; k < 3; ++k) {
                st->acc[sl[k]][0] = (int32_t)acc[2 * k];
                st->acc[sl[k]][1] = (int32_t)acc[2 * k + 1];
            }
            loops[chn] = s_loop;
        } else {
            n_dumps[chn] = 0;
        }
    }
}

// Lock metrics and bit synchronisation of channel blockIdx.x over its
// closed dumps: prompt I and Q of dump k at rows[(ch * max_dumps + k) *
// stride + col] and [... + col + 1].  One thread per window (C/N0 by the
// moments estimator, lock ratio), per bit-period start (navigation bits),
// and a block-wide histogram of prompt sign changes.
__global__ __launch_bounds__(256) void k_lock_metrics(
    const int32_t* __restrict__ rows, int stride, int col, const uint32_t* __restrict__ n_dumps,
    uint32_t max_dumps, uint32_t K, double T, double lock_min,
    const uint32_t* __restrict__ phase, double* __restrict__ cn0, double* __restrict__ lock,
    uint32_t max_windows, uint32_t* __restrict__ n_windows, uint32_t* __restrict__ lock_fails,
    uint32_t* __restrict__ hist, uint32_t* __restrict__ edge, uint8_t* __restrict__ bits,
    uint32_t max_bits, uint32_t* __restrict__ n_bits) {
#pragma clang fp contract(off)
    __shared__ uint32_t s_hist[20];
    __shared__ uint32_t s_fails;
    __shared__ uint32_t s_edge;
    const int ch = blockIdx.x, tid = threadIdx.x;
    const uint32_t n = min(n_dumps[ch], max_dumps);
    const int32_t* r = rows + (uint64_t)ch * max_dumps * stride + col;
    const uint32_t ph = phase ? phase[ch] % 20 : 0;
    if (tid < 20) s_hist[tid] = 0;
    if (tid == 0) s_fails = 0;
    __syncthreads();
    const uint32_t nw = n / K;
    for (uint32_t w = tid; w < nw; w += blockDim.x) {
        double m2 = 0.0, m4 = 0.0, ii = 0.0, qq = 0.0;
        for (uint32_t k = w * K; k < (w + 1) * K; ++k) {
            const double i = (double)r[(uint64_t)k * stride], q = (double)r[(uint64_t)k * stride + 1];
            const double p = i * i + q * q;
            m2 += p;
            m4 += p * p;
            ii += i * i;
            qq += q * q;
        }
        m2 = m2 / (double)K;
        m4 = m4 / (double)K;
        const double d = 2.0 * m2 * m2 - m4;
        double c = __builtin_nan("");
        if (d > 0.0) {
            const double a = __builtin_sqrt(d);
            if (m2 - a > 0.0) c = 10.0 * log10((a / (m2 - a)) / T);
        }
        const double ratio = (ii + qq) > 0.0 ? (ii - qq) / (ii + qq) : 0.0;
        if (w < max_windows) {
            cn0[(uint64_t)ch * max_windows + w] = c;
            lock[(uint64_t)ch * max_windows + w] = ratio;
        }
        if (ratio < lock_min) atomicAdd(&s_fails, 1u);
    }
    for (uint32_t k = 1 + tid; k < n; k += blockDim.x) {
        const bool a = r[(uint64_t)(k - 1) * stride] < 0, b = r[(uint64_t)k * stride] < 0;
        if (a != b) atomicAdd(&s_hist[(k + ph) % 20], 1u);
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t e = 0;
        for (uint32_t j = 1; j < 20; ++j)
            if (s_hist[j] > s_hist[e]) e = j;
        s_edge = e;
        for (int j = 0; j < 20; ++j) hist[ch * 20 + j] = s_hist[j];
        edge[ch] = e;
        n_windows[ch] = min(nw, max_windows);
        lock_fails[ch] = s_fails;
    }
    __syncthreads();
    const uint32_t k0 = (s_edge + 20 - ph) % 20;
    const uint32_t nb = n >= k0 + 20 ? (n - k0) / 20 : 0;
    for (uint32_t j = tid; j < nb && j < max_bits; j += blockDim.x) {
        int64_t sum = 0;
        for (uint32_t t = 0; t < 20; ++t) sum += r[(uint64_t)(k0 + 20 * j + t) * stride];
        bits[(uint64_t)ch * max_bits + j] = (uint8_t)(sum < 0);
    }
    if (tid == 0) n_bits[ch] = min(nb, max_bits);
}

}  // namespace

hipError_t launch_lock_metrics(const int32_t* rows, int stride, int col, const uint32_t* n_dumps,
                               int n_chan, uint32_t max_dumps, uint32_t K, double T,
                               double lock_min, const uint32_t* phase, double* cn0, double* lock,
                               uint32_t max_windows, uint32_t* n_windows, uint32_t* lock_fails,
                               uint32_t* hist, uint32_t* edge, uint8_t* bits, uint32_t max_bits,
                               uint32_t* n_bits, hipStream_t s) {
    hipLaunchKernelGGL(k_lock_metrics, dim3(n_chan), dim3(256), 0, s, rows, stride, col, n_dumps,
                       max_dumps, K, T, lock_min, phase, cn0, lock, max_windows, n_windows,
                       lock_fails, hist, edge, bits, max_bits, n_bits);
    return hipGetLastError();
}

hipError_t launch_track(const uint8_t* samples, uint64_t n, int fmt, const DevChan* chans,
                        gc_chan_state* state, gc_loop_state* loop, const TrackConsts& consts,
                        int n_chan, int32_t* rows, uint32_t* dump_n, uint32_t* n_dumps,
                        int32_t* status, uint32_t max_dumps, const uint32_t* tables,
                        hipStream_t s) {
#define GC_T(F)                                                                             \
    hipLaunchKernelGGL((k_track<F>), dim3(n_chan), dim3(kThreads), 0, s, samples, n, chans, \
                       state, loop, consts, rows, dump_n, n_dumps, status, max_dumps, tables)
    if (fmt == GC_I8_REAL) GC_T(GC_I8_REAL);
    else if (fmt == GC_I8_IQ) GC_T(GC_I8_IQ);
    else if (fmt == GC_I2_REAL) GC_T(GC_I2_REAL);
    else return hipErrorInvalidValue;
#undef GC_T
    return hipGetLastError();
}

}  // namespace gc
