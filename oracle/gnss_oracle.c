/*
 * gnss_oracle.c -- plain, slow, obviously-correct CPU oracle for the GPS L1 C/A
 * software-correlator hot path (carrier wipe-off, code replica, per-tap
 * multiply-accumulate, code-epoch-aligned dumps).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no code,
 * header, table or constant with the HIP path: the Gold-code construction,
 * sin/cos table, NCO word conversion and correlation loop below are written
 * independently from the definitions they cite.
 *
 * What the paper fixes (Schmidt & Akopian, "Exploiting Acceleration Features
 * of LabVIEW platform for Real-Time GNSS Software Receiver Optimization"):
 *   - the C/A signal model, Eq. (1): the C/A code rides the in-phase carrier;
 *   - C/A code facts, Sec. 3.1: 1023 chips of +-1 at 1.023 Mcps, 1 ms period,
 *     one code per satellite 1..32, 50 bps navigation data (20 code periods);
 *   - synchronisation by code-phase alignment plus carrier wipe-off, Sec. 3.1;
 *   - early-late spacing of 1/2 chip, Table 3; 1 ms integrations, Sec. 4.
 * The paper gives none of the correlator arithmetic; the readings used here
 * (LUT size and amplitude, NCO word sizes, wipe-off sign, dump alignment,
 * 2-bit coding, chip-to-sign mapping) are stated at each function below.
 * The Gold-code generator polynomials and per-PRN G2 phase-selector taps
 * come from IS-GPS-200, Sec. 3.2.1.3 and Table 3-Ia.
 *
 * Parity pins: every function here is pinned by -m "not gpu" tests against
 * values that do not come from this file (IS-GPS-200 first-ten-chip octal
 * words, Gold-family correlation values, closed-form correlations of
 * noiseless signals, a hand formula for the fs/4 carrier, brute force).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_CODE_LEN 1023
#define ORC_LUT_SIZE 256
#define ORC_LUT_AMP 24.0
#define ORC_TWO32 4294967296.0

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ERANGE = -4, ORC_ENOSPC = -7 };
enum { ORC_I8_REAL = 0, ORC_I8_IQ = 1, ORC_I2_REAL = 2, ORC_I2_IQ = 3 };

/* Complex formats: the wipe-off multiplies (xI + j xQ) by exp(-j*theta). */
static int orc_is_complex(int fmt) { return fmt == ORC_I8_IQ || fmt == ORC_I2_IQ; }

/* ------------------------------------------------------------------------ */
/* C/A Gold code, IS-GPS-200 Sec. 3.2.1.3.                                   */
/*   G1 = 1 + x^3 + x^10,  G2 = 1 + x^2 + x^3 + x^6 + x^8 + x^9 + x^10.       */
/* Both 10-stage registers start all ones at the code epoch.  G1's output is */
/* stage 10; the satellite's G2 output is the XOR of two G2 stages (the      */
/* phase-selector taps of Table 3-Ia).  Chip = G1 out XOR G2i out.           */
/* ------------------------------------------------------------------------ */
static const int orc_g2_sel[32][2] = {
    {2, 6},  {3, 7},  {4, 8},  {5, 9},  {1, 9},  {2, 10}, {1, 8},  {2, 9},
    {3, 10}, {2, 3},  {3, 4},  {5, 6},  {6, 7},  {7, 8},  {8, 9},  {9, 10},
    {1, 4},  {2, 5},  {3, 6},  {4, 7},  {5, 8},  {6, 9},  {1, 3},  {4, 6},
    {5, 7},  {6, 8},  {7, 9},  {8, 10}, {1, 6},  {2, 7},  {3, 8},  {4, 9}};

/* Logic levels of the C/A code for one PRN: out[i] in {0,1}, i = 0..1022. */
int orc_ca_bits(int prn, uint8_t* out)
{
    if (prn < 1 || prn > 32 || !out) return ORC_EINVAL;
    int g1[11], g2[11]; /* stage s at index s, 1..10 */
    for (int s = 1; s <= 10; ++s) { g1[s] = 1; g2[s] = 1; }
    const int a = orc_g2_sel[prn - 1][0], b = orc_g2_sel[prn - 1][1];
    for (int i = 0; i < ORC_CODE_LEN; ++i) {
        int g1_out = g1[10];
        int g2_out = g2[a] ^ g2[b];
        out[i] = (uint8_t)(g1_out ^ g2_out);
        int f1 = g1[3] ^ g1[10];
        int f2 = g2[2] ^ g2[3] ^ g2[6] ^ g2[8] ^ g2[9] ^ g2[10];
        for (int s = 10; s > 1; --s) { g1[s] = g1[s - 1]; g2[s] = g2[s - 1]; }
        g1[1] = f1;
        g2[1] = f2;
    }
    return ORC_OK;
}

/* Plain G2 sequence (stage-10 output), used by the tests to check the
 * "G2 delayed by the listed delay" column of Table 3-Ia. */
int orc_g2_bits(uint8_t* out)
{
    if (!out) return ORC_EINVAL;
    int g2[11];
    for (int s = 1; s <= 10; ++s) g2[s] = 1;
    for (int i = 0; i < ORC_CODE_LEN; ++i) {
        out[i] = (uint8_t)g2[10];
        int f2 = g2[2] ^ g2[3] ^ g2[6] ^ g2[8] ^ g2[9] ^ g2[10];
        for (int s = 10; s > 1; --s) g2[s] = g2[s - 1];
        g2[1] = f2;
    }
    return ORC_OK;
}

/* The satellite's G2 output alone (XOR of its two phase-selector stages),
 * used by the tests for the same column check. */
int orc_g2i_bits(int prn, uint8_t* out)
{
    if (prn < 1 || prn > 32 || !out) return ORC_EINVAL;
    int g2[11];
    for (int s = 1; s <= 10; ++s) g2[s] = 1;
    const int a = orc_g2_sel[prn - 1][0], b = orc_g2_sel[prn - 1][1];
    for (int i = 0; i < ORC_CODE_LEN; ++i) {
        out[i] = (uint8_t)(g2[a] ^ g2[b]);
        int f2 = g2[2] ^ g2[3] ^ g2[6] ^ g2[8] ^ g2[9] ^ g2[10];
        for (int s = 10; s > 1; --s) g2[s] = g2[s - 1];
        g2[1] = f2;
    }
    return ORC_OK;
}

/* Chip values: logic 0 -> +1, logic 1 -> -1 (Sec. 3.1 says only "+1's and
 * -1's"; the mapping is a global sign). */
int orc_ca_code(int prn, int8_t* out)
{
    uint8_t bits[ORC_CODE_LEN];
    int rc = orc_ca_bits(prn, bits);
    if (rc) return rc;
    for (int i = 0; i < ORC_CODE_LEN; ++i) out[i] = bits[i] ? -1 : 1;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Carrier sin/cos table.  256 entries indexed by the top 8 bits of the      */
/* 32-bit carrier phase word; entry l holds round(24*cos(2*pi*(l+1/2)/256))  */
/* and round(24*sin(...)), rounding half away from zero (no ties occur).     */
/* ------------------------------------------------------------------------ */
static int8_t orc_round_away(double v)
{
    return (int8_t)(v >= 0.0 ? floor(v + 0.5) : -floor(-v + 0.5));
}

int orc_lut(int8_t* cos_out, int8_t* sin_out)
{
    if (!cos_out || !sin_out) return ORC_EINVAL;
    for (int l = 0; l < ORC_LUT_SIZE; ++l) {
        double ang = 2.0 * M_PI * ((double)l + 0.5) / (double)ORC_LUT_SIZE;
        cos_out[l] = orc_round_away(ORC_LUT_AMP * cos(ang));
        sin_out[l] = orc_round_away(ORC_LUT_AMP * sin(ang));
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* NCO words from physical parameters.                                       */
/*   carrier step  = round_half_even(f_carr / fs * 2^32) mod 2^32            */
/*   carrier phase = round_half_even(frac(phase_cycles) * 2^32) mod 2^32     */
/*   code step     = round_half_even(code_rate / fs * 2^32)   (Q32 chips)    */
/*   code phase    = round_half_even(p * 2^32) mod W,  p = chips mod T*1023  */
/* W = T*1023*2^32 is the integration window of T code periods.             */
/* ------------------------------------------------------------------------ */
int orc_nco_words(double fs_hz, double carr_hz, double carr_phase_cyc,
                  double code_rate_cps, double code_phase_chips, int int_periods,
                  uint32_t* carr_phase, uint32_t* carr_step,
                  uint64_t* code_phase, uint64_t* code_step)
{
    if (!(fs_hz > 0.0) || int_periods < 1 || !(code_rate_cps > 0.0)) return ORC_EINVAL;
    double span = (double)int_periods * ORC_CODE_LEN;
    uint64_t W = (uint64_t)int_periods * ORC_CODE_LEN * (uint64_t)4294967296ULL;

    double cs = nearbyint(carr_hz / fs_hz * ORC_TWO32);
    *carr_step = (uint32_t)(uint64_t)(int64_t)cs;

    double fr = carr_phase_cyc - floor(carr_phase_cyc);
    double cp = nearbyint(fr * ORC_TWO32);
    *carr_phase = (uint32_t)(uint64_t)(int64_t)cp;

    double ks = nearbyint(code_rate_cps / fs_hz * ORC_TWO32);
    if (!(ks >= 1.0) || ks >= 18446744073709551616.0) return ORC_EINVAL;
    *code_step = (uint64_t)ks;

    double p = fmod(code_phase_chips, span);
    if (p < 0.0) p += span;
    double kp = nearbyint(p * ORC_TWO32);
    uint64_t w = (uint64_t)kp;
    *code_phase = w % W;
    return ORC_OK;
}

/* floor(v / 2^32) for a signed 64-bit value, written out. */
static int64_t orc_floor_div_2_32(int64_t v)
{
    const int64_t d = (int64_t)4294967296LL;
    int64_t q = v / d;
    if ((v % d) != 0 && v < 0) q -= 1;
    return q;
}

static int64_t orc_mod(int64_t a, int64_t m)
{
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

/* One sample, unpacked: real formats set xq = 0.
 * 2-bit real: value codes 0,1,2,3 -> -3,-1,+1,+3, four samples per byte,
 * sample j of a byte in bits [2j, 2j+1] (least significant pair first).
 * 2-bit complex: the 2-bit real packing of the interleaved stream I0 Q0 I1
 * Q1 ..., so two samples per byte, sample j's I in bits [4j, 4j+1] and its
 * Q in bits [4j+2, 4j+3], same value codes. */
static void orc_sample(int fmt, const uint8_t* buf, uint64_t n, int* xi, int* xq)
{
    if (fmt == ORC_I8_REAL) {
        *xi = (int)(int8_t)buf[n];
        *xq = 0;
    } else if (fmt == ORC_I8_IQ) {
        *xi = (int)(int8_t)buf[2 * n];
        *xq = (int)(int8_t)buf[2 * n + 1];
    } else if (fmt == ORC_I2_REAL) {
        int code = (buf[n >> 2] >> (2 * (n & 3))) & 3;
        *xi = 2 * code - 3;
        *xq = 0;
    } else {
        const int byte = buf[n >> 1], sh = 4 * (int)(n & 1);
        *xi = 2 * ((byte >> sh) & 3) - 3;
        *xq = 2 * ((byte >> (sh + 2)) & 3) - 3;
    }
}

static int orc_fits_i32(int64_t v) { return v >= INT32_MIN && v <= INT32_MAX; }

/*
 * Integer (LUT) correlator for one channel over one block of samples.
 *
 * Per sample n = 0..N-1 (all integer, exact):
 *   Phi_n = Phi_0 + n*dPhi (mod 2^32),  l = Phi_n >> 24,  (c, s) = LUT[l]
 *   wipe-off by exp(-j*theta):
 *     real     wI =  x*c,            wQ = -x*s
 *     complex  wI =  xI*c + xQ*s,    wQ =  xQ*c - xI*s
 *   U_n = P_0 + n*dP (unwrapped Q32 chips), window m = floor(U_n / W)
 *   a sample of a later window closes the open dump first
 *   P = U_n - m*W;  for each tap k: chip = floor((P + delta_k) / 2^32) mod 1023
 *     I_k += wI * C[chip],  Q_k += wQ * C[chip]
 * At the end of the block every window that U_N (the phase of the next
 * sample) has passed is closed as well, so the open dump always holds the
 * samples of window floor(U_N / W) and any split of a stream into blocks
 * gives the same dumps.
 *
 * acc[] (int64, n_taps*2, I then Q per tap) and acc_n carry the open dump in
 * and out; dumps[] receives closed dumps as [dump][tap][I,Q], dump_n[] their
 * sample counts.  Returns ORC_ERANGE if any accumulation leaves int32,
 * ORC_ENOSPC if more than max_dumps dumps close.
 */
int orc_correlate_lut(int fmt, const uint8_t* buf, uint64_t n_samples,
                      int prn, int n_taps, const int64_t* tap_q32, int int_periods,
                      uint32_t* carr_phase, uint32_t carr_step,
                      uint64_t* code_phase, uint64_t code_step,
                      int64_t* acc, uint32_t* acc_n,
                      int64_t* dumps, uint32_t* dump_n, uint32_t max_dumps,
                      uint32_t* n_dumps)
{
    if (fmt < 0 || fmt > 3 || n_taps < 1 || int_periods < 1 || !acc || !acc_n || !n_dumps)
        return ORC_EINVAL;
    int8_t code[ORC_CODE_LEN], lc[ORC_LUT_SIZE], ls[ORC_LUT_SIZE];
    if (orc_ca_code(prn, code)) return ORC_EINVAL;
    orc_lut(lc, ls);

    const uint64_t W = (uint64_t)int_periods * ORC_CODE_LEN * 4294967296ULL;
    const uint32_t phi0 = *carr_phase;
    const uint64_t p0 = *code_phase;
    if (p0 >= W) return ORC_EINVAL;
    uint64_t cur = 0;      /* window index of the open dump */
    uint32_t nd = 0;
    int rc = ORC_OK;

    for (uint64_t n = 0; n < n_samples; ++n) {
        uint32_t phi = phi0 + (uint32_t)n * carr_step;
        int l = (int)(phi >> 24);
        int c = lc[l], s = ls[l];
        int xi, xq;
        orc_sample(fmt, buf, n, &xi, &xq);
        int64_t wi, wq;
        if (orc_is_complex(fmt)) {
            wi = (int64_t)xi * c + (int64_t)xq * s;
            wq = (int64_t)xq * c - (int64_t)xi * s;
        } else {
            wi = (int64_t)xi * c;
            wq = -(int64_t)xi * s;
        }
        uint64_t u = p0 + n * code_step;
        uint64_t m = u / W;
        while (m > cur) {
            if (nd >= max_dumps || !dumps || !dump_n) return ORC_ENOSPC;
            for (int k = 0; k < 2 * n_taps; ++k) {
                if (!orc_fits_i32(acc[k])) rc = ORC_ERANGE;
                dumps[(uint64_t)nd * 2 * n_taps + k] = acc[k];
                acc[k] = 0;
            }
            dump_n[nd++] = *acc_n;
            *acc_n = 0;
            ++cur;
        }
        int64_t p = (int64_t)(u - m * W);
        for (int k = 0; k < n_taps; ++k) {
            int64_t chip = orc_mod(orc_floor_div_2_32(p + tap_q32[k]), ORC_CODE_LEN);
            int r = code[chip];
            acc[2 * k] += wi * r;
            acc[2 * k + 1] += wq * r;
        }
        *acc_n += 1;
    }
    uint64_t u_end = p0 + n_samples * code_step;
    uint64_t m_end = u_end / W;
    while (m_end > cur) {
        if (nd >= max_dumps || !dumps || !dump_n) return ORC_ENOSPC;
        for (int k = 0; k < 2 * n_taps; ++k) {
            if (!orc_fits_i32(acc[k])) rc = ORC_ERANGE;
            dumps[(uint64_t)nd * 2 * n_taps + k] = acc[k];
            acc[k] = 0;
        }
        dump_n[nd++] = *acc_n;
        *acc_n = 0;
        ++cur;
    }
    for (int k = 0; k < 2 * n_taps; ++k)
        if (!orc_fits_i32(acc[k])) rc = ORC_ERANGE;
    *carr_phase = phi0 + (uint32_t)n_samples * carr_step;
    *code_phase = u_end - m_end * W;
    *n_dumps = nd;
    return rc;
}

/*
 * FP64 form of the same correlator, the reference for the FP32 carrier
 * variant.  The carrier is (cos, sin)(2*pi*frac(phi_0 + n*f)) in double,
 * with phi_0 in cycles and f in cycles per sample, and wipe-off and
 * accumulation are in double; the code NCO, replica, taps and dump rule are
 * the integer ones of orc_correlate_lut unchanged.  On return *carr_phase_cyc
 * is frac(phi_0 + N*f).
 */
int orc_correlate_f64(int fmt, const uint8_t* buf, uint64_t n_samples,
                      int prn, int n_taps, const int64_t* tap_q32, int int_periods,
                      double* carr_phase_cyc, double carr_freq_cyc,
                      uint64_t* code_phase, uint64_t code_step,
                      double* acc, uint32_t* acc_n,
                      double* dumps, uint32_t* dump_n, uint32_t max_dumps,
                      uint32_t* n_dumps)
{
    if (fmt < 0 || fmt > 3 || n_taps < 1 || int_periods < 1 || !acc || !acc_n || !n_dumps)
        return ORC_EINVAL;
    int8_t code[ORC_CODE_LEN];
    if (orc_ca_code(prn, code)) return ORC_EINVAL;
    const uint64_t W = (uint64_t)int_periods * ORC_CODE_LEN * 4294967296ULL;
    const double ph0 = *carr_phase_cyc;
    const uint64_t p0 = *code_phase;
    if (p0 >= W) return ORC_EINVAL;
    uint64_t cur = 0;
    uint32_t nd = 0;

    for (uint64_t n = 0; n < n_samples; ++n) {
        double t = ph0 + (double)n * carr_freq_cyc;
        double th = 2.0 * M_PI * (t - floor(t));
        double c = cos(th), s = sin(th);
        int xi, xq;
        orc_sample(fmt, buf, n, &xi, &xq);
        double wi, wq;
        if (orc_is_complex(fmt)) {
            wi = xi * c + xq * s;
            wq = xq * c - xi * s;
        } else {
            wi = xi * c;
            wq = -xi * s;
        }
        uint64_t u = p0 + n * code_step;
        uint64_t m = u / W;
        while (m > cur) {
            if (nd >= max_dumps || !dumps || !dump_n) return ORC_ENOSPC;
            for (int k = 0; k < 2 * n_taps; ++k) {
                dumps[(uint64_t)nd * 2 * n_taps + k] = acc[k];
                acc[k] = 0.0;
            }
            dump_n[nd++] = *acc_n;
            *acc_n = 0;
            ++cur;
        }
        int64_t p = (int64_t)(u - m * W);
        for (int k = 0; k < n_taps; ++k) {
            int64_t chip = orc_mod(orc_floor_div_2_32(p + tap_q32[k]), ORC_CODE_LEN);
            int r = code[chip];
            acc[2 * k] += wi * r;
            acc[2 * k + 1] += wq * r;
        }
        *acc_n += 1;
    }
    uint64_t u_end = p0 + n_samples * code_step;
    uint64_t m_end = u_end / W;
    while (m_end > cur) {
        if (nd >= max_dumps || !dumps || !dump_n) return ORC_ENOSPC;
        for (int k = 0; k < 2 * n_taps; ++k) {
            dumps[(uint64_t)nd * 2 * n_taps + k] = acc[k];
            acc[k] = 0.0;
        }
        dump_n[nd++] = *acc_n;
        *acc_n = 0;
        ++cur;
    }
    double t_end = ph0 + (double)n_samples * carr_freq_cyc;
    *carr_phase_cyc = t_end - floor(t_end);
    *code_phase = u_end - m_end * W;
    *n_dumps = nd;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Closed tracking loops (Table 3): a 2nd-order DLL with the normalised     */
/* early-minus-late envelope discriminator and carrier aiding, and a        */
/* 2nd-order PLL (atan discriminator) assisted by a 1st-order FLL (atan2    */
/* discriminator).  The paper names the loop types only; the filter form   */
/* and its coefficients follow the softGNSS receiver it builds on:          */
/*   Wn = B * 8 z / (4 z^2 + 1),  tau1 = k / Wn^2,  tau2 = 2 z / Wn,          */
/*   nco += (tau2 / tau1) (e - e_prev) + e (T / tau1),                        */
/* with B the noise bandwidth (Hz), z the damping ratio, k the loop gain and */
/* T the dump length (int_periods ms).  The FLL is first order with gain    */
/* 4 B_f T on the frequency basis.  Angles come from a vectoring CORDIC on  */
/* the integer dumps (Volder, 1959), so that every step is exact integer    */
/* arithmetic or a correctly rounded double operation.                      */
/* ------------------------------------------------------------------------ */
#define ORC_CORDIC_N 31
#define ORC_Q30 1073741824.0

/* atan2(y, x) for x >= 0, in units of 2^-30 rad: the vector is scaled into */
/* [2^39, 2^40) by shifts, then rotated towards the x axis by +-atan(2^-i). */
static int64_t orc_cordic_tab[ORC_CORDIC_N];  /* round(atan(2^-i) * 2^30) */

__attribute__((constructor)) static void orc_cordic_init(void)
{
    for (int i = 0; i < ORC_CORDIC_N; ++i)
        orc_cordic_tab[i] = llround(atan(ldexp(1.0, -i)) * ORC_Q30);
}

static int64_t orc_atan2_q30(int64_t y, int64_t x)
{
    const int64_t* tab = orc_cordic_tab;
    if (x == 0 && y == 0) return 0;
    const int64_t hi = (int64_t)1 << 40, lo = (int64_t)1 << 39;
    while (llabs(x) >= hi || llabs(y) >= hi) { x >>= 1; y >>= 1; }
    while (llabs(x) < lo && llabs(y) < lo) { x *= 2; y *= 2; }
    int64_t z = 0;
    for (int i = 0; i < ORC_CORDIC_N; ++i) {
        const int64_t xs = x >> i, ys = y >> i;
        if (y > 0) { x += ys; y -= xs; z += tab[i]; }
        else       { x -= ys; y += xs; z -= tab[i]; }
    }
    return z;
}

int orc_cordic_table(int64_t* out)
{
    if (!out) return ORC_EINVAL;
    for (int i = 0; i < ORC_CORDIC_N; ++i) out[i] = orc_cordic_tab[i];
    return ORC_OK;
}

int orc_cordic_atan2(int64_t y, int64_t x, int64_t* out)
{
    if (!out || x < 0) return ORC_EINVAL;
    *out = orc_atan2_q30(y, x);
    return ORC_OK;
}

/* Loop coefficients (tau1, tau2) of a loop with noise bandwidth B, damping */
/* z and gain k. */
static void orc_loop_coef(double B, double z, double k, double* tau1, double* tau2)
{
    const double wn = B * 8.0 * z / (4.0 * z * z + 1.0);
    *tau1 = k / (wn * wn);
    *tau2 = 2.0 * z / wn;
}

int orc_loop_coefficients(double B, double z, double k, double* out2)
{
    if (!out2 || !(B > 0.0) || !(z > 0.0) || !(k > 0.0)) return ORC_EINVAL;
    orc_loop_coef(B, z, k, &out2[0], &out2[1]);
    return ORC_OK;
}

/* Halve all four values until each magnitude is below 2^30 (products and */
/* their sums then stay inside int64). */
static void orc_shrink4(int64_t* a, int64_t* b, int64_t* c, int64_t* d)
{
    const int64_t lim = (int64_t)1 << 30;
    while (llabs(*a) >= lim || llabs(*b) >= lim || llabs(*c) >= lim || llabs(*d) >= lim) {
        *a >>= 1; *b >>= 1; *c >>= 1; *d >>= 1;
    }
}

/*
 * Loop update at the close of a dump.
 *   prm[9]  = fs, IF, DLL (B, z, k), PLL (B, z, k), FLL B        (Hz, -, -)
 *   ls[7]   = carr_freq (Hz), code_freq (chips/s), FLL basis (Hz),
 *             PLL nco (Hz), previous PLL error (cycles), DLL nco (chips/s),
 *             previous DLL error
 *   is[3]   = previous prompt I, Q, and whether they are set
 *   d[6]    = E I, E Q, P I, P Q, L I, L Q of the closed dump
 * PLL error = atan(Q_P / I_P) / (2 pi) cycles; FLL error = atan2(cross,
 * dot) / (2 pi T) Hz with cross = I'Q - Q'I, dot = I'I + Q'Q of the previous
 * (') and current prompts, the dot product's sign removed (a navigation-bit
 * flip between dumps turns the prompt by pi, not the frequency); DLL error =
 * (|E| - |L|) / (|E| + |L|).  Carrier frequency = FLL basis + PLL nco; code
 * frequency = 1.023 MHz (1 + (carrier - IF) / 1575.42 MHz) + DLL nco.  The
 * new NCO steps are round_half_even(f / fs * 2^32).  Returns ORC_ERANGE when
 * the code step leaves [1, 2^31).
 */
/* The largest |wipe-off| of one sample: 128 * 24 (int8 real), 128 * the   */
/* largest |cos| + |sin| of the table (int8 I/Q), 3 * 24 (2-bit real), 3 * */
/* the largest |cos| + |sin| (2-bit I/Q). */
static int64_t orc_max_w(int fmt)
{
    if (fmt == ORC_I8_REAL) return 128 * 24;
    if (fmt == ORC_I2_REAL) return 3 * 24;
    int8_t c[ORC_LUT_SIZE], s[ORC_LUT_SIZE];
    orc_lut(c, s);
    int m = 0;
    for (int l = 0; l < ORC_LUT_SIZE; ++l) {
        const int v = abs(c[l]) + abs(s[l]);
        if (v > m) m = v;
    }
    return (fmt == ORC_I2_IQ ? 3 : 128) * (int64_t)m;
}

/* A code step keeps every dump inside int32 when a window of W holds at   */
/* most floor((W - 1) / dp) + 1 samples of at most max|w| each.            */
static int orc_step_in_range(uint64_t dp, uint64_t W, int fmt)
{
    if (dp < 1 || dp >= ((uint64_t)1 << 31)) return 0;
    const uint64_t cnt = (W - 1) / dp + 1;
    return cnt * (uint64_t)orc_max_w(fmt) < ((uint64_t)1 << 31);
}

static int orc_loop_update(const double* prm, int int_periods, const int64_t* d, double* ls,
                           int32_t* is, uint32_t* carr_step, uint64_t* code_step)
{
    const double T = (double)int_periods * 1e-3;
    double t1c, t2c, t1d, t2d;
    orc_loop_coef(prm[5], prm[6], prm[7], &t1c, &t2c);
    orc_loop_coef(prm[2], prm[3], prm[4], &t1d, &t2d);
    const int64_t ie = d[0], qe = d[1], ip = d[2], qp = d[3], il = d[4], ql = d[5];
    /* PLL */
    const int64_t a = ip >= 0 ? orc_atan2_q30(qp, ip) : orc_atan2_q30(-qp, -ip);
    const double carr_err = ((double)a / ORC_Q30) / (2.0 * M_PI);
    /* FLL */
    if (is[2]) {
        int64_t i0 = is[0], q0 = is[1], i1 = ip, q1 = qp;
        orc_shrink4(&i0, &q0, &i1, &q1);
        const int64_t dot = i0 * i1 + q0 * q1;
        const int64_t cross = i0 * q1 - q0 * i1;
        const int64_t f = dot >= 0 ? orc_atan2_q30(cross, dot) : orc_atan2_q30(-cross, -dot);
        const double f_err = ((double)f / ORC_Q30) / (2.0 * M_PI * T);
        ls[2] = ls[2] + (4.0 * prm[8] * T) * f_err;
    }
    is[0] = (int32_t)ip;
    is[1] = (int32_t)qp;
    is[2] = 1;
    /* PLL filter */
    {
        const double u1 = (t2c / t1c) * (carr_err - ls[4]);
        const double u2 = carr_err * (T / t1c);
        ls[3] = ls[3] + (u1 + u2);
        ls[4] = carr_err;
    }
    ls[0] = ls[2] + ls[3];
    /* DLL */
    {
        const double fe = (double)ie, ge = (double)qe, fl = (double)il, gl = (double)ql;
        const double E = sqrt(fe * fe + ge * ge), L = sqrt(fl * fl + gl * gl);
        const double code_err = (E + L) > 0.0 ? (E - L) / (E + L) : 0.0;
        const double u1 = (t2d / t1d) * (code_err - ls[6]);
        const double u2 = code_err * (T / t1d);
        ls[5] = ls[5] + (u1 + u2);
        ls[6] = code_err;
    }
    ls[1] = 1.023e6 * (1.0 + (ls[0] - prm[1]) / 1575.42e6) + ls[5];
    const double cs = nearbyint(ls[0] / prm[0] * ORC_TWO32);
    *carr_step = (uint32_t)(uint64_t)(int64_t)cs;
    const double ks = nearbyint(ls[1] / prm[0] * ORC_TWO32);
    if (!(ks >= 1.0) || !(ks < 2147483648.0)) return ORC_ERANGE;
    *code_step = (uint64_t)ks;
    return ORC_OK;
}

/*
 * Closed-loop tracking of one E/P/L channel (taps +1/2, 0, -1/2 chip) over
 * one block.  Per sample the correlation is that of orc_correlate_lut with
 * the code phase kept inside the window: before sample n, a phase that has
 * reached W closes the dump (its sums, its sample count and the NCO steps
 * used for it are emitted, the loops update the steps) and the phase drops
 * by W; the end of the block closes a dump whose phase has reached W as
 * well.  rows[] receives per closed dump the six sums followed by the
 * carrier and code steps used, as int32 (the steps' bit patterns).  The
 * code step, at the start and after every update, must keep a window's sums
 * inside int32 (the bound of orc_step_in_range), else ORC_ERANGE.
 */
int orc_track(int fmt, const uint8_t* buf, uint64_t n_samples, int prn, int int_periods,
              const double* prm, uint32_t* carr_phase, uint32_t* carr_step,
              uint64_t* code_phase, uint64_t* code_step, int64_t* acc, uint32_t* acc_n,
              double* ls, int32_t* is, int32_t* rows, uint32_t* dump_n, uint32_t max_dumps,
              uint32_t* n_dumps)
{
    if (fmt < 0 || fmt > 3 || int_periods < 1 || !prm || !acc || !acc_n || !ls || !is ||
        !n_dumps || !carr_phase || !carr_step || !code_phase || !code_step)
        return ORC_EINVAL;
    int8_t code[ORC_CODE_LEN], lc[ORC_LUT_SIZE], ls8[ORC_LUT_SIZE];
    if (orc_ca_code(prn, code)) return ORC_EINVAL;
    orc_lut(lc, ls8);
    const int64_t taps[3] = {(int64_t)1 << 31, 0, -((int64_t)1 << 31)};
    const uint64_t W = (uint64_t)int_periods * ORC_CODE_LEN * 4294967296ULL;
    uint32_t phi = *carr_phase, dphi = *carr_step;
    uint64_t p = *code_phase, dp = *code_step;
    if (p >= W) return ORC_EINVAL;
    if (!orc_step_in_range(dp, W, fmt)) return ORC_ERANGE;
    uint32_t nd = 0;
    int rc = ORC_OK;
    for (uint64_t n = 0; n <= n_samples; ++n) {
        if (p >= W) {
            if (nd >= max_dumps || !rows || !dump_n) return ORC_ENOSPC;
            for (int k = 0; k < 6; ++k) {
                if (!orc_fits_i32(acc[k])) rc = ORC_ERANGE;
                rows[(uint64_t)nd * 8 + k] = (int32_t)acc[k];
            }
            rows[(uint64_t)nd * 8 + 6] = (int32_t)dphi;
            rows[(uint64_t)nd * 8 + 7] = (int32_t)(uint32_t)dp;
            dump_n[nd++] = *acc_n;
            const int u = orc_loop_update(prm, int_periods, acc, ls, is, &dphi, &dp);
            if (u != ORC_OK) return u;
            if (!orc_step_in_range(dp, W, fmt)) return ORC_ERANGE;
            for (int k = 0; k < 6; ++k) acc[k] = 0;
            *acc_n = 0;
            p -= W;
        }
        if (n == n_samples) break;
        const int l = (int)(phi >> 24);
        const int c = lc[l], s = ls8[l];
        int xi, xq;
        orc_sample(fmt, buf, n, &xi, &xq);
        int64_t wi, wq;
        if (orc_is_complex(fmt)) {
            wi = (int64_t)xi * c + (int64_t)xq * s;
            wq = (int64_t)xq * c - (int64_t)xi * s;
        } else {
            wi = (int64_t)xi * c;
            wq = -(int64_t)xi * s;
        }
        for (int k = 0; k < 3; ++k) {
            const int64_t chip = orc_mod(orc_floor_div_2_32((int64_t)p + taps[k]), ORC_CODE_LEN);
            acc[2 * k] += wi * code[chip];
            acc[2 * k + 1] += wq * code[chip];
        }
        *acc_n += 1;
        phi += dphi;
        p += dp;
    }
    for (int k = 0; k < 6; ++k)
        if (!orc_fits_i32(acc[k])) rc = ORC_ERANGE;
    *carr_phase = phi;
    *carr_step = dphi;
    *code_phase = p;
    *code_step = dp;
    *n_dumps = nd;
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Lock metrics and bit synchronisation over a channel's closed dumps       */
/* (the Channel Health indicators of Sec. 3.6 and the 20-period navigation */
/* bits of Sec. 3.1).  prompt[k] = (I_k, Q_k) of dump k, k = 0 .. n-1.       */
/*                                                                          */
/* C/N0 per window of K consecutive dumps, by the moments (M2M4) estimator  */
/* of Pauluzzi and Beaulieu (2000): with P_k = I_k^2 + Q_k^2,               */
/*   M2 = mean P_k,  M4 = mean P_k^2,  A = sqrt(2 M2^2 - M4) (signal power), */
/*   SNR = A / (M2 - A),  C/N0 = 10 log10(SNR / T)  (dB-Hz, T in seconds);  */
/* a window whose 2 M2^2 - M4 <= 0 or M2 - A <= 0 gets NaN.                  */
/* Carrier lock ratio per window, the estimate of cos(2 phase error):       */
/*   sum (I_k^2 - Q_k^2) / sum (I_k^2 + Q_k^2)  (0 for an all-zero window). */
/* A window is a lock failure when its ratio is below lock_min.             */
/* Bit edge: for each k >= 1 whose prompt I changes sign from dump k-1 to    */
/* k (zero counts as positive), position (k + phase) mod 20 gets one count; */
/* the edge is the position with the most counts (the lowest on ties).      */
/* With the edge e, bit j sums I over dumps k with (k + phase - e) mod 20    */
/* = 0 .. 19 of the j-th whole period after the edge, and is 1 when the sum */
/* is negative (logic 1 -> -1, as for the code chips).                      */
/* ------------------------------------------------------------------------ */
int orc_lock_metrics(const int32_t* prompt, uint32_t n, uint32_t K, double T, double lock_min,
                     uint32_t phase, double* cn0, double* lock, uint32_t* n_windows,
                     uint32_t* lock_fails, uint32_t* hist, uint32_t* edge, uint8_t* bits,
                     uint32_t max_bits, uint32_t* n_bits)
{
    if (!prompt && n) return ORC_EINVAL;
    if (K < 2 || !(T > 0.0) || !n_windows || !lock_fails || !hist || !edge || !n_bits)
        return ORC_EINVAL;
    const uint32_t nw = n / K;
    uint32_t fails = 0;
    for (uint32_t w = 0; w < nw; ++w) {
        double m2 = 0.0, m4 = 0.0, ii = 0.0, qq = 0.0;
        for (uint32_t k = w * K; k < (w + 1) * K; ++k) {
            const double i = (double)prompt[2 * k], q = (double)prompt[2 * k + 1];
            const double p = i * i + q * q;
            m2 += p;
            m4 += p * p;
            ii += i * i;
            qq += q * q;
        }
        m2 = m2 / (double)K;
        m4 = m4 / (double)K;
        const double d = 2.0 * m2 * m2 - m4;
        double c = NAN;
        if (d > 0.0) {
            const double a = sqrt(d);
            if (m2 - a > 0.0) c = 10.0 * log10((a / (m2 - a)) / T);
        }
        const double r = (ii + qq) > 0.0 ? (ii - qq) / (ii + qq) : 0.0;
        if (cn0) cn0[w] = c;
        if (lock) lock[w] = r;
        if (r < lock_min) ++fails;
    }
    *n_windows = nw;
    *lock_fails = fails;
    for (int j = 0; j < 20; ++j) hist[j] = 0;
    for (uint32_t k = 1; k < n; ++k) {
        const int a = prompt[2 * (k - 1)] < 0, b = prompt[2 * k] < 0;
        if (a != b) hist[(k + phase) % 20] += 1;
    }
    uint32_t e = 0;
    for (uint32_t j = 1; j < 20; ++j)
        if (hist[j] > hist[e]) e = j;
    *edge = e;
    /* first dump of the first whole bit: smallest k with (k + phase) % 20 == e */
    const uint32_t k0 = (e + 20 - phase % 20) % 20;
    uint32_t nb = 0;
    for (uint64_t k = k0; k + 20 <= n; k += 20) {
        int64_t s = 0;
        for (uint32_t t = 0; t < 20; ++t) s += prompt[2 * (k + t)];
        if (nb < max_bits && bits) bits[nb] = (uint8_t)(s < 0);
        ++nb;
    }
    *n_bits = nb < max_bits ? nb : max_bits;
    return ORC_OK;
}
