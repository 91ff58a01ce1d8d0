"""Pins of the CPU oracle to facts that do not come from the oracle itself.

IS-GPS-200 Table 3-Ia columns, Gold-family correlation values, the nearest-
integer property of the carrier table, exact rational NCO words, closed-form
geometric sums, the fs/4 carrier hand formula, three-valued correlations
through the whole correlator, chunking invariance and a matrix-form brute
force.  None of these needs a GPU.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute

HERE = os.path.dirname(os.path.abspath(__file__))
TWO32 = 1 << 32


def _table_3_1a():
    rows = []
    with open(os.path.join(HERE, "golden", "is_gps_200_table_3_1a.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                prn, a, b, d, octal = line.split()
                rows.append((int(prn), int(a), int(b), int(d), octal))
    assert len(rows) == 32
    return rows


# ---------------------------------------------------------------- Gold codes
@pytest.mark.parametrize("row", _table_3_1a(), ids=lambda r: "prn%d" % r[0])
def test_first_ten_chips_octal(row):
    prn, _, _, _, octal = row
    bits = oracle.ca_bits(prn)
    word = int("".join(str(int(b)) for b in bits[:10]), 2)
    assert format(word, "o") == octal


@pytest.mark.parametrize("row", _table_3_1a(), ids=lambda r: "prn%d" % r[0])
def test_g2_taps_equal_listed_delay(row):
    prn, _, _, delay, _ = row
    g2 = oracle.g2_bits()
    g2i = oracle.g2i_bits(prn)
    idx = (np.arange(1023) - delay) % 1023
    assert np.array_equal(g2i, g2[idx])


def test_g1_part_is_the_same_for_all_prns():
    g1 = [oracle.ca_bits(p) ^ oracle.g2i_bits(p) for p in range(1, 33)]
    for g in g1[1:]:
        assert np.array_equal(g, g1[0])
    assert np.all(g1[0][:10] == 1)  # all-ones start: the first output is stage 10 = 1
    assert int(g1[0].sum()) == 512  # an m-sequence of period 1023 has 512 ones


def _circ_xcorr(a, b):
    fa = np.fft.fft(a.astype(np.float64))
    fb = np.fft.fft(b.astype(np.float64))
    # r[k] = sum_i a[i] * b[i + k]
    return np.rint(np.real(np.fft.ifft(np.conj(fa) * fb))).astype(np.int64)


def test_gold_auto_and_cross_correlation_three_valued():
    codes = [oracle.ca_code(p).astype(np.int64) for p in range(1, 33)]
    allowed = {-65, -1, 63}
    for i, a in enumerate(codes):
        r = _circ_xcorr(a, a)
        assert r[0] == 1023
        assert set(np.unique(r[1:])) <= allowed
        for b in codes[i + 1:]:
            assert set(np.unique(_circ_xcorr(a, b))) <= allowed


def test_code_values_and_prn_range():
    c = oracle.ca_code(1)
    assert c.dtype == np.int8 and set(np.unique(c)) == {-1, 1}
    assert np.array_equal(c, np.where(oracle.ca_bits(1) == 1, -1, 1))
    with pytest.raises(ValueError):
        oracle.ca_code(0)
    with pytest.raises(ValueError):
        oracle.ca_code(33)


# ---------------------------------------------------------------- carrier table
def test_lut_is_the_nearest_integer_table():
    c, s = oracle.lut()
    ang = 2 * np.pi * (np.arange(256) + 0.5) / 256
    # nearest integer is unique when no value sits on a .5 tie
    assert np.all(np.abs(c - 24 * np.cos(ang)) < 0.5)
    assert np.all(np.abs(s - 24 * np.sin(ang)) < 0.5)
    assert np.min(np.abs(np.abs(24 * np.cos(ang) - np.floor(24 * np.cos(ang))) - 0.5)) > 1e-3


def test_lut_symmetries():
    c, s = oracle.lut()
    c = c.astype(int)
    s = s.astype(int)
    l = np.arange(256)
    assert np.array_equal(c[(l + 128) % 256], -c)
    assert np.array_equal(s[(l + 128) % 256], -s)
    assert np.array_equal(c[(l + 64) % 256], -s)
    assert np.array_equal(s[(l + 64) % 256], c)
    assert (c[0], c[64], c[128], c[192]) == (24, 0, -24, 0)
    assert (s[0], s[64], s[128], s[192]) == (0, 24, 0, -24)
    assert np.max(np.abs(c) + np.abs(s)) == 34


# ---------------------------------------------------------------- NCO words
def _rhe(fr: Fraction) -> int:
    """round half to even of an exact rational."""
    fl = fr.numerator // fr.denominator
    rem = fr - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        return fl + 1
    return fl


@pytest.mark.parametrize("fs,carr,rate,p0,T", [
    (4.092e6, 1.0245e6, 1.023e6 * (1 + 1500 / 1575.42e6), 300.25, 1),
    (16.368e6, 4.092e6 - 3210.5, 1.023e6 * (1 - 3210.5 / 1575.42e6), 1022.9, 1),
    (16.368e6, 4.092e6 + 4999.0, 1.023e6, 17000.5, 20),
    (20.46e6, -4321.0, 1.023e6 * (1 - 4321 / 1575.42e6), 5.0, 4),
])
def test_nco_words_match_exact_rational_rounding(fs, carr, rate, p0, T):
    cp, cs, kp, ks = oracle.nco_words(fs, carr, 0.0, rate, p0, T)
    # the doubles themselves are exact rationals; the rounding rule is what is pinned
    assert cs == _rhe(Fraction(carr) / Fraction(fs) * TWO32) % TWO32
    assert ks == _rhe(Fraction(rate) / Fraction(fs) * TWO32)
    assert kp == _rhe(Fraction(p0) * TWO32) % (T * 1023 * TWO32)
    assert cp == 0


def test_nco_worked_numbers_single_channel_workload():
    cp, cs, kp, ks = oracle.nco_words(4.092e6, 1.023e6 + 1500.0, 0.0,
                                      1.023e6 * (1 + 1500.0 / 1575.42e6), 300.25, 1)
    assert cs == 1_075_316_226
    assert ks == 1_073_742_846
    assert kp == 300 * TWO32 + TWO32 // 4


def test_negative_frequency_wraps_twos_complement():
    _, cs, _, _ = oracle.nco_words(4e6, -1e6, 0.0, 1.023e6, 0.0, 1)
    assert cs == TWO32 - TWO32 // 4


# ---------------------------------------------------------------- helpers
def _fresh(carr_phase, carr_step, code_phase, code_step, K):
    return oracle.OracleState(carr_phase, carr_step, code_phase, code_step, K)


def _rand_buf(rng, fmt, n):
    nb = {0: n, 1: 2 * n, 2: (n + 3) // 4, 3: (n + 1) // 2}[fmt]
    return rng.integers(0, 256, size=nb, dtype=np.uint8)


def _i2iq_as_i8iq(buf, n):
    """A 2-bit complex block rewritten as int8 complex: the interleaved
    stream I0 Q0 I1 Q1 ... of 2-bit value codes (four per byte, lowest bit
    pair first), each code c as the int8 2c - 3."""
    b = np.asarray(buf, np.uint8)[: (n + 1) // 2].astype(np.int64)
    codes = np.stack([(b >> s) & 3 for s in (0, 2, 4, 6)], axis=1).reshape(-1)[: 2 * n]
    return (2 * codes - 3).astype(np.int8).view(np.uint8)


# ---------------------------------------------------------------- correlator
@pytest.mark.parametrize("seed", range(12))
def test_brute_force_matches_oracle(seed):
    rng = np.random.default_rng(seed)
    fmt = int(rng.integers(0, 3))
    n = int(rng.integers(1, 160))
    T = int(rng.integers(1, 3))
    W = T * 1023 * TWO32
    code_step = int(rng.integers(TWO32 // 20, TWO32 // 2))
    # start near the window end so that dumps close inside the block
    code_phase = int(W - rng.integers(0, n * code_step + 1)) % W
    carr_phase = int(rng.integers(0, TWO32))
    carr_step = int(rng.integers(0, TWO32))
    K = int(rng.integers(1, 7))
    taps = rng.integers(-3 * TWO32, 3 * TWO32, size=K, dtype=np.int64)
    prn = int(rng.integers(1, 33))
    buf = _rand_buf(rng, fmt, n)
    lc, ls = oracle.lut()
    code = oracle.ca_code(prn)
    bd, bn, bopen, bopen_n, bcp, bkp = brute.correlate(fmt, buf, n, code, taps, T, carr_phase,
                                                       carr_step, code_phase, code_step, lc, ls)
    st = _fresh(carr_phase, carr_step, code_phase, code_step, K)
    od, on = oracle.correlate_lut(fmt, buf, n, prn, taps, T, st)
    assert np.array_equal(od, bd)
    assert np.array_equal(on, bn)
    assert np.array_equal(st.acc.reshape(K, 2), bopen)
    assert st.acc_n == bopen_n
    assert st.carr_phase == bcp and st.code_phase == bkp


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_matches_oracle_i2iq(seed):
    # 2-bit complex: the matrix-form brute force unpacks through numpy's bit
    # unpacking, the oracle through shifts of each byte
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(1, 160))
    T = int(rng.integers(1, 3))
    W = T * 1023 * TWO32
    code_step = int(rng.integers(TWO32 // 20, TWO32 // 2))
    code_phase = int(W - rng.integers(0, n * code_step + 1)) % W
    carr_phase = int(rng.integers(0, TWO32))
    carr_step = int(rng.integers(0, TWO32))
    K = int(rng.integers(1, 7))
    taps = rng.integers(-3 * TWO32, 3 * TWO32, size=K, dtype=np.int64)
    prn = int(rng.integers(1, 33))
    buf = _rand_buf(rng, 3, n)
    lc, ls = oracle.lut()
    bd, bn, bopen, bopen_n, bcp, bkp = brute.correlate(3, buf, n, oracle.ca_code(prn), taps, T,
                                                       carr_phase, carr_step, code_phase,
                                                       code_step, lc, ls)
    st = _fresh(carr_phase, carr_step, code_phase, code_step, K)
    od, on = oracle.correlate_lut(3, buf, n, prn, taps, T, st)
    assert np.array_equal(od, bd) and np.array_equal(on, bn)
    assert np.array_equal(st.acc.reshape(K, 2), bopen) and st.acc_n == bopen_n
    assert st.carr_phase == bcp and st.code_phase == bkp


@pytest.mark.parametrize("f64", [False, True])
def test_i2iq_equals_i8iq_on_expanded_stream(f64):
    # the same complex values given as 2-bit codes and as int8 give the same
    # dumps, open dump and NCO words (integer and FP64 carrier)
    rng = np.random.default_rng(520 + f64)
    n = 60001
    buf2 = _rand_buf(rng, 3, n)
    buf8 = _i2iq_as_i8iq(buf2, n)
    assert buf8.size == 2 * n and set(np.unique(buf8.view(np.int8))) <= {-3, -1, 1, 3}
    for T, taps in ((1, oracle.EPL_TAPS_Q32), (4, np.array([5 << 27, -(3 << 29)], np.int64))):
        a = _fresh(0x12345678, 0x3F00ABCD, 700 * TWO32 + 99, TWO32 // 7, len(taps))
        a.carr_phase_f, a.carr_freq_f = 0.3125, 0.2471
        b = a.copy()
        if f64:
            da, na = oracle.correlate_f64(3, buf2, n, 9, taps, T, a)
            db, nb = oracle.correlate_f64(1, buf8, n, 9, taps, T, b)
        else:
            da, na = oracle.correlate_lut(3, buf2, n, 9, taps, T, a)
            db, nb = oracle.correlate_lut(1, buf8, n, 9, taps, T, b)
        assert len(da) >= 2
        assert np.array_equal(da, db) and np.array_equal(na, nb)
        assert np.array_equal(a.acc, b.acc) and a.acc_n == b.acc_n
        assert a.code_phase == b.code_phase and a.carr_phase == b.carr_phase


def test_i2iq_bit_layout_by_hand():
    # byte 0b11_10_01_00 holds I0 = code 0, Q0 = code 1, I1 = code 2, Q1 =
    # code 3: samples (-3, -1) and (+1, +3).  With a carrier of phase 0 and
    # step 0 (table entry 0: c = cL[0], s = sL[0]) and one prompt tap on a
    # zero code phase, each sample adds (xI c + xQ s, xQ c - xI s) * C[0].
    lc, ls = oracle.lut()
    c, s = int(lc[0]), int(ls[0])
    r = int(oracle.ca_code(3)[0])
    st = _fresh(0, 0, 0, 1 << 28, 1)
    oracle.correlate_lut(3, np.array([0b11100100], np.uint8), 2, 3, np.array([0], np.int64), 1, st)
    want_i = ((-3) * c + (-1) * s + 1 * c + 3 * s) * r
    want_q = ((-1) * c - (-3) * s + 3 * c - 1 * s) * r
    assert list(st.acc) == [want_i, want_q] and st.acc_n == 2


@pytest.mark.parametrize("fmt", [0, 1, 2, 3])
def test_chunking_invariance(fmt):
    rng = np.random.default_rng(100 + fmt)
    n = 40000
    T = 1
    code_step = TWO32 // 4 + 1234
    st0 = _fresh(123456789, 987654321, 1000 * TWO32 + 77, code_step, 3)
    buf = _rand_buf(rng, fmt, n)
    whole = st0.copy()
    d_all, n_all = oracle.correlate_lut(fmt, buf, n, 5, oracle.EPL_TAPS_Q32, T, whole)
    cuts = np.sort(rng.choice(np.arange(1, n // 4), size=7, replace=False)) * 4
    cuts = [0] + list(cuts) + [n]
    st = st0.copy()
    ds, ns = [], []
    for a, b in zip(cuts[:-1], cuts[1:]):
        nb = {0: (a, b), 1: (2 * a, 2 * b), 2: (a // 4, b // 4), 3: (a // 2, b // 2)}[fmt]
        d, dn = oracle.correlate_lut(fmt, buf[nb[0]:nb[1]], b - a, 5, oracle.EPL_TAPS_Q32, T, st)
        ds.append(d)
        ns.append(dn)
    assert np.array_equal(np.concatenate(ds), d_all)
    assert np.array_equal(np.concatenate(ns), n_all)
    assert np.array_equal(st.acc, whole.acc) and st.acc_n == whole.acc_n
    assert (st.carr_phase, st.code_phase) == (whole.carr_phase, whole.code_phase)
    # closed form of the NCO words equals what the loop carried
    cp, kp = oracle.advance_words(st0.carr_phase, st0.carr_step, st0.code_phase, code_step, T, n)
    assert (cp, kp) == (whole.carr_phase, whole.code_phase)
    # every sample lands in exactly one dump or the open one
    assert int(n_all.sum()) + whole.acc_n == n


def test_split_exactly_on_a_dump_boundary():
    # a block that ends exactly where a window ends closes that dump itself
    code_step = TWO32 // 4
    st = _fresh(0, 0, 0, code_step, 1)
    buf = np.full(4092, 1, np.uint8)
    d, dn = oracle.correlate_lut(0, buf, 4092, 1, [0], 1, st)
    assert len(d) == 1 and dn[0] == 4092 and st.acc_n == 0 and st.code_phase == 0


def test_fs_over_4_hand_formula():
    # carrier step 2^32/4 from phase 0 visits l = 0, 64, 128, 192 where
    # (c, s) = (24, 0), (0, 24), (-24, 0), (0, -24): wI = 24*x*(1,0,-1,0)[n%4],
    # wQ = -24*x*(0,1,0,-1)[n%4]; code step 2^32/4 -> chip = c0 + n//4.
    rng = np.random.default_rng(7)
    n = 4 * 1023
    buf = rng.integers(0, 256, size=n, dtype=np.uint8)
    x = buf.view(np.int8).astype(np.int64)
    c0 = 17
    prn = 9
    code = oracle.ca_code(prn).astype(np.int64)
    st = _fresh(0, TWO32 // 4, c0 * TWO32, TWO32 // 4, 1)
    d, dn = oracle.correlate_lut(0, buf, n, prn, [0], 1, st)
    k = np.arange(n)
    chip = code[(c0 + k // 4) % 1023]
    ci = np.array([1, 0, -1, 0])[k % 4]
    sq = np.array([0, 1, 0, -1])[k % 4]
    I_hand = int(np.sum(24 * x * ci * chip))
    Q_hand = int(np.sum(-24 * x * sq * chip))
    # window boundary at chip 1023 (after 4*(1023-17) samples): one dump + open rest
    split = 4 * (1023 - c0)
    assert len(d) == 1 and dn[0] == split
    assert d[0, 0, 0] == int(np.sum((24 * x * ci * chip)[:split]))
    assert d[0, 0, 1] == int(np.sum((-24 * x * sq * chip)[:split]))
    assert d[0, 0, 0] + st.acc[0] == I_hand
    assert d[0, 0, 1] + st.acc[1] == Q_hand


@pytest.mark.parametrize("pa,pb", [(1, 1), (3, 3), (1, 2), (7, 19), (31, 4)])
def test_three_valued_correlation_through_the_correlator(pa, pb):
    # complex zero-IF input x = a*C_a (I only), zero carrier, 4 samples per chip
    # and taps at whole-chip offsets: I_k = 4*24*a*R_ab(k), Q_k = 0.
    a = 3
    ca = oracle.ca_code(pa).astype(np.int64)
    n = 4 * 1023
    xi = a * ca[np.arange(n) // 4]
    buf = np.zeros(2 * n, np.int8)
    buf[0::2] = xi
    lags = list(range(-3, 4)) + [100, 511, 1000]
    taps = np.array([k * TWO32 for k in lags], np.int64)
    st = _fresh(0, 0, 0, TWO32 // 4, len(taps))
    d, dn = oracle.correlate_lut(1, buf.view(np.uint8), n, pb, taps, 1, st)
    assert len(d) == 1 and dn[0] == n
    cb = oracle.ca_code(pb).astype(np.int64)
    for j, k in enumerate(lags):
        r = int(np.sum(ca * np.roll(cb, -k)))  # sum_c C_a[c] C_b[c+k]
        assert d[0, j, 0] == 4 * 24 * a * r
        assert d[0, j, 1] == 0
        if pa == pb and k == 0:
            assert r == 1023
        else:
            assert r in (-65, -1, 63)


def test_early_late_on_noiseless_aligned_code():
    # E/P on a noiseless aligned code: the +-1/2-chip replicas disagree with the
    # prompt only on the half chip next to each chip transition.
    prn = 11
    c = oracle.ca_code(prn).astype(np.int64)
    spc = 16
    n = spc * 1023
    x = 10 * c[np.arange(n) // spc]
    buf = np.zeros(2 * n, np.int8)
    buf[0::2] = x
    st = _fresh(0, 0, 0, TWO32 // spc, 3)
    d, _ = oracle.correlate_lut(1, buf.view(np.uint8), n, prn, oracle.EPL_TAPS_Q32, 1, st)
    E, P, L = d[0, :, 0]
    transitions = int(np.sum(c != np.roll(c, -1)))
    assert P == 240 * n
    assert E == L == 240 * (n - 2 * (spc // 2) * transitions)
    assert abs(E / P - (1 - transitions / 1023)) < 1e-12


def test_int32_range_is_reported():
    # 1024 samples per chip, x = 127*C aligned: 3048 per sample, past 2^31 at 704,556
    n = 720_000
    c = oracle.ca_code(1).astype(np.int64)
    buf = (127 * c[np.arange(n) // 1024]).astype(np.int8).view(np.uint8)
    st = _fresh(0, 0, 0, TWO32 // 1024, 1)
    with pytest.raises(OverflowError):
        oracle.correlate_lut(0, buf, n, 1, [0], 1, st)
    st = _fresh(0, 0, 0, TWO32 // 1024, 1)
    oracle.correlate_lut(0, buf[:704_555], 704_555, 1, [0], 1, st)
    assert st.acc[0] == 3048 * 704_555


# ---------------------------------------------------------------- FP64 form
def _geom(phi0, f, N):
    """sum_{n<N} exp(j 2 pi (phi0 + n f)), closed form."""
    z = np.exp(2j * np.pi * f)
    return np.exp(2j * np.pi * phi0) * (1 - z ** N) / (1 - z)


@pytest.mark.parametrize("f,phi0", [(0.25 + 1e-4, 0.1), (-0.0371, 0.77), (0.123456789, 0.0)])
def test_f64_closed_form_on_noiseless_code(f, phi0):
    # x = K*C (real int8): the aligned prompt sees K*cos and -K*sin of the carrier
    prn = 4
    c = oracle.ca_code(prn).astype(np.int64)
    K = 7
    spc = 4
    n = spc * 1023
    buf = (K * c[np.arange(n) // spc]).astype(np.int8).view(np.uint8)
    st = oracle.OracleState(0, 0, 0, TWO32 // spc, 1, carr_phase_f=phi0, carr_freq_f=f)
    d, _ = oracle.correlate_f64(0, buf, n, prn, [0], 1, st)
    S = K * _geom(phi0, f, n)
    assert abs(d[0, 0, 0] - S.real) < 1e-9 * n * K
    assert abs(d[0, 0, 1] + S.imag) < 1e-9 * n * K
    # complex input j*K*C: wI = x_q*s, wQ = x_q*c
    buf2 = np.zeros(2 * n, np.int8)
    buf2[1::2] = K * c[np.arange(n) // spc]
    st2 = oracle.OracleState(0, 0, 0, TWO32 // spc, 1, carr_phase_f=phi0, carr_freq_f=f)
    d2, _ = oracle.correlate_f64(1, buf2.view(np.uint8), n, prn, [0], 1, st2)
    assert abs(d2[0, 0, 0] - S.imag) < 1e-9 * n * K
    assert abs(d2[0, 0, 1] - S.real) < 1e-9 * n * K
    assert abs(st.carr_phase_f - ((phi0 + n * f) % 1.0)) < 1e-9


def test_lut_path_within_quantisation_bound_of_f64_path():
    # |LUT(l) - 24 e^{j theta}| <= 0.5*sqrt(2) (rounding) + 24*pi/256 (phase bin)
    rng = np.random.default_rng(3)
    n = 20000
    buf = rng.integers(0, 256, size=2 * n, dtype=np.uint8)
    cp, cs = 0x12345678, 0x0ABCDEF1
    st_i = _fresh(cp, cs, 5 * TWO32, TWO32 // 5, 3)
    st_f = oracle.OracleState(cp, cs, 5 * TWO32, TWO32 // 5, 3,
                              carr_phase_f=cp / TWO32, carr_freq_f=cs / TWO32)
    di, ni = oracle.correlate_lut(1, buf, n, 2, oracle.EPL_TAPS_Q32, 1, st_i)
    df, nf = oracle.correlate_f64(1, buf, n, 2, oracle.EPL_TAPS_Q32, 1, st_f)
    assert np.array_equal(ni, nf)
    xabs = np.abs(buf.view(np.int8).astype(np.float64))
    bound = (0.5 * np.sqrt(2) + 24 * np.pi / 256) * (xabs[0::2] + xabs[1::2]).sum()
    assert np.all(np.abs(di - 24 * df) <= bound)
    assert np.all(np.abs(st_i.acc - 24 * st_f.acc) <= bound)
