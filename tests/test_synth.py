"""The seeded generator: its codes, its determinism and its C/N0 calibration."""
import math

import numpy as np
import pytest

import oracle
from paper_1907_00463_amd import synth

TWO32 = 1 << 32


@pytest.mark.parametrize("prn", range(1, 33))
def test_generator_codes_equal_oracle_codes(prn):
    # two independent constructions (G2 delay here, G2 phase-selector taps there)
    assert np.array_equal(synth.ca_chips(prn), oracle.ca_code(prn))


def test_deterministic_and_thread_count_free():
    st, _, rng = synth.workload_single_channel(seconds=0.05)
    a = synth.synth_samples(st, rng, chunk=50_000, threads=1)
    st, _, rng = synth.workload_single_channel(seconds=0.05)
    b = synth.synth_samples(st, rng, chunk=50_000, threads=4)
    assert np.array_equal(a, b)
    assert a.dtype == np.uint8 and a.size == st.n


def test_two_bit_packing_and_levels():
    st, _, rng = synth.workload_twelve_channels(seconds=0.01)
    buf = synth.synth_samples(st, rng)
    assert buf.size == st.n // 4
    codes = np.stack([(buf >> (2 * j)) & 3 for j in range(4)], axis=1).ravel()
    frac = np.bincount(codes, minlength=4) / codes.size
    # thresholds 0, +-1 sigma on unit noise: P(|x| > 1) = 0.3173
    assert abs(frac[0] + frac[3] - 0.3173) < 0.01
    assert abs(frac[0] - frac[3]) < 0.01


def test_two_bit_complex_packing_and_levels():
    st, chans, rng = synth.workload_iq2(seconds=0.01)
    buf = synth.synth_samples(st, rng)
    assert st.fmt == synth.I2_IQ and buf.size == st.n // 2
    codes = np.stack([(buf >> (2 * j)) & 3 for j in range(4)], axis=1).ravel()
    # each component is noise of variance 1/2 plus half of the satellites'
    # power (complex amplitude sqrt(C/N0 / fs) each), against 0 and
    # +-sqrt(1/2): P(|x| > sqrt(1/2)) = erfc(sqrt(1/2) / (sqrt(2) sigma))
    p_sig = sum(10 ** (s.cn0_dbhz / 10) / st.fs for s in st.sats)
    sigma = math.sqrt(0.5 + p_sig / 2)
    want = math.erfc(math.sqrt(0.5) / (math.sqrt(2) * sigma))
    for comp in (codes[0::2], codes[1::2]):  # I codes, Q codes
        frac = np.bincount(comp, minlength=4) / comp.size
        assert abs(frac[0] + frac[3] - want) < 0.006
        assert abs(frac[0] - frac[3]) < 0.01


def test_cn0_recovered_from_prompt_dumps():
    # single-channel workload: 45 dB-Hz, 1000 one-millisecond dumps
    st, chans, rng = synth.workload_single_channel(seconds=1.0)
    buf = synth.synth_samples(st, rng)
    ch = chans[0]
    cp, cs, kp, ks = oracle.nco_words(st.fs, ch.carr_hz, ch.carr_phase0, ch.code_rate,
                                      ch.code_phase0, 1)
    sig = oracle.OracleState(cp, cs, kp, ks, 3)
    d, dn = oracle.correlate_lut(0, buf, st.n, ch.prn, oracle.EPL_TAPS_Q32, 1, sig)
    assert len(d) == 1000  # a short head dump plus 999 full ones
    assert dn[0] == 2891 and np.all(dn[1:] >= 4091)
    noise = oracle.OracleState(cp, cs, kp, ks, 3)
    dz, _ = oracle.correlate_lut(0, buf, st.n, 30, oracle.EPL_TAPS_Q32, 1, noise)
    full = slice(1, None)
    P = d[full, 1, 0].astype(np.float64) + 1j * d[full, 1, 1]
    Z = dz[full, 1, 0].astype(np.float64) + 1j * dz[full, 1, 1]
    sigma2 = np.mean(np.abs(Z) ** 2) / 2.0
    snr = (np.mean(np.abs(P) ** 2) - 2 * sigma2) / (2 * sigma2)
    cn0 = 10 * math.log10(snr / 1e-3)
    assert abs(cn0 - 45.0) < 0.5
    # open loop at the true parameters: the prompt sits on the I arm, nav bits flip its sign
    assert np.mean(np.abs(P.real)) > 5 * np.mean(np.abs(P.imag))
