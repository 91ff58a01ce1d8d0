"""Pins of the acquisition oracle (parallel code-phase search), each against
something other than its FFT route: the correlator oracle's own sums at each
code phase (brute force on tiny inputs), the three-valued correlation of Gold
codes, and detection of the synthetic signals' satellites at their Doppler
and code phase."""
import numpy as np
import pytest

import oracle
from oracle import acquire as A


def _correlator_y(fmt, buf, R, step, prn, b, L, tau, total):
    """Y of block b at code phase tau through the correlator oracle: one E/P/L
    channel with only a prompt tap, its window longer than the buffer, so the
    block's sum stays in the open dump."""
    T = total // (1023 * R) + 4
    st = oracle.OracleState((b * L * step) % (1 << 32), step, tau * ((1 << 32) // R),
                            (1 << 32) // R, 1)
    sub = _slice(fmt, buf, b * L, L)
    d, nd = oracle.correlate_lut(fmt, sub, L, prn, np.array([0], np.int64), T, st)
    assert len(nd) == 0
    return int(st.acc[0]), int(st.acc[1])


def _slice(fmt, buf, n0, n):
    if fmt == oracle.I2_REAL:
        assert n0 % 4 == 0
        return buf[n0 // 4:(n0 + n + 3) // 4]
    k = 2 if fmt == oracle.I8_IQ else 1
    return buf[k * n0:k * (n0 + n)]


@pytest.mark.parametrize("fmt,R,Mc,Knc", [(oracle.I8_REAL, 1, 1, 2), (oracle.I2_REAL, 2, 2, 2),
                                          (oracle.I8_IQ, 1, 2, 2), (oracle.I2_REAL, 1, 3, 1)])
def test_search_equals_the_correlator_at_every_code_phase(fmt, R, Mc, Knc):
    rng = np.random.default_rng(10 * R + fmt + Mc)
    N = 1023 * R
    L = Mc * N
    nbytes = {oracle.I8_REAL: Knc * L, oracle.I8_IQ: 2 * Knc * L, oracle.I2_REAL: Knc * L // 4 + 1}
    buf = rng.integers(0, 256, nbytes[fmt], dtype=np.uint8)
    if_hz = 0.25 * R * 1.023e6 if fmt != oracle.I8_IQ else 0.0
    prns, bins = [5, 29], 3
    P = A.search(fmt, buf, R, if_hz, -1500.0, 1500.0, bins, prns, Mc, Knc)
    steps = A.bin_steps(R, if_hz, -1500.0, 1500.0, bins)
    # every code phase of one (PRN, bin), and a sample of the others
    for k, prn in enumerate(prns):
        for d in range(bins):
            taus = range(N) if (k, d) == (0, 1) else rng.integers(0, N, 12)
            for tau in taus:
                want = 0
                for b in range(Knc):
                    yi, yq = _correlator_y(fmt, buf, R, int(steps[d]), prn, b, L, int(tau),
                                           Knc * L)
                    want += yi * yi + yq * yq
                assert int(P[k, d, tau]) == want, (prn, d, tau)


def test_gold_code_correlations_are_three_valued():
    # at one sample per chip, zero carrier and a noise-free code as the input,
    # the carrier table's entry 0 is (24, 0), so Y = 24 x the periodic
    # correlation of two Gold codes: 1023 at the code's own phase, and
    # otherwise only -1, -65 and 63 (auto- and cross-correlation of the
    # length-1023 Gold family)
    lc, ls = oracle.lut()
    assert (int(lc[0]), int(ls[0])) == (24, 0)
    t0 = 417
    x = np.roll(oracle.ca_code(13).astype(np.int8), -t0)     # x[n] = C13[(n + t0) mod 1023]
    buf = x.view(np.uint8)
    P = A.search(oracle.I8_REAL, buf, 1, 0.0, 0.0, 1.0, 1, [13, 2, 30], 1, 1)
    allowed = {24 * 24 * v * v for v in (1, 65, 63)}
    auto = P[0, 0]
    assert int(np.argmax(auto)) == t0 and int(auto[t0]) == (24 * 1023) ** 2
    assert set(int(v) for v in np.delete(auto, t0)) <= allowed
    for k in (1, 2):
        assert set(int(v) for v in P[k, 0]) <= allowed
    det = A.detect(P, 1, 0.0, 1.0, 2.5)
    assert det[0]["tau"] == t0 and det[0]["acquired"]
    assert det[0]["second"] == (24 * 65) ** 2
    assert det[0]["metric"] == pytest.approx(1023 ** 2 / 65 ** 2, rel=1e-15)
    assert not det[1]["acquired"] and not det[2]["acquired"]


def test_detect_tie_and_exclusion_rules():
    # ties go to the lower bin and then the lower tau; the second peak skips
    # the peak's chip and its two neighbours (circularly) in the peak's bin
    R = 2
    P = np.ones((1, 3, 1023 * R), np.uint64)
    P[0, 1, 10] = P[0, 2, 3] = P[0, 1, 900] = 50
    P[0, 1, 0] = 40        # chip 0: five chips away, counts
    P[0, 1, 8] = 45        # chip 4: excluded
    P[0, 1, 13] = 44       # chip 6: excluded
    P[0, 1, 14] = 30       # chip 7: counts
    P[0, 0, 5] = 49        # another bin: ignored for the second peak
    d = A.detect(P, R, -100.0, 50.0, 1.2)[0]
    assert (d["bin"], d["tau"], d["peak"]) == (1, 10, 50)
    assert d["second"] == 50                 # tau 900 (chip 450) ties the peak
    assert d["metric"] == 1.0 and not d["acquired"]
    P[0, 1, 900] = 1
    d = A.detect(P, R, -100.0, 50.0, 1.2)[0]
    assert d["second"] == 40 and d["metric"] == 50 / 40 and d["acquired"]
    assert d["doppler_hz"] == -50.0 and d["code_phase_chips"] == 5.0
    # wrap-around: a peak at chip 0 excludes chip 1022
    P = np.ones((1, 1, 1023 * R), np.uint64)
    P[0, 0, 1] = 9
    P[0, 0, 2045] = 8      # chip 1022
    P[0, 0, 4] = 7         # chip 2
    assert A.detect(P, R, 0.0, 1.0, 1.0)[0]["second"] == 7


def test_search_finds_the_single_channel_satellite():
    # PRN 7 at +1.5 kHz and 300.25 chips (int8, 4.092 MHz = 4 samples per
    # chip): the peak is in the 1.5 kHz bin at tau = 4 x 300.25 = 1201 (the
    # code Doppler moves it by 0.002 chip over 2 ms); absent PRNs stay below
    # the threshold
    from paper_1907_00463_amd import synth
    st, chans, rng = synth.workload_single_channel(seconds=0.003)
    buf = synth.synth_samples(st, rng)
    P = A.search(st.fmt, buf, 4, st.if_hz, -5000.0, 500.0, 21, [7, 3, 19], 1, 2)
    det = A.detect(P, 4, -5000.0, 500.0, 2.5)
    assert det[0]["acquired"] and det[0]["bin"] == 13 and det[0]["doppler_hz"] == 1500.0
    assert abs(det[0]["tau"] - 1201) <= 1
    assert not det[1]["acquired"] and not det[2]["acquired"]


def test_search_finds_twelve_channel_satellites():
    # the 2-bit 16.368 MHz stream (16 samples per chip): its three strongest
    # satellites peak within a bin step of their Doppler (500 Hz bins over
    # 1 ms lose under 1 dB, so with noise a neighbour of the nearest bin can
    # win) and within 2 samples of 16 x their code phase; a PRN not in the
    # stream is not acquired
    from paper_1907_00463_amd import synth
    st, chans, rng = synth.workload_twelve_channels(seconds=0.0021)
    buf = synth.synth_samples(st, rng)
    strong = sorted(range(12), key=lambda i: -st.sats[i].cn0_dbhz)[:3]
    prns = [st.sats[i].prn for i in strong]
    absent = next(p for p in range(1, 33) if p not in [s.prn for s in st.sats])
    P = A.search(st.fmt, buf, 16, st.if_hz, -5000.0, 500.0, 21, prns + [absent], 1, 2)
    det = A.detect(P, 16, -5000.0, 500.0, 2.5)
    for k, i in enumerate(strong):
        s = st.sats[i]
        assert det[k]["acquired"], (s.prn, det[k])
        assert abs(det[k]["doppler_hz"] - s.doppler_hz) < 500.0
        dtau = (det[k]["tau"] - 16 * s.code_phase0) % 16368
        assert min(dtau, 16368 - dtau) <= 2.0, (s.prn, det[k]["tau"], 16 * s.code_phase0)
    assert not det[3]["acquired"]
