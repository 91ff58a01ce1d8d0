"""Pins of the oracle's lock metrics and bit synchronisation (Sec. 3.6,
channel health: C/N0 by the moments estimator and the carrier lock ratio;
Sec. 3.1: 20 code periods per navigation bit), each against a closed form,
a constructed input with a known answer, or the synthetic signal's own
navigation bits."""
import math

import numpy as np
import pytest

import oracle


def _prompts(i, q):
    return np.stack([np.asarray(i, np.int64), np.asarray(q, np.int64)], axis=1).astype(np.int32)


def test_m2m4_two_level_closed_form():
    # powers alternating between p1 and p2: M2 = (p1 + p2) / 2, M4 = (p1^2 +
    # p2^2) / 2, so 2 M2^2 - M4 = p1 p2 and SNR = sqrt(p1 p2) / (M2 - sqrt(p1 p2))
    for (i1, q1), (i2, q2), T in [((2, 0), (1, 0), 1e-3), ((3, 4), (0, -1), 1e-3),
                                  ((300, 0), (-100, 0), 4e-3), ((7, 1), (5, 4), 2e-2)]:
        p1, p2 = i1 * i1 + q1 * q1, i2 * i2 + q2 * q2
        i = [i1, i2] * 10
        q = [q1, q2] * 10
        m = oracle.lock_metrics(_prompts(i, q), K=20, T=T)
        a = math.sqrt(p1 * p2)
        want = 10.0 * math.log10(a / ((p1 + p2) / 2.0 - a) / T)
        assert len(m["cn0"]) == 1
        assert m["cn0"][0] == pytest.approx(want, rel=1e-12)
    # 2, 1 at T = 1 ms: SNR 4 -> 10 log10(4000) dB-Hz
    m = oracle.lock_metrics(_prompts([2, 1] * 10, [0] * 20), K=20, T=1e-3)
    assert m["cn0"][0] == pytest.approx(36.02059991327962, rel=1e-13)


def test_m2m4_degenerate_windows_are_nan():
    # constant power: M4 = M2^2, A = M2, no noise power left -> NaN; all
    # zero: 2 M2^2 - M4 = 0 -> NaN; one spike among zeros: 2 M2^2 < M4 -> NaN
    for i in ([5] * 20, [0] * 20, [0] * 19 + [9]):
        m = oracle.lock_metrics(_prompts(i, [0] * 20), K=20)
        assert math.isnan(m["cn0"][0])
    # the window count is floor(n / K); a short tail gives no window
    m = oracle.lock_metrics(_prompts([1, 2] * 25, [0] * 50), K=20)
    assert len(m["cn0"]) == 2 and len(m["lock"]) == 2
    assert len(oracle.lock_metrics(_prompts([1] * 19, [0] * 19), K=20)["cn0"]) == 0


@pytest.mark.parametrize("cn0", [35.0, 42.0, 48.0])
def test_m2m4_recovers_the_snr_of_gaussian_dumps(cn0):
    # I = A b_k + n_I, Q = n_Q with n ~ N(0, s^2) per component: the signal
    # to noise power ratio is A^2 / (2 s^2) per dump, C/N0 = that / T.  The
    # moments estimator is consistent: over windows of 1000 dumps the median
    # lies within 0.25 dB; over windows of 20 (its small-sample bias is
    # upward, a few tenths of a dB) within 1 dB
    rng = np.random.default_rng(int(cn0))
    T, s = 1e-3, 400.0
    A = math.sqrt(2.0 * s * s * 10.0 ** (cn0 / 10.0) * T)
    n = 20000
    b = np.repeat(rng.choice([-1, 1], n // 20), 20)
    i = np.rint(A * b + rng.normal(0, s, n))
    q = np.rint(rng.normal(0, s, n))
    for K, tol in ((1000, 0.25), (20, 1.0)):
        m = oracle.lock_metrics(_prompts(i, q), K=K, T=T)
        assert len(m["cn0"]) == n // K
        est = m["cn0"][np.isfinite(m["cn0"])]
        assert len(est) > 0.95 * (n // K)
        assert abs(np.median(est) - cn0) < tol, K


@pytest.mark.parametrize("phi_deg", [0.0, 10.0, 30.0, 45.0, 60.0, 90.0, 135.0, -20.0])
def test_lock_ratio_is_cos_two_phi(phi_deg):
    # noiseless prompts A b_k (cos phi, sin phi): (I^2 - Q^2) / (I^2 + Q^2) =
    # cos 2 phi whatever the bits; rounding to integers moves it by < 1e-5
    rng = np.random.default_rng(4)
    phi = math.radians(phi_deg)
    A = 2.0e6
    b = rng.choice([-1, 1], 40)
    m = oracle.lock_metrics(_prompts(np.rint(A * b * math.cos(phi)), np.rint(A * b * math.sin(phi))),
                            K=20, lock_min=0.5)
    assert np.allclose(m["lock"], math.cos(2 * phi), atol=1e-5)
    want_fail = 2 if math.cos(2 * phi) < 0.5 - 1e-5 else 0
    assert m["lock_fails"] == want_fail
    # an all-zero window gives 0 and counts as a failure for lock_min > 0
    z = oracle.lock_metrics(np.zeros((20, 2), np.int32), K=20, lock_min=0.5)
    assert z["lock"][0] == 0.0 and z["lock_fails"] == 1


@pytest.mark.parametrize("edge,phase", [(0, 0), (7, 0), (13, 5), (19, 19), (3, 41)])
def test_bit_edge_and_bits_on_constructed_prompts(edge, phase):
    # dump k belongs to bit floor((k + phase - edge) / 20): the transitions
    # all fall on position `edge` of the cycle, the bits come back in order,
    # and a partial bit at either end is dropped
    rng = np.random.default_rng(100 + edge)
    n = 20 * 30 + 11
    k = np.arange(n)
    bit_of = (k + phase - edge) // 20
    nav = rng.choice([-1, 1], bit_of.max() - bit_of.min() + 1)
    b = nav[bit_of - bit_of.min()]
    i = np.rint(b * 1000 + rng.normal(0, 100, n))
    q = np.rint(rng.normal(0, 100, n))
    m = oracle.lock_metrics(_prompts(i, q), K=20, phase=phase)
    assert m["edge"] == edge
    assert int(m["hist"][edge]) > 0
    assert int(np.sum(m["hist"])) == int(np.sum((i[1:] < 0) != (i[:-1] < 0)))
    first = int(np.argmax((k + phase) % 20 == edge))     # first dump on an edge position
    whole = [j for j in range(bit_of.min(), bit_of.max() + 1)
             if np.sum(bit_of == j) == 20 and np.argmax(bit_of == j) >= first]
    want = np.array([1 if nav[j - bit_of.min()] < 0 else 0 for j in whole], np.uint8)
    assert np.array_equal(m["bits"], want)


def test_bit_edge_ties_and_no_transitions():
    # no sign change: an all-zero histogram, edge 0; a tie goes to the lower
    # position; zero counts as positive
    m = oracle.lock_metrics(_prompts([5] * 45, [0] * 45))
    assert not np.any(m["hist"]) and m["edge"] == 0 and len(m["bits"]) == 2
    assert list(m["bits"]) == [0, 0]
    i = [1] * 60
    i[7] = -1                 # changes at k = 7 and k = 8
    m = oracle.lock_metrics(_prompts(i, [0] * 60))
    assert m["hist"][7] == 1 and m["hist"][8] == 1 and m["edge"] == 7
    i = [-1] * 4 + [0] * 36   # -1 -> 0 is a change (zero is positive)
    m = oracle.lock_metrics(_prompts(i, [0] * 40))
    assert m["hist"][4] == 1 and m["edge"] == 4


def test_tracked_signal_gives_its_navigation_bits():
    # PRN 7 at 45 dB-Hz tracked by the oracle's loops for 2 s from a 30 Hz and
    # 0.2 chip offset: dump k is code period k of the stream (the first dump
    # closes the period the stream starts in), so bit edges fall on position
    # 0 and the bits after the loops settle equal the transmitted ones up to
    # the sign the PLL locks with; C/N0 comes out near 45 dB-Hz
    from paper_1907_00463_amd import synth
    st, chans, rng = synth.workload_single_channel(seconds=2.0, seed=1001)
    ch = chans[0]
    buf = synth.synth_samples(st, rng)
    cp, cs, kp, ks = oracle.nco_words(st.fs, ch.carr_hz + 30.0, ch.carr_phase0, ch.code_rate,
                                      ch.code_phase0 + 0.2, 1)
    ts = oracle.track_state(oracle.OracleState(cp, cs, kp, ks, 3), ch.carr_hz + 30.0,
                            ch.code_rate)
    prm = oracle.LoopParams(fs=st.fs, if_hz=st.if_hz)
    rows, _ = oracle.track(st.fmt, buf, st.n, ch.prn, 1, prm, ts)
    assert len(rows) in (1999, 2000)
    m = oracle.lock_metrics(rows[:, 2:4], K=20, T=1e-3, lock_min=0.8)
    assert m["edge"] == 0
    nav = st.sats[0].nav_bits
    got = m["bits"].astype(np.int64)
    want = (nav[:len(got)] < 0).astype(np.int64)
    settled = slice(25, len(got))                  # after the first half second
    agree = np.mean(got[settled] == want[settled])
    assert agree in (0.0, 1.0)
    late = m["cn0"][50:]
    assert abs(np.median(late) - 45.0) < 2.0
    assert np.all(m["lock"][50:] > 0.8)
