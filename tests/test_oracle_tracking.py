"""Pins of the oracle's closed tracking loops (Table 3: 2nd-order DLL with the
normalised early-minus-late envelope discriminator and carrier aiding,
2nd-order PLL with an atan discriminator, 1st-order FLL with an atan2
discriminator), each against something other than the oracle itself."""
import decimal
import math

import numpy as np
import pytest

import oracle


def _atan_decimal(x: decimal.Decimal) -> decimal.Decimal:
    """atan(x) for |x| <= 1/2 by its Taylor series, or pi/4 (Machin) for x = 1."""
    if x == 1:
        return 4 * _atan_decimal(decimal.Decimal(1) / 5) - _atan_decimal(decimal.Decimal(1) / 239)
    s, term, k = decimal.Decimal(0), x, 0
    x2 = x * x
    while True:
        t = term / (2 * k + 1)
        if abs(t) < decimal.Decimal(10) ** -45:
            return s
        s += t if k % 2 == 0 else -t
        term *= x2
        k += 1


def test_cordic_table_is_exactly_rounded():
    # round(atan(2^-i) * 2^30), the angles of Volder's CORDIC, against
    # 50-digit decimal arithmetic
    decimal.getcontext().prec = 60
    tab = oracle.cordic_table()
    for i in range(31):
        a = _atan_decimal(decimal.Decimal(1) / (2 ** i)) * (2 ** 30)
        exact = int(a.to_integral_value(rounding=decimal.ROUND_HALF_EVEN))
        assert int(tab[i]) == exact, i


def test_cordic_atan2_within_its_error_bound():
    # vectoring CORDIC after 31 rotations on a vector scaled into [2^39,
    # 2^40): the residual angle is below atan(2^-30) and each of the 31 table
    # angles is off by at most 1/2 unit, so |error| < 17 units of 2^-30 rad
    rng = np.random.default_rng(3)
    cases = [(0, 1), (1, 1), (-1, 1), (1, 0), (-1, 0), (5, 10 ** 15), (-(2 ** 62), 3),
             (2 ** 31 - 1, 2 ** 31 - 1), (7, 2 ** 62)]
    cases += [(int(y), int(x)) for y, x in zip(rng.integers(-2 ** 40, 2 ** 40, 300),
                                               rng.integers(0, 2 ** 40, 300))]
    cases += [(int(y), int(x)) for y, x in zip(rng.integers(-100, 100, 300),
                                               rng.integers(0, 100, 300))]
    for y, x in cases:
        if x == 0 and y == 0:
            continue
        got = oracle.cordic_atan2(y, x)
        assert abs(got - math.atan2(y, x) * 2 ** 30) < 17, (y, x)
    assert oracle.cordic_atan2(0, 0) == 0
    with pytest.raises(ValueError):
        oracle.cordic_atan2(1, -1)


@pytest.mark.parametrize("bw,zeta,k", [(2.0, 0.7, 1.0), (25.0, 0.7, 0.25), (10.0, 1.0, 1.0),
                                       (0.5, 0.5, 2.0)])
def test_loop_coefficients_give_the_noise_bandwidth(bw, zeta, k):
    # a 2nd-order loop with natural frequency wn and damping z has the
    # one-sided noise bandwidth B = (wn / 2) (z + 1 / (4 z)) (Gardner); the
    # filter's tau1 = k / wn^2 and tau2 = 2 z / wn must give B back
    tau1, tau2 = oracle.loop_coefficients(bw, zeta, k)
    wn = math.sqrt(k / tau1)
    z = tau2 * wn / 2.0
    assert z == pytest.approx(zeta, rel=1e-12)
    assert (wn / 2.0) * (z + 1.0 / (4.0 * z)) == pytest.approx(bw, rel=1e-12)


def _single(seconds=1.0, seed=1001):
    from paper_1907_00463_amd import synth
    st, chans, rng = synth.workload_single_channel(seconds=seconds, seed=seed)
    return st, chans[0], synth.synth_samples(st, rng)


def _start(st, ch, dcarr, dcode):
    cp, cs, kp, ks = oracle.nco_words(st.fs, ch.carr_hz + dcarr, ch.carr_phase0, ch.code_rate,
                                      ch.code_phase0 + dcode, 1)
    return oracle.track_state(oracle.OracleState(cp, cs, kp, ks, 3), ch.carr_hz + dcarr,
                              ch.code_rate)


@pytest.mark.parametrize("dcarr,dcode", [(40.0, 0.2), (-60.0, -0.3), (0.0, 0.0)])
def test_loops_converge_from_offsets(dcarr, dcode):
    # PRN 7 at 45 dB-Hz, +1.5 kHz, int8 at 4.092 MHz: from a 40-60 Hz carrier
    # and 0.2-0.3 chip code offset the loops settle within 0.3 s; over the
    # last half second the code error stays below 0.15 chip (with 4 samples
    # per chip the early-minus-late discriminator cannot tell offsets within
    # +-1/8 chip apart), the mean carrier error below 3 Hz, and the prompt
    # phase within 20 degrees of 0 or 180 (navigation bits flip the prompt)
    st, ch, buf = _single()
    ts = _start(st, ch, dcarr, dcode)
    prm = oracle.LoopParams(fs=st.fs, if_hz=st.if_hz)
    blk = 4092 * 50
    code_err, carr = [], []
    rows_all = []
    for b in range(0, st.n, blk):
        n = min(blk, st.n - b)
        rows, _ = oracle.track(st.fmt, buf[b:b + n], n, ch.prn, 1, prm, ts)
        rows_all.append(rows)
        t = (b + n) / st.fs
        if t > 0.5:
            true_p = (ch.code_phase0 + ch.code_rate * (b + n) / st.fs) % 1023
            trk_p = (ts.words.code_phase / 2 ** 32) % 1023
            code_err.append((trk_p - true_p + 511.5) % 1023 - 511.5)
            carr.append(ts.ls[0] - ch.carr_hz)
    rows = np.concatenate(rows_all)
    assert max(abs(e) for e in code_err) < 0.15
    assert abs(np.mean(carr)) < 3.0
    ph = np.degrees(np.arctan2(rows[500:, 3], rows[500:, 2]))
    dev = np.minimum(np.abs(ph), 180.0 - np.abs(ph))
    assert np.percentile(dev, 95) < 20.0


def test_tracking_is_independent_of_block_splits():
    # the dump rule closes a dump when the code phase reaches the window end,
    # before the next sample or at the end of a block, so any split of the
    # stream gives the same dumps, steps and loop state, bit for bit
    st, ch, buf = _single(seconds=0.3)
    prm = oracle.LoopParams(fs=st.fs, if_hz=st.if_hz)
    whole = _start(st, ch, 25.0, 0.1)
    r0, d0 = oracle.track(st.fmt, buf, st.n, ch.prn, 1, prm, whole)
    rng = np.random.default_rng(9)
    cuts = np.sort(rng.choice(np.arange(1, st.n), size=40, replace=False))
    cuts = np.concatenate([[0], cuts, [st.n]])
    # a cut exactly on a dump end as well
    cuts = np.unique(np.concatenate([cuts, [int(np.sum(d0[:7]))]]))
    split = _start(st, ch, 25.0, 0.1)
    rs, ds = [], []
    for a, b in zip(cuts[:-1], cuts[1:]):
        r, d = oracle.track(st.fmt, buf[a:b], int(b - a), ch.prn, 1, prm, split)
        rs.append(r)
        ds.append(d)
    assert np.array_equal(np.concatenate(rs), r0)
    assert np.array_equal(np.concatenate(ds), d0)
    assert split.ls.tobytes() == whole.ls.tobytes()
    assert np.array_equal(split.is_, whole.is_)
    assert (split.words.carr_phase, split.words.carr_step, split.words.code_phase,
            split.words.code_step, split.words.acc_n) == (
        whole.words.carr_phase, whole.words.carr_step, whole.words.code_phase,
        whole.words.code_step, whole.words.acc_n)


def test_first_dump_equals_the_open_loop_correlator():
    # before the first dump closes, no loop has acted: the first row and the
    # open dump equal the fixed-NCO correlator's
    st, ch, buf = _single(seconds=0.01)
    ts = _start(st, ch, 10.0, 0.05)
    w = ts.words.copy()
    prm = oracle.LoopParams(fs=st.fs, if_hz=st.if_hz)
    n = 6000
    rows, dn = oracle.track(st.fmt, buf, n, ch.prn, 1, prm, ts)
    d, dn2 = oracle.correlate_lut(st.fmt, buf, int(dn[0]), ch.prn, oracle.EPL_TAPS_Q32, 1, w)
    assert np.array_equal(rows[0, :6], d[0].reshape(-1))
    assert rows[0, 6] == np.int32(np.uint32(w.carr_step))
    assert int(dn[0]) == int(dn2[0])


# ---------------------------------------------------------------------------
# Loop dynamics against the closed forms of loop theory.  The input is a
# noiseless complex signal (int8 I then Q at 5 MHz, the paper's format and
# rate, Sec. 4) whose carrier phase and code phase are given functions of
# time, so that every discriminator reads the true error: the PLL's
# atan(Q/I) gives the dump's mean phase error (a linear phase across the
# dump sums to a real multiple of its mid-dump value), the FLL's atan2 gives
# the rotation between consecutive prompts, and the normalised early-minus-
# late envelope gives 2*(1024/1022)*delta on the main peak of the C/A
# autocorrelation (taps at +-1/2 chip, |delta| < 1/2 chip).  The IF keeps
# the carrier table's quantisation averaging out over a dump.
# ---------------------------------------------------------------------------
FS = 5.0e6
IF_HZ = 1234567.0
F_L1 = 1575.42e6
CHIP_RATE = 1.023e6


def _iq_signal(n, prn, theta, code, amp=100.0):
    """amp * C[floor(code(t)) mod 1023] * exp(j 2 pi theta(t)) at FS, rounded
    to int8, I then Q (theta in cycles, code in chips)."""
    from paper_1907_00463_amd import synth
    t = np.arange(n, dtype=np.float64) / FS
    chips = synth.ca_chips(prn).astype(np.float64)
    c = chips[np.floor(code(t)).astype(np.int64) % 1023]
    ph = theta(t)
    x = amp * c * np.exp(2j * np.pi * (ph - np.floor(ph)))
    out = np.empty(2 * n, np.int8)
    out[0::2] = np.clip(np.round(x.real), -127, 127)
    out[1::2] = np.clip(np.round(x.imag), -127, 127)
    return out.view(np.uint8)


def _run_loops(buf, n, prm, carr_hz, code_chips, code_cps, block=25000):
    """oracle.track over the signal in blocks; returns the rows, the dump
    sample counts, and per block its end sample, the replica code phase
    there (chips) and the loop state."""
    cp, cs, kp, ks = oracle.nco_words(FS, carr_hz, 0.0, code_cps, code_chips, 1)
    ts = oracle.track_state(oracle.OracleState(cp, cs, kp, ks, 3), carr_hz, code_cps)
    rows, dn, ends, code, ls = [], [], [], [], []
    for b in range(0, n, block):
        m = min(block, n - b)
        r, d = oracle.track(oracle.I8_IQ, buf[2 * b: 2 * (b + m)], m, 7, 1, prm, ts)
        rows.append(r)
        dn.append(d)
        ends.append(b + m)
        code.append(ts.words.code_phase / 2.0 ** 32)
        ls.append(ts.ls.copy())
    return (np.concatenate(rows), np.concatenate(dn), np.array(ends), np.array(code),
            np.array(ls))


def _second_order_error(t, delta, w, z):
    """Phase error of a type-2 second-order loop (natural frequency w, damping
    z < 1) after a phase step delta at t = 0 from rest: the inverse Laplace
    transform of delta * s / (s^2 + 2 z w s + w^2) (Gardner)."""
    wd = w * math.sqrt(1.0 - z * z)
    return delta * np.exp(-z * w * t) * (np.cos(wd * t) - z / math.sqrt(1.0 - z * z) *
                                         np.sin(wd * t))


@pytest.mark.parametrize("ramp_hz_s", [300.0, 600.0])
def test_pll_steady_state_error_under_a_doppler_ramp(ramp_hz_s):
    # A type-2 loop follows a frequency ramp R (Hz/s) with a constant phase
    # error R / wn^2 (Gardner); for the PI filter F(s) = (tau2 s + 1) /
    # (tau1 s) ahead of the NCO's integrator, wn^2 = 1 / tau1, so the error is
    # R * tau1 cycles.  The FLL adds nothing in the steady state (its input,
    # the rotation between consecutive prompts, is then zero).  The code
    # follows the carrier by aiding (same Doppler scaled by 1.023/1575.42).
    fd0 = 1000.0
    n = int(1.5 * FS)
    theta = lambda t: (IF_HZ + fd0) * t + 0.5 * ramp_hz_s * t * t                  # noqa: E731
    code = lambda t: 100.0 + CHIP_RATE * (t + (fd0 * t + 0.5 * ramp_hz_s * t * t) / F_L1)  # noqa: E731
    buf = _iq_signal(n, 7, theta, code)
    prm = oracle.LoopParams(fs=FS, if_hz=IF_HZ)
    rows, *_ = _run_loops(buf, n, prm, IF_HZ + fd0, 100.0, CHIP_RATE * (1.0 + fd0 / F_L1))
    err = np.arctan2(rows[:, 3], rows[:, 2]) / (2.0 * math.pi)
    tau1, _ = oracle.loop_coefficients(prm.pll_bw, prm.pll_zeta, prm.pll_k)
    settled = err[700:]
    assert np.mean(settled) == pytest.approx(ramp_hz_s * tau1, rel=0.02)
    assert np.std(settled) < 0.02 * ramp_hz_s * tau1


def test_pll_phase_step_response():
    # With the FLL off and gain k = 1 the PLL is the textbook type-2 loop:
    # wn^2 = 1 / tau1, 2 z wn = tau2 / tau1 (z = 0.7 here).  After a phase
    # step of 0.1 cycle its error follows the second-order closed form,
    # undershoot included, sampled at the dump midpoints.
    n = int(0.6 * FS)
    t0, step, fd = 0.2, 0.1, 800.0
    theta = lambda t: (IF_HZ + fd) * t + step * (t >= t0)                # noqa: E731
    code = lambda t: 100.0 + CHIP_RATE * (1.0 + fd / F_L1) * t           # noqa: E731
    buf = _iq_signal(n, 7, theta, code)
    prm = oracle.LoopParams(fs=FS, if_hz=IF_HZ, pll_bw=10.0, pll_zeta=0.7, pll_k=1.0,
                            fll_bw=0.0)
    rows, dn, *_ = _run_loops(buf, n, prm, IF_HZ + fd, 100.0, CHIP_RATE * (1.0 + fd / F_L1))
    err = np.arctan2(rows[:, 3], rows[:, 2]) / (2.0 * math.pi)
    tau1, tau2 = oracle.loop_coefficients(10.0, 0.7, 1.0)
    w = math.sqrt(1.0 / tau1)
    z = (tau2 / tau1) / (2.0 * w)
    starts = np.concatenate([[0], np.cumsum(dn)[:-1]])
    t = (starts + dn / 2.0) / FS - t0
    sel = (t > 5e-4) & (t < 0.35)
    pred = _second_order_error(t[sel], step, w, z)
    assert np.max(np.abs(err[sel] - pred)) < 0.06 * step
    assert np.all(np.abs(err[t < -5e-4]) < 0.005 * step)
    # the undershoot of the closed form (about -0.2 of the step at z = 0.7)
    assert np.min(err[sel]) == pytest.approx(np.min(pred), abs=0.03 * step)


def test_fll_pull_in_has_the_first_order_time_constant():
    # A first-order loop with gain K has noise bandwidth B = K / 4, so the
    # FLL of bandwidth B (frequency error measured from the rotation between
    # consecutive prompts, K = 4 B) pulls a frequency offset in as
    # exp(-4 B t).  The PLL is made negligible (0.01 Hz).
    n = int(0.15 * FS)
    fd, df0, bw = -700.0, 60.0, 10.0
    theta = lambda t: (IF_HZ + fd) * t                                   # noqa: E731
    code = lambda t: 100.0 + CHIP_RATE * (1.0 + fd / F_L1) * t           # noqa: E731
    buf = _iq_signal(n, 7, theta, code)
    prm = oracle.LoopParams(fs=FS, if_hz=IF_HZ, pll_bw=0.01, fll_bw=bw)
    rows, dn, *_ = _run_loops(buf, n, prm, IF_HZ + fd + df0, 100.0,
                              CHIP_RATE * (1.0 + fd / F_L1))
    f_used = rows[:, 6].view(np.uint32).astype(np.float64) * FS / 2.0 ** 32
    t = np.concatenate([[0], np.cumsum(dn)[:-1]]) / FS
    sel = (t > 0.005) & (t < 0.08)
    ratio = (f_used[sel] - (IF_HZ + fd)) / (df0 * np.exp(-4.0 * bw * t[sel]))
    assert np.all((ratio > 0.85) & (ratio < 1.15))


def test_dll_code_step_response():
    # The DLL's PI filter drives the code NCO (chips/s) from a discriminator
    # of gain 2 per chip (normalised early-minus-late envelope at +-1/2 chip
    # on the autocorrelation triangle), so its closed loop has wn'^2 = 2 /
    # tau1 and 2 z' wn' = 2 tau2 / tau1 (z' = 0.71 for z = 0.5, k = 1).  A
    # 0.2 chip code offset at the start decays as the second-order closed
    # form.  The carrier is known, so aiding gives the exact code Doppler.
    n = int(2.0 * FS)
    fd, d0 = 3000.0, 0.2
    rc = CHIP_RATE * (1.0 + fd / F_L1)
    theta = lambda t: (IF_HZ + fd) * t                                   # noqa: E731
    code = lambda t: 100.0 + rc * t                                      # noqa: E731
    buf = _iq_signal(n, 7, theta, code)
    prm = oracle.LoopParams(fs=FS, if_hz=IF_HZ, dll_bw=2.0, dll_zeta=0.5, dll_k=1.0)
    _, _, ends, rep, _ = _run_loops(buf, n, prm, IF_HZ + fd, 100.0 - d0, rc)
    t = ends / FS
    err = ((code(t) - rep) + 511.5) % 1023.0 - 511.5
    tau1, tau2 = oracle.loop_coefficients(2.0, 0.5, 1.0)
    w = math.sqrt(2.0 / tau1)
    z = (2.0 * tau2 / tau1) / (2.0 * w)
    pred = _second_order_error(t, d0, w, z)
    assert np.max(np.abs(err - pred)) < 0.1 * d0
    assert np.min(err) == pytest.approx(np.min(pred), abs=0.03 * d0)


def test_carrier_aiding_carries_the_code_doppler():
    # With the carrier NCO at IF + fD, aiding sets the code rate to 1.023 MHz
    # (1 + fD / 1575.42 MHz), the code Doppler of the same line-of-sight
    # motion.  Started at the nominal chip rate, the code must then stay
    # aligned with the DLL filter near zero: without aiding (or with a
    # wrong sign or scale) the DLL would have to carry the 2.6 chips/s of
    # code Doppler itself.
    n = int(2.0 * FS)
    fd = 4000.0
    rc = CHIP_RATE * (1.0 + fd / F_L1)
    theta = lambda t: (IF_HZ + fd) * t                                   # noqa: E731
    code = lambda t: 100.0 + rc * t                                      # noqa: E731
    buf = _iq_signal(n, 7, theta, code)
    prm = oracle.LoopParams(fs=FS, if_hz=IF_HZ)
    _, _, ends, rep, ls = _run_loops(buf, n, prm, IF_HZ + fd, 100.0, CHIP_RATE)
    t = ends / FS
    err = ((code(t) - rep) + 511.5) % 1023.0 - 511.5
    assert np.max(np.abs(err)) < 0.01
    assert np.max(np.abs(ls[:, 5])) < 0.1
    assert abs(ls[-1, 1] - rc) < 0.1
