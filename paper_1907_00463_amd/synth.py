"""Seeded synthetic GPS L1 C/A sample streams (the transmitter side).

This module makes inputs; it holds none of the correlator's arithmetic and
is shared by the tests, the benchmark and the CPU oracle runs.  Everything is
drawn from ``numpy.random.default_rng(seed)`` (PCG64) in a fixed order.

Signal model (Eq. (1), C/A in-phase branch only; P/Y omitted), per satellite:
    x(t) = A * d(t) * C[floor(p(t)) mod 1023] * cos(2*pi*(IF + fD)*t + phi0)
with code phase p(t) = p0 + Rc*t, Rc = 1.023e6 * (1 + fD / 1575.42e6)
(carrier-aided code Doppler), 50 bps navigation bits d = +-1 that change on
code epochs every 20 periods (Sec. 3.1), plus white Gaussian noise of unit
variance.  Complex baseband uses exp(j*...) instead of cos.  Amplitude from
C/N0 (linear): real A = 2*sqrt(C/N0/fs); complex A = sqrt(C/N0/fs) with unit
total noise power.

Quantisation: int8 = clip(round(8*x/sigma_c), -127, 127) per component with
sigma_c the per-component noise std (so noise is 8 LSB); 2-bit real with
thresholds 0 and +-1 sigma to values -3,-1,+1,+3 (codes 0..3), packed four
per byte, sample j of a byte in bits [2j, 2j+1].

The C/A codes are built here from the G1/G2 registers and each satellite's
G2 delay (IS-GPS-200, Table 3-Ia), a construction of this module's own.
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import List, Optional

import numpy as np

F_L1 = 1575.42e6
CHIP_RATE = 1.023e6
I8_REAL, I8_IQ, I2_REAL, I2_IQ = 0, 1, 2, 3
FMT_NAMES = {I8_REAL: "i8_real", I8_IQ: "i8_iq", I2_REAL: "i2_real", I2_IQ: "i2_iq"}

# G2 delay in chips for PRN 1..32 (IS-GPS-200, Table 3-Ia, "G2 delay" column).
_G2_DELAY = [5, 6, 7, 8, 17, 18, 139, 140, 141, 251, 252, 254, 255, 256, 257, 258,
             469, 470, 471, 472, 473, 474, 509, 512, 513, 514, 515, 516, 859, 860, 861, 862]


def _mseq(feedback_stages):
    reg = [1] * 10  # reg[0] is stage 1
    out = np.zeros(1023, np.uint8)
    for i in range(1023):
        out[i] = reg[9]
        f = 0
        for s in feedback_stages:
            f ^= reg[s - 1]
        reg = [f] + reg[:9]
    return out


_G1 = _mseq((3, 10))
_G2 = _mseq((2, 3, 6, 8, 9, 10))


def ca_chips(prn: int) -> np.ndarray:
    """C/A chips as +-1 (logic 0 -> +1, logic 1 -> -1), int8[1023]."""
    d = _G2_DELAY[prn - 1]
    g2d = np.roll(_G2, d)  # g2d[i] = G2[(i - d) mod 1023]
    bits = _G1 ^ g2d
    return (1 - 2 * bits.astype(np.int8)).astype(np.int8)


def code_rate(doppler_hz: float) -> float:
    return CHIP_RATE * (1.0 + doppler_hz / F_L1)


@dataclasses.dataclass
class Satellite:
    prn: int
    doppler_hz: float
    code_phase0: float     # chips at t = 0
    cn0_dbhz: float
    carr_phase0: float     # cycles at t = 0
    nav_bits: np.ndarray   # +-1 per 20-period bit, index 0 starts at true code epoch 0


@dataclasses.dataclass
class Stream:
    fs: float
    if_hz: float
    fmt: int
    n: int
    sats: List[Satellite]
    seed: int


def _amplitude(cn0_dbhz: float, fs: float, complex_: bool) -> float:
    c_n0 = 10.0 ** (cn0_dbhz / 10.0)
    return math.sqrt(c_n0 / fs) if complex_ else 2.0 * math.sqrt(c_n0 / fs)


def _nav_bits(rng, n, fs, p0, rc):
    periods = int(math.ceil((p0 + rc * n / fs) / 1023.0 / 20.0)) + 2
    return rng.choice(np.array([-1, 1], np.int8), size=periods)


def _sat_contribution(s: Satellite, code: np.ndarray, c0: int, m: int, fs: float, if_hz: float,
                      complex_: bool) -> np.ndarray:
    a = _amplitude(s.cn0_dbhz, fs, complex_)
    rc = code_rate(s.doppler_hz)
    k = np.arange(m, dtype=np.float64)
    # code phase and carrier cycles at the chunk start in float64, then offsets
    p = (s.code_phase0 + rc * (c0 / fs)) + (rc / fs) * k
    pi = np.floor(p).astype(np.int64)
    amp = (a * code[pi % 1023]) * s.nav_bits[np.minimum(pi // (1023 * 20), len(s.nav_bits) - 1)]
    cyc0 = s.carr_phase0 + (if_hz + s.doppler_hz) * (c0 / fs)
    cyc = (cyc0 - math.floor(cyc0)) + ((if_hz + s.doppler_hz) / fs) * k
    ph = (2.0 * np.pi) * (cyc - np.floor(cyc))
    if complex_:
        return amp * np.exp(1j * ph)
    return amp * np.cos(ph)


def synth_samples(st: Stream, rng: np.random.Generator, chunk: int = 1 << 20,
                  threads: Optional[int] = None) -> np.ndarray:
    """Sample buffer as uint8 bytes in the stream's format.

    Noise is drawn chunk by chunk from ``rng`` in stream order; satellite
    contributions are computed in a thread pool and summed in satellite order,
    so the result does not depend on the thread count."""
    from concurrent.futures import ThreadPoolExecutor

    complex_ = st.fmt in (I8_IQ, I2_IQ)
    codes = {s.prn: ca_chips(s.prn).astype(np.float64) for s in st.sats}
    if st.fmt == I2_REAL:
        assert st.n % 4 == 0
        out = np.empty(st.n // 4, np.uint8)
    elif st.fmt == I2_IQ:
        assert st.n % 2 == 0
        out = np.empty(st.n // 2, np.uint8)
    elif complex_:
        out = np.empty(2 * st.n, np.uint8)
    else:
        out = np.empty(st.n, np.uint8)
    nthr = threads or min(16, max(1, len(st.sats)), (os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=nthr) as pool:
        for c0 in range(0, st.n, chunk):
            m = min(chunk, st.n - c0)
            if complex_:
                x = (rng.standard_normal(m) + 1j * rng.standard_normal(m)) * math.sqrt(0.5)
            else:
                x = rng.standard_normal(m)
            futs = [pool.submit(_sat_contribution, s, codes[s.prn], c0, m, st.fs, st.if_hz,
                                complex_) for s in st.sats]
            for f in futs:
                x += f.result()
            if st.fmt == I2_REAL:
                q = ((x >= -1.0).astype(np.uint8) + (x >= 0.0) + (x >= 1.0)).reshape(-1, 4)
                out[c0 // 4: (c0 + m) // 4] = q[:, 0] | (q[:, 1] << 2) | (q[:, 2] << 4) | (q[:, 3] << 6)
            elif st.fmt == I2_IQ:
                # each component against 0 and +-1 sigma (sigma = sqrt(1/2)),
                # packed as the interleaved stream I0 Q0 I1 Q1 of value codes
                t = math.sqrt(0.5)
                comp = np.empty(2 * m)
                comp[0::2] = x.real
                comp[1::2] = x.imag
                q = ((comp >= -t).astype(np.uint8) + (comp >= 0.0) + (comp >= t)).reshape(-1, 4)
                out[c0 // 2: (c0 + m) // 2] = q[:, 0] | (q[:, 1] << 2) | (q[:, 2] << 4) | (q[:, 3] << 6)
            elif complex_:
                sc = 8.0 / math.sqrt(0.5)
                inter = np.empty(2 * m, np.int8)
                inter[0::2] = np.clip(np.rint(x.real * sc), -127, 127)
                inter[1::2] = np.clip(np.rint(x.imag * sc), -127, 127)
                out[2 * c0: 2 * (c0 + m)] = inter.view(np.uint8)
            else:
                out[c0: c0 + m] = np.clip(np.rint(x * 8.0), -127, 127).astype(np.int8).view(np.uint8)
    return out


def make_sat(rng, fs, n, prn, doppler_hz, code_phase0, cn0_dbhz, carr_phase0=None) -> Satellite:
    if carr_phase0 is None:
        carr_phase0 = float(rng.random())
    bits = _nav_bits(rng, n, fs, code_phase0, code_rate(doppler_hz))
    return Satellite(prn, doppler_hz, code_phase0, cn0_dbhz, carr_phase0, bits)


# --------------------------------------------------------------------------
# Channel descriptions for the correlator (physical parameters only; the NCO
# word conversion belongs to the correlator library and to the oracle).
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Channel:
    prn: int
    carr_hz: float          # IF + Doppler
    carr_phase0: float      # cycles at sample 0
    code_rate: float        # chips/s
    code_phase0: float      # chips at sample 0
    int_periods: int = 1
    taps_chips: tuple = (0.5, 0.0, -0.5)


def epl_taps_q32(spacing_chips: float = 0.5) -> np.ndarray:
    h = int(round(spacing_chips * (1 << 32)))
    return np.array([h, 0, -h], dtype=np.int64)


def taps_to_q32(taps_chips) -> np.ndarray:
    return np.array([int(round(t * (1 << 32))) for t in taps_chips], dtype=np.int64)


def channel_for(sat: Satellite, if_hz: float, int_periods: int = 1, taps=(0.5, 0.0, -0.5),
                code_offset_chips: float = 0.0, doppler_offset_hz: float = 0.0) -> Channel:
    """Open-loop channel at the satellite's true parameters (plus optional offsets)."""
    fd = sat.doppler_hz + doppler_offset_hz
    return Channel(prn=sat.prn, carr_hz=if_hz + fd, carr_phase0=sat.carr_phase0,
                   code_rate=code_rate(fd), code_phase0=sat.code_phase0 + code_offset_chips,
                   int_periods=int_periods, taps_chips=tuple(taps))


# --------------------------------------------------------------------------
# The five workloads (seed 1000 + workload number).
# --------------------------------------------------------------------------
def workload_single_channel(seconds: float = 1.0, seed: int = 1001):
    """PRN 7, fs 4.092 MHz, IF 1.023 MHz, int8 real, +1.5 kHz, 300.25 chips, 45 dB-Hz."""
    rng = np.random.default_rng(seed)
    fs, if_hz = 4.092e6, 1.023e6
    n = int(round(seconds * fs))
    sat = make_sat(rng, fs, n, 7, 1500.0, 300.25, 45.0)
    st = Stream(fs, if_hz, I8_REAL, n, [sat], seed)
    return st, [channel_for(sat, if_hz)], rng


def workload_twelve_channels(seconds: float = 10.0, seed: int = 1002):
    """12 PRNs, fs 16.368 MHz, IF 4.092 MHz, 2-bit real, fD ~ U(-5,5) kHz, C/N0 ~ U(35,50)."""
    rng = np.random.default_rng(seed)
    fs, if_hz = 16.368e6, 4.092e6
    n = int(round(seconds * fs))
    n -= n % 4
    prns = rng.choice(np.arange(1, 33), size=12, replace=False)
    dop = rng.uniform(-5000.0, 5000.0, size=12)
    p0 = rng.uniform(0.0, 1023.0, size=12)
    cn0 = rng.uniform(35.0, 50.0, size=12)
    sats = [make_sat(rng, fs, n, int(prns[i]), float(dop[i]), float(p0[i]), float(cn0[i]))
            for i in range(12)]
    st = Stream(fs, if_hz, I2_REAL, n, sats, seed)
    return st, [channel_for(s, if_hz) for s in sats], rng


def workload_paper(seconds: float = 10.0, seed: int = 1010):
    """The paper's offline configuration (Sec. 4): complex int8, I then Q, at
    fs 5 MHz from a direct-conversion front end (IF 0, Sec. 2.2), 12 satellites
    in view, 1 ms integrations.  PRNs, Dopplers ~ U(-5, 5) kHz, code phases
    and C/N0 ~ U(35, 50) dB-Hz are drawn as for the 12-channel workload."""
    rng = np.random.default_rng(seed)
    fs, if_hz = 5.0e6, 0.0
    n = int(round(seconds * fs))
    n -= n % 4
    prns = rng.choice(np.arange(1, 33), size=12, replace=False)
    dop = rng.uniform(-5000.0, 5000.0, size=12)
    p0 = rng.uniform(0.0, 1023.0, size=12)
    cn0 = rng.uniform(35.0, 50.0, size=12)
    sats = [make_sat(rng, fs, n, int(prns[i]), float(dop[i]), float(p0[i]), float(cn0[i]))
            for i in range(12)]
    st = Stream(fs, if_hz, I8_IQ, n, sats, seed)
    return st, [channel_for(s, if_hz) for s in sats], rng


def workload_iq2(seconds: float = 10.0, seed: int = 1011):
    """2-bit complex baseband (I then Q codes interleaved, two samples per
    byte) at fs 8.184 MHz from a zero-IF front end, 12 satellites, 1 ms
    integrations; PRNs, Dopplers ~ U(-5, 5) kHz, code phases and C/N0 ~
    U(35, 50) dB-Hz drawn as for the 12-channel workload."""
    rng = np.random.default_rng(seed)
    fs, if_hz = 8.184e6, 0.0
    n = int(round(seconds * fs))
    n -= n % 4
    prns = rng.choice(np.arange(1, 33), size=12, replace=False)
    dop = rng.uniform(-5000.0, 5000.0, size=12)
    p0 = rng.uniform(0.0, 1023.0, size=12)
    cn0 = rng.uniform(35.0, 50.0, size=12)
    sats = [make_sat(rng, fs, n, int(prns[i]), float(dop[i]), float(p0[i]), float(cn0[i]))
            for i in range(12)]
    st = Stream(fs, if_hz, I2_IQ, n, sats, seed)
    return st, [channel_for(s, if_hz) for s in sats], rng


def workload_if_recording(seconds: float = 10.0, seed: int = 1012):
    """A recording of the GN3S kind (offline mode's IF files): real samples
    at fs 16.3676 MHz with IF 4.1304 MHz, stored one int8 per sample, 12
    satellites, 1 ms integrations.  At 16.0 samples per chip less a little,
    the half chips are not a whole number of samples long."""
    rng = np.random.default_rng(seed)
    fs, if_hz = 16.3676e6, 4.1304e6
    n = int(round(seconds * fs))
    n -= n % 4
    prns = rng.choice(np.arange(1, 33), size=12, replace=False)
    dop = rng.uniform(-5000.0, 5000.0, size=12)
    p0 = rng.uniform(0.0, 1023.0, size=12)
    cn0 = rng.uniform(35.0, 50.0, size=12)
    sats = [make_sat(rng, fs, n, int(prns[i]), float(dop[i]), float(p0[i]), float(cn0[i]))
            for i in range(12)]
    st = Stream(fs, if_hz, I8_REAL, n, sats, seed)
    return st, [channel_for(s, if_hz) for s in sats], rng


def workload_multicorrelator(seconds: float = 2.0, seed: int = 1004, n_chan: int = 256):
    """Complex int8 at 20.46 MHz, IF 0; 12 satellites in the stream; 256 channels =
    32 PRNs x 8 (Doppler, code) hypotheses; 128 taps at -2 + k/32 chips."""
    rng = np.random.default_rng(seed)
    fs, if_hz = 20.46e6, 0.0
    n = int(round(seconds * fs))
    prns = rng.choice(np.arange(1, 33), size=12, replace=False)
    dop = rng.uniform(-5000.0, 5000.0, size=12)
    p0 = rng.uniform(0.0, 1023.0, size=12)
    cn0 = rng.uniform(35.0, 50.0, size=12)
    sats = [make_sat(rng, fs, n, int(prns[i]), float(dop[i]), float(p0[i]), float(cn0[i]))
            for i in range(12)]
    st = Stream(fs, if_hz, I8_IQ, n, sats, seed)
    taps = tuple(-2.0 + k / 32.0 for k in range(128))
    by_prn = {s.prn: s for s in sats}
    chans = []
    for c in range(n_chan):
        prn = c % 32 + 1
        hyp = c // 32
        if prn in by_prn:
            s = by_prn[prn]
            ch = channel_for(s, if_hz, taps=taps, code_offset_chips=0.25 * hyp,
                             doppler_offset_hz=25.0 * hyp)
        else:
            fd = float(rng.uniform(-5000.0, 5000.0))
            ch = Channel(prn=prn, carr_hz=if_hz + fd, carr_phase0=0.0, code_rate=code_rate(fd),
                         code_phase0=float(rng.uniform(0.0, 1023.0)), taps_chips=taps)
        chans.append(ch)
    return st, chans, rng


def workload_batched(seconds: float = 1.0, seed: int = 1003, n_rx: int = 64):
    """64 receivers x U{8..14} channels, one satellite per channel; fs uniform
    over {4.092, 8.184, 16.368} MHz with IF = fs/4; int8 or 2-bit real; the
    integration of each channel uniform over {1, 4, 20} periods; 1 s each.
    Receiver r draws from its own generator default_rng([seed, r]): rate,
    format, channel count, PRNs, Dopplers, code phases, C/N0, periods, then
    the satellites' carrier phases and navigation bits, then (in
    synth_batched) its samples.  Returns [(Stream, [Channel], rng_r)]."""
    rates = np.array([4.092e6, 8.184e6, 16.368e6])
    out = []
    for r in range(n_rx):
        rng = np.random.default_rng([seed, r])
        fs = float(rng.choice(rates))
        fmt = int(rng.choice([I8_REAL, I2_REAL]))
        n = int(round(seconds * fs))
        n -= n % 4
        k = int(rng.integers(8, 15))
        prns = rng.choice(np.arange(1, 33), size=k, replace=False)
        dop = rng.uniform(-5000.0, 5000.0, size=k)
        p0 = rng.uniform(0.0, 1023.0, size=k)
        cn0 = rng.uniform(35.0, 50.0, size=k)
        periods = rng.choice(np.array([1, 4, 20]), size=k)
        sats = [make_sat(rng, fs, n, int(prns[i]), float(dop[i]), float(p0[i]), float(cn0[i]))
                for i in range(k)]
        st = Stream(fs, fs / 4, fmt, n, sats, seed)
        out.append((st, [channel_for(sats[i], fs / 4, int_periods=int(periods[i]))
                         for i in range(k)], rng))
    return out


def synth_batched(workload, threads: Optional[int] = None):
    """Sample buffers of every receiver of workload_batched, receivers in
    parallel (each from its own generator, so the result does not depend on
    the thread count)."""
    from concurrent.futures import ThreadPoolExecutor

    nthr = threads or min(16, (os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=nthr) as pool:
        return list(pool.map(lambda w: synth_samples(w[0], w[2], threads=1), workload))


def workload_serving(seed: int = 1005, n_rx: int = 500, stream_ms: float = 24.0):
    """500 receivers x U{4..14} channels, drawn as in workload_batched (rate
    over {4.092, 8.184, 16.368} MHz with IF = fs/4, int8 or 2-bit real,
    integrations over {1, 4, 20} periods) from default_rng([seed, r]); each
    receiver has stream_ms of samples that its requests slice (see
    serving_schedule).  Returns [(Stream, [Channel], rng_r)]."""
    rates = np.array([4.092e6, 8.184e6, 16.368e6])
    out = []
    for r in range(n_rx):
        rng = np.random.default_rng([seed, r])
        fs = float(rng.choice(rates))
        fmt = int(rng.choice([I8_REAL, I2_REAL]))
        n = int(round(stream_ms * 1e-3 * fs))
        n -= n % 4
        k = int(rng.integers(4, 15))
        prns = rng.choice(np.arange(1, 33), size=k, replace=False)
        dop = rng.uniform(-5000.0, 5000.0, size=k)
        p0 = rng.uniform(0.0, 1023.0, size=k)
        cn0 = rng.uniform(35.0, 50.0, size=k)
        periods = rng.choice(np.array([1, 4, 20]), size=k)
        sats = [make_sat(rng, fs, n, int(prns[i]), float(dop[i]), float(p0[i]), float(cn0[i]))
                for i in range(k)]
        st = Stream(fs, fs / 4, fmt, n, sats, seed)
        out.append((st, [channel_for(sats[i], fs / 4, int_periods=int(periods[i]))
                         for i in range(k)], rng))
    return out


def serving_schedule(workload, rate_hz: float = 2000.0, seconds: float = 10.0,
                     seed: int = 1006):
    """Poisson arrivals at rate_hz over `seconds`: exponential gaps, each
    request for a receiver drawn uniformly, lasting U{1..20} ms of its
    samples.  A receiver's requests take consecutive slices of its stream
    (offsets are multiples of 4 samples, wrapping to the start when the next
    slice would not fit), so its channels see a continuing signal up to the
    wrap.  Returns arrays (t_arrival s, receiver, offset, n_samples)."""
    rng = np.random.default_rng(seed)
    n_req = int(rng.poisson(rate_hz * seconds))
    t = np.sort(rng.uniform(0.0, seconds, size=n_req))
    rx = rng.integers(0, len(workload), size=n_req)
    dur = rng.integers(1, 21, size=n_req)
    off = np.zeros(n_req, np.int64)
    ns = np.zeros(n_req, np.int64)
    cur = np.zeros(len(workload), np.int64)
    for i in range(n_req):
        st = workload[int(rx[i])][0]
        n = int(round(int(dur[i]) * 1e-3 * st.fs))
        n -= n % 4
        if cur[rx[i]] + n > st.n:
            cur[rx[i]] = 0
        off[i], ns[i] = cur[rx[i]], n
        cur[rx[i]] += n
    return t, rx, off, ns
