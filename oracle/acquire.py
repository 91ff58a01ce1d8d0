"""Oracle of the acquisition search: parallel code-phase search (PCS) over
Doppler bins and PRNs (Sec. 3.3: the ACQ module searches a buffer of whole
code periods before tracking starts; Sec. 3.7: FFT-based search).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The search, in the steps of the classic FFT-based parallel code-phase search
(Borre et al., "A Software-Defined GPS and Galileo Receiver", 2007):

* The buffer holds Knc blocks of Mc whole code periods at R samples per chip
  (fs = R * 1.023 MHz, N = 1023 R samples per period).
* Bin d has the carrier frequency IF + f_lo + d * f_step and the 32-bit NCO
  step round_half_even(f / fs * 2^32) mod 2^32.  Its phase is 0 at the first
  sample of the buffer and runs on over every block.  The wipe-off is the
  correlator's integer one: the top 8 phase bits index the 256-entry
  amplitude-24 table, and the sample is multiplied by exp(-j theta).
* The replica at code phase tau (samples, 0 <= tau < N) gives sample n the
  chip floor((n + tau) / R) mod 1023 of the PRN's code.  So for each block
  the coherent sum Y[tau] = sum_n w[n] C[floor((n + tau) / R) mod 1023] is a
  circular cross-correlation of period N.  It is computed here with fp64
  FFTs of the block folded to one period and rounded to the nearest
  integer.  The inputs are small integers, so the rounding recovers the
  exact value; a margin check guards this.
* Power P[p, d, tau] = sum over blocks of Y_I^2 + Y_Q^2 (exact integers).
* Detection per PRN: the peak is the largest P over (d, tau).  Ties go to the
  lower bin, then the lower tau.  The chip of tau is j = floor(tau / R).  The
  second peak is the largest P in the peak's bin over the chips at least two
  chips (circularly) from the peak's chip.  The metric is peak / second, as
  doubles, and the PRN counts as acquired when the metric reaches the
  threshold.
"""
from __future__ import annotations

import numpy as np

from .oracle import I2_REAL, I8_IQ, I8_REAL, ca_code, lut, nco_words

CHIP_HZ = 1.023e6
CODE_LEN = 1023


def decode(fmt: int, buf, n: int):
    """Samples 0..n-1 of a buffer as (xI, xQ) int64 arrays (xQ = 0 for real
    formats); 2-bit codes 0..3 map to -3, -1, +1, +3, least significant pair
    first."""
    b = np.asarray(buf, dtype=np.uint8)
    if fmt == I8_REAL:
        return b[:n].view(np.int8).astype(np.int64), np.zeros(n, np.int64)
    if fmt == I8_IQ:
        v = b[:2 * n].view(np.int8).astype(np.int64)
        return v[0::2], v[1::2]
    if fmt == I2_REAL:
        codes = np.stack([(b >> (2 * j)) & 3 for j in range(4)], axis=1).reshape(-1)[:n]
        return 2 * codes.astype(np.int64) - 3, np.zeros(n, np.int64)
    raise ValueError("format")


def bin_steps(R: int, if_hz: float, f_lo: float, f_step: float, n_bins: int) -> np.ndarray:
    """The carrier NCO step of every Doppler bin (uint32)."""
    fs = float(R) * CHIP_HZ
    out = np.zeros(n_bins, np.uint64)
    for d in range(n_bins):
        f = if_hz + (f_lo + float(d) * f_step)
        out[d] = nco_words(fs, f, 0.0, CHIP_HZ, 0.0, 1)[1]
    return out


def wipe(xi, xq, step: int, n0: int, complex_in: bool):
    """Wiped-off samples (wI, wQ) of sample indices n0 .. n0 + len - 1."""
    lc, ls = lut()
    n = np.arange(n0, n0 + len(xi), dtype=np.uint64)
    ph = (n * np.uint64(step)) & np.uint64(0xFFFFFFFF)
    idx = (ph >> np.uint64(24)).astype(np.int64)
    c = lc[idx].astype(np.int64)
    s = ls[idx].astype(np.int64)
    if complex_in:
        return xi * c + xq * s, xq * c - xi * s
    return xi * c, -xi * s


def replica(prn: int, R: int) -> np.ndarray:
    """One period of the replica at tau = 0: C[floor(n / R)], n = 0 .. N-1."""
    return np.repeat(ca_code(prn).astype(np.float64), R)


def circular_xcorr(wi, wq, r):
    """Y[tau] = sum_m (wI + j wQ)[m] r[(m + tau) mod N] as exact int64 pairs."""
    x = wi.astype(np.float64) + 1j * wq.astype(np.float64)
    y = np.fft.ifft(np.fft.fft(r) * np.conj(np.fft.fft(np.conj(x))))
    yi, yq = np.rint(y.real), np.rint(y.imag)
    margin = max(float(np.max(np.abs(y.real - yi))), float(np.max(np.abs(y.imag - yq))))
    assert margin < 0.25, "FFT rounding margin lost"
    return yi.astype(np.int64), yq.astype(np.int64)


def search(fmt: int, buf, R: int, if_hz: float, f_lo: float, f_step: float, n_bins: int,
           prns, Mc: int, Knc: int) -> np.ndarray:
    """Power surface uint64 [n_prn, n_bins, N] over Knc blocks of Mc periods."""
    N = CODE_LEN * R
    L = Mc * N
    xi, xq = decode(fmt, buf, Knc * L)
    steps = bin_steps(R, if_hz, f_lo, f_step, n_bins)
    reps = [replica(p, R) for p in prns]
    P = np.zeros((len(prns), n_bins, N), np.uint64)
    for b in range(Knc):
        for d in range(n_bins):
            wi, wq = wipe(xi[b * L:(b + 1) * L], xq[b * L:(b + 1) * L], int(steps[d]), b * L,
                          fmt == I8_IQ)
            # the replica has period N: fold the block onto one period
            fi = wi.reshape(Mc, N).sum(axis=0)
            fq = wq.reshape(Mc, N).sum(axis=0)
            for k, r in enumerate(reps):
                yi, yq = circular_xcorr(fi, fq, r)
                P[k, d] += (yi * yi + yq * yq).astype(np.uint64)
    return P


def detect(P: np.ndarray, R: int, f_lo: float, f_step: float, threshold: float):
    """Per PRN: dict(peak, second, bin, tau, doppler_hz, code_phase_chips,
    metric, acquired) from a power surface [n_prn, n_bins, N]."""
    out = []
    N = P.shape[2]
    n_chips = N // R
    for k in range(P.shape[0]):
        flat = int(np.argmax(P[k].reshape(-1)))        # first maximum: lowest bin, then tau
        d, tau = divmod(flat, N)
        peak = int(P[k, d, tau])
        j = tau // R
        chips = np.arange(N) // R
        dist = np.minimum((chips - j) % n_chips, (j - chips) % n_chips)
        far = P[k, d][dist >= 2]
        second = int(far.max()) if len(far) else 0
        metric = float(peak) / float(second) if second > 0 else float("inf")
        out.append({"peak": peak, "second": second, "bin": d, "tau": tau,
                    "doppler_hz": f_lo + float(d) * f_step, "code_phase_chips": tau / R,
                    "metric": metric, "acquired": bool(metric >= threshold)})
    return out
