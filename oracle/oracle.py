"""ctypes front end of the C oracle (``gnss_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).  The wrappers only
marshal numpy arrays; every number is computed by the C code.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

I8_REAL, I8_IQ, I2_REAL, I2_IQ = 0, 1, 2, 3
ERANGE, ENOSPC = -4, -7
TWO32 = 1 << 32

# Early / prompt / late at +1/2, 0, -1/2 chip from prompt (Table 3: 1/2-chip
# early-late spacing, read as the offset of each of E and L from P).
EPL_TAPS_Q32 = np.array([1 << 31, 0, -(1 << 31)], dtype=np.int64)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gnss_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-Wall", "-ffp-contract=off",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        lib.orc_ca_bits.argtypes = [C.c_int, P]
        lib.orc_g2_bits.argtypes = [P]
        lib.orc_g2i_bits.argtypes = [C.c_int, P]
        lib.orc_ca_code.argtypes = [C.c_int, P]
        lib.orc_lut.argtypes = [P, P]
        lib.orc_nco_words.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double,
                                      C.c_double, C.c_int, P, P, P, P]
        lib.orc_correlate_lut.argtypes = [C.c_int, P, C.c_uint64, C.c_int, C.c_int, P, C.c_int,
                                          P, C.c_uint32, P, C.c_uint64, P, P, P, P,
                                          C.c_uint32, P]
        lib.orc_correlate_f64.argtypes = [C.c_int, P, C.c_uint64, C.c_int, C.c_int, P, C.c_int,
                                          P, C.c_double, P, C.c_uint64, P, P, P, P,
                                          C.c_uint32, P]
        lib.orc_cordic_table.argtypes = [P]
        lib.orc_cordic_atan2.argtypes = [C.c_int64, C.c_int64, P]
        lib.orc_loop_coefficients.argtypes = [C.c_double, C.c_double, C.c_double, P]
        lib.orc_track.argtypes = [C.c_int, P, C.c_uint64, C.c_int, C.c_int, P, P, P, P, P, P, P,
                                  P, P, P, P, C.c_uint32, P]
        lib.orc_lock_metrics.argtypes = [P, C.c_uint32, C.c_uint32, C.c_double, C.c_double,
                                         C.c_uint32, P, P, P, P, P, P, P, C.c_uint32, P]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def ca_bits(prn: int) -> np.ndarray:
    out = np.zeros(1023, np.uint8)
    if _load().orc_ca_bits(prn, _p(out)):
        raise ValueError("prn out of range")
    return out


def g2_bits() -> np.ndarray:
    out = np.zeros(1023, np.uint8)
    _load().orc_g2_bits(_p(out))
    return out


def g2i_bits(prn: int) -> np.ndarray:
    out = np.zeros(1023, np.uint8)
    if _load().orc_g2i_bits(prn, _p(out)):
        raise ValueError("prn out of range")
    return out


def ca_code(prn: int) -> np.ndarray:
    out = np.zeros(1023, np.int8)
    if _load().orc_ca_code(prn, _p(out)):
        raise ValueError("prn out of range")
    return out


def lut():
    c = np.zeros(256, np.int8)
    s = np.zeros(256, np.int8)
    _load().orc_lut(_p(c), _p(s))
    return c, s


def nco_words(fs_hz, carr_hz, carr_phase_cyc, code_rate_cps, code_phase_chips, int_periods):
    """(carr_phase, carr_step, code_phase, code_step) words."""
    cp = np.zeros(1, np.uint32)
    cs = np.zeros(1, np.uint32)
    kp = np.zeros(1, np.uint64)
    ks = np.zeros(1, np.uint64)
    rc = _load().orc_nco_words(fs_hz, carr_hz, carr_phase_cyc, code_rate_cps, code_phase_chips,
                               int_periods, _p(cp), _p(cs), _p(kp), _p(ks))
    if rc:
        raise ValueError("bad NCO parameters")
    return int(cp[0]), int(cs[0]), int(kp[0]), int(ks[0])


def advance_words(carr_phase, carr_step, code_phase, code_step, int_periods, n):
    """Closed-form NCO words after n samples (carrier mod 2^32, code mod W)."""
    W = int_periods * 1023 * TWO32
    return (carr_phase + n * carr_step) % TWO32, (code_phase + n * code_step) % W


@dataclasses.dataclass
class OracleState:
    """One channel's open state: NCO words plus the open dump."""
    carr_phase: int
    carr_step: int
    code_phase: int
    code_step: int
    n_taps: int
    acc: np.ndarray = None      # int64 [n_taps*2] (LUT) or float64 (f64 form)
    acc_n: int = 0
    carr_phase_f: float = 0.0   # cycles, FP64 form
    carr_freq_f: float = 0.0    # cycles per sample, FP64 form

    def copy(self):
        return dataclasses.replace(self, acc=None if self.acc is None else self.acc.copy())


def _max_dumps(n, st, T):
    W = T * 1023 * TWO32
    return (st.code_phase + n * st.code_step) // W + 1


def correlate_lut(fmt, buf, n, prn, taps_q32, T, st: OracleState, check_range=True):
    """Integer correlator for one channel; returns (dumps int64 [D,K,2], dump_n [D]).

    ``st`` is updated in place (carrier/code phase words, open dump)."""
    lib = _load()
    taps = np.ascontiguousarray(taps_q32, dtype=np.int64)
    K = len(taps)
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    if st.acc is None:
        st.acc = np.zeros(2 * K, np.int64)
    md = _max_dumps(n, st, T)
    dumps = np.zeros((md, K, 2), np.int64)
    dump_n = np.zeros(md, np.uint32)
    cp = np.array([st.carr_phase], np.uint32)
    kp = np.array([st.code_phase], np.uint64)
    an = np.array([st.acc_n], np.uint32)
    nd = np.zeros(1, np.uint32)
    acc = np.ascontiguousarray(st.acc, dtype=np.int64)
    rc = lib.orc_correlate_lut(fmt, _p(buf), n, prn, K, _p(taps), T, _p(cp), st.carr_step,
                               _p(kp), st.code_step, _p(acc), _p(an), _p(dumps), _p(dump_n),
                               md, _p(nd))
    if rc == ERANGE and check_range:
        raise OverflowError("accumulation leaves int32")
    if rc and rc != ERANGE:
        raise RuntimeError("oracle error %d" % rc)
    st.carr_phase, st.code_phase, st.acc, st.acc_n = int(cp[0]), int(kp[0]), acc, int(an[0])
    d = int(nd[0])
    return dumps[:d], dump_n[:d]


def correlate_f64(fmt, buf, n, prn, taps_q32, T, st: OracleState):
    """FP64-carrier correlator for one channel; returns (dumps f64 [D,K,2], dump_n [D])."""
    lib = _load()
    taps = np.ascontiguousarray(taps_q32, dtype=np.int64)
    K = len(taps)
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    if st.acc is None:
        st.acc = np.zeros(2 * K, np.float64)
    md = _max_dumps(n, st, T)
    dumps = np.zeros((md, K, 2), np.float64)
    dump_n = np.zeros(md, np.uint32)
    cp = np.array([st.carr_phase_f], np.float64)
    kp = np.array([st.code_phase], np.uint64)
    an = np.array([st.acc_n], np.uint32)
    nd = np.zeros(1, np.uint32)
    acc = np.ascontiguousarray(st.acc, dtype=np.float64)
    rc = lib.orc_correlate_f64(fmt, _p(buf), n, prn, K, _p(taps), T, _p(cp), st.carr_freq_f,
                               _p(kp), st.code_step, _p(acc), _p(an), _p(dumps), _p(dump_n),
                               md, _p(nd))
    if rc:
        raise RuntimeError("oracle error %d" % rc)
    st.carr_phase_f, st.code_phase, st.acc, st.acc_n = float(cp[0]), int(kp[0]), acc, int(an[0])
    d = int(nd[0])
    return dumps[:d], dump_n[:d]


# ---------------------------------------------------------------- closed loops
@dataclasses.dataclass
class LoopParams:
    """Tracking-loop parameters (Table 3 names the loop types; the bandwidths,
    damping ratios and gains are this library's defaults, those of softGNSS
    for the DLL and PLL)."""
    fs: float
    if_hz: float
    dll_bw: float = 2.0
    dll_zeta: float = 0.7
    dll_k: float = 1.0
    pll_bw: float = 25.0
    pll_zeta: float = 0.7
    pll_k: float = 0.25
    fll_bw: float = 10.0

    def array(self) -> np.ndarray:
        return np.array([self.fs, self.if_hz, self.dll_bw, self.dll_zeta, self.dll_k,
                         self.pll_bw, self.pll_zeta, self.pll_k, self.fll_bw], np.float64)


@dataclasses.dataclass
class TrackState:
    """A tracked channel: NCO words and open dump (``words``, 3 taps), loop
    state ``ls`` = (carrier Hz, code chips/s, FLL basis Hz, PLL nco Hz, PLL
    error cycles, DLL nco chips/s, DLL error) and ``is_`` = (previous prompt
    I, Q, set)."""
    words: OracleState
    ls: np.ndarray
    is_: np.ndarray

    def copy(self):
        return TrackState(self.words.copy(), self.ls.copy(), self.is_.copy())


def track_state(words: OracleState, carr_hz: float, code_rate: float) -> TrackState:
    ls = np.array([carr_hz, code_rate, carr_hz, 0.0, 0.0, 0.0, 0.0], np.float64)
    return TrackState(words, ls, np.zeros(3, np.int32))


def cordic_table() -> np.ndarray:
    out = np.zeros(31, np.int64)
    _load().orc_cordic_table(_p(out))
    return out


def cordic_atan2(y: int, x: int) -> int:
    """atan2(y, x), x >= 0, in units of 2^-30 rad."""
    out = np.zeros(1, np.int64)
    if _load().orc_cordic_atan2(int(y), int(x), _p(out)):
        raise ValueError("x must be >= 0")
    return int(out[0])


def loop_coefficients(bw, zeta, k):
    out = np.zeros(2, np.float64)
    if _load().orc_loop_coefficients(bw, zeta, k, _p(out)):
        raise ValueError("bad loop parameters")
    return float(out[0]), float(out[1])


def track(fmt, buf, n, prn, T, params: LoopParams, st: TrackState):
    """Closed-loop E/P/L tracking of one channel over one block; returns
    (rows int32 [D, 8]: E I, E Q, P I, P Q, L I, L Q, carrier step, code step
    used; dump_n [D]).  ``st`` is updated in place."""
    lib = _load()
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    w = st.words
    if w.acc is None:
        w.acc = np.zeros(6, np.int64)
    md = n // (T * 2046) + 2              # code steps stay below 2^31
    rows = np.zeros((md, 8), np.int32)
    dump_n = np.zeros(md, np.uint32)
    cp = np.array([w.carr_phase], np.uint32)
    cs = np.array([w.carr_step], np.uint32)
    kp = np.array([w.code_phase], np.uint64)
    ks = np.array([w.code_step], np.uint64)
    an = np.array([w.acc_n], np.uint32)
    nd = np.zeros(1, np.uint32)
    acc = np.ascontiguousarray(w.acc, dtype=np.int64)
    ls = np.ascontiguousarray(st.ls, dtype=np.float64)
    is_ = np.ascontiguousarray(st.is_, dtype=np.int32)
    prm = params.array()
    rc = lib.orc_track(fmt, _p(buf), n, prn, T, _p(prm), _p(cp), _p(cs), _p(kp), _p(ks),
                       _p(acc), _p(an), _p(ls), _p(is_), _p(rows), _p(dump_n), md, _p(nd))
    if rc == ERANGE:
        raise OverflowError("accumulation leaves int32 or a code step leaves [1, 2^31)")
    if rc:
        raise RuntimeError("oracle error %d" % rc)
    w.carr_phase, w.carr_step = int(cp[0]), int(cs[0])
    w.code_phase, w.code_step = int(kp[0]), int(ks[0])
    w.acc, w.acc_n = acc, int(an[0])
    st.ls, st.is_ = ls, is_
    d = int(nd[0])
    return rows[:d], dump_n[:d]


def lock_metrics(prompt, K=20, T=1e-3, lock_min=0.5, phase=0):
    """C/N0 (dB-Hz) and lock ratio per window of K dumps, lock failures, the
    20-position bit-transition histogram, the bit edge and the navigation
    bits, from prompts int32 [n, 2] (I, Q) of consecutive dumps; ``phase``
    is the position of dump 0 in the 20-dump cycle."""
    lib = _load()
    prompt = np.ascontiguousarray(prompt, dtype=np.int32).reshape(-1, 2)
    n = len(prompt)
    nw_max = max(1, n // K)
    cn0 = np.zeros(nw_max, np.float64)
    lock = np.zeros(nw_max, np.float64)
    nw = np.zeros(1, np.uint32)
    fails = np.zeros(1, np.uint32)
    hist = np.zeros(20, np.uint32)
    edge = np.zeros(1, np.uint32)
    max_bits = n // 20 + 1
    bits = np.zeros(max_bits, np.uint8)
    nb = np.zeros(1, np.uint32)
    rc = lib.orc_lock_metrics(_p(prompt), n, K, T, lock_min, phase, _p(cn0), _p(lock), _p(nw),
                              _p(fails), _p(hist), _p(edge), _p(bits), max_bits, _p(nb))
    if rc:
        raise ValueError("bad lock-metric arguments")
    w = int(nw[0])
    return {"cn0": cn0[:w], "lock": lock[:w], "lock_fails": int(fails[0]), "hist": hist,
            "edge": int(edge[0]), "bits": bits[:int(nb[0])]}
