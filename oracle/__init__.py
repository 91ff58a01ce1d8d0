"""CPU oracle for the GPS L1 C/A correlator hot path.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
path (``paper_1907_00463_amd``) never imports it and shares no code with it.

``gnss_oracle.c`` holds the definition (plain C loops, int64 / fp64);
``oracle.py`` loads it with ctypes; ``brute.py`` is an independent numpy
matrix-form brute force for tiny inputs, used as one of the pins;
``acquire.py`` is the FFT-based parallel code-phase search (numpy, fp64).
"""
from .oracle import (  # noqa: F401
    I8_REAL, I8_IQ, I2_REAL, I2_IQ, EPL_TAPS_Q32, OracleState,
    build, ca_bits, ca_code, g2_bits, g2i_bits, lut, nco_words,
    correlate_lut, correlate_f64, advance_words,
    LoopParams, TrackState, track_state, cordic_table, cordic_atan2, loop_coefficients, track,
    lock_metrics,
)
from . import acquire  # noqa: F401,E402
