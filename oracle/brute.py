"""Matrix-form brute force of the integer correlator, for tiny inputs.

TEST INFRASTRUCTURE ONLY.  It restates the correlator in a different shape
from the C oracle so that the two can pin each other on tiny inputs:

  * wipe-off as one complex multiplication x * conj(c + j s) instead of the
    written-out real formulas (a wrong sign in either form shows up);
  * the replica as an explicit [samples x taps] sign matrix built with numpy
    floor division over Python integers;
  * dumps as a [windows x samples] membership matrix times that product.

The carrier table and the code are inputs (pinned on their own).
"""
from __future__ import annotations

import numpy as np

TWO32 = 1 << 32


def unpack(fmt: int, buf: np.ndarray, n: int) -> np.ndarray:
    """Complex sample values (imaginary part 0 for real formats)."""
    buf = np.asarray(buf, dtype=np.uint8)
    if fmt == 0:
        return buf[:n].view(np.int8).astype(np.int64) + 0j
    if fmt == 1:
        v = buf[: 2 * n].view(np.int8).astype(np.int64)
        return v[0::2] + 1j * v[1::2]
    if fmt == 2:
        idx = np.arange(n)
        codes = (buf[idx // 4] >> (2 * (idx % 4))) & 3
        return (2 * codes.astype(np.int64) - 3) + 0j
    # 2-bit complex: the 2-bit real packing of the interleaved stream I0 Q0 I1 Q1 ...
    bits = np.unpackbits(buf[: (n + 1) // 2], bitorder="little").reshape(-1, 2)
    codes = bits[:, 0].astype(np.int64) + 2 * bits[:, 1]           # value codes, stream order
    vals = (2 * codes - 3)[: 2 * n]
    return vals[0::2] + 1j * vals[1::2]


def correlate(fmt, buf, n, code_pm1, taps_q32, T, carr_phase, carr_step, code_phase, code_step,
              lut_cos, lut_sin):
    """Fresh channel (empty open dump) over one block.

    Returns (dumps int64 [D,K,2], dump_n, open int64 [K,2], open_n, carr_phase', code_phase')."""
    W = T * 1023 * TWO32
    x = unpack(fmt, buf, n)
    ns = [int(i) for i in range(n)]
    phi = np.array([(carr_phase + i * carr_step) % TWO32 for i in ns], dtype=np.int64)
    l = phi >> 24
    carrier = lut_cos[l].astype(np.int64) + 1j * lut_sin[l].astype(np.int64)
    w = x * np.conj(carrier)  # small integers: exact in float64
    wi = np.rint(w.real).astype(np.int64)
    wq = np.rint(w.imag).astype(np.int64)
    u = [code_phase + i * code_step for i in ns]
    m = [ui // W for ui in u]
    p = [ui - mi * W for ui, mi in zip(u, m)]
    K = len(taps_q32)
    R = np.zeros((n, K), dtype=np.int64)
    for i in range(n):
        for k in range(K):
            R[i, k] = code_pm1[((p[i] + int(taps_q32[k])) // TWO32) % 1023]
    m_end = (code_phase + n * code_step) // W
    n_win = m_end + 1
    M = np.zeros((n_win, n), dtype=np.int64)
    for i in range(n):
        M[m[i], i] = 1
    I = M @ (wi[:, None] * R)
    Q = M @ (wq[:, None] * R)
    out = np.stack([I, Q], axis=-1)
    counts = M.sum(axis=1)
    return (out[:m_end], counts[:m_end].astype(np.uint32), out[m_end], int(counts[m_end]),
            (carr_phase + n * carr_step) % TWO32, (code_phase + n * code_step) - m_end * W)
