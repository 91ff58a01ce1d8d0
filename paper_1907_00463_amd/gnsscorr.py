"""Python binding of libgnsscorr (ctypes; argument marshalling only).

Every function named ``gc_*`` calls the C entry point of the same name in
``libgnsscorr.so``; every step of the correlator runs in the library's HIP
kernels.  torch is used for device memory and streams only.  There is no
fallback: if the built library is missing, importing the binding raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgnsscorr.so")

GC_OK, GC_EINVAL, GC_ENOMEM, GC_EDEVICE, GC_ERANGE, GC_EBUSY, GC_EAGAIN, GC_ENOSPC = (
    0, -1, -2, -3, -4, -5, -6, -7)
GC_I8_REAL, GC_I8_IQ, GC_I2_REAL, GC_I2_IQ = 0, 1, 2, 3
GC_CARRIER_LUT, GC_CARRIER_F32 = 0, 1
GC_KERNEL_PERIODIC, GC_KERNEL_BINNED, GC_KERNEL_MTAP = 1, 2, 4
GC_SERVER_PLAIN = 1
GC_MAX_TAPS = 128
GC_NOALLOC_MAX_CHANNELS = 1024
GC_LUT_AMP = 24
TWO32 = 1 << 32

# ABI structs (layouts fixed by include/gnsscorr.h)
CHAN_CFG = np.dtype([("prn", "<i4"), ("n_taps", "<i4"), ("int_periods", "<i4"),
                     ("reserved", "<i4"), ("tap_q32", "<i8", (GC_MAX_TAPS,))])
CHAN_STATE = np.dtype([("code_phase", "<u8"), ("code_step", "<u8"), ("carr_phase", "<u4"),
                       ("carr_step", "<u4"), ("acc_n", "<u4"), ("flags", "<u4"),
                       ("carr_phase_f", "<f8"), ("carr_freq_f", "<f8"),
                       ("acc", "<i4", (GC_MAX_TAPS, 2)), ("acc_f", "<f4", (GC_MAX_TAPS, 2))])
RX_DESC = np.dtype([("samples", "<u8"), ("n_samples", "<u8"), ("fmt", "<i4"),
                    ("reserved", "<i4")])
SERVER_TIMING = np.dtype([("launches", "<u8"), ("launched_requests", "<u8"),
                          ("enqueue_mean_ms", "<f8"), ("enqueue_max_ms", "<f8"),
                          ("device_mean_ms", "<f8"), ("device_max_ms", "<f8"),
                          ("submit_max_ms", "<f8")])
assert CHAN_CFG.itemsize == 1040 and CHAN_STATE.itemsize == 2096 and RX_DESC.itemsize == 24
assert SERVER_TIMING.itemsize == 56
LOOP_PARAMS = np.dtype([("fs_hz", "<f8"), ("if_hz", "<f8"), ("dll_bw_hz", "<f8"),
                        ("dll_zeta", "<f8"), ("dll_gain", "<f8"), ("pll_bw_hz", "<f8"),
                        ("pll_zeta", "<f8"), ("pll_gain", "<f8"), ("fll_bw_hz", "<f8")])
LOOP_STATE = np.dtype([("carr_hz", "<f8"), ("code_cps", "<f8"), ("fll_basis_hz", "<f8"),
                       ("pll_nco_hz", "<f8"), ("pll_err_prev", "<f8"), ("dll_nco_cps", "<f8"),
                       ("dll_err_prev", "<f8"), ("prompt_i_prev", "<i4"),
                       ("prompt_q_prev", "<i4"), ("have_prev", "<i4"), ("reserved", "<i4")])
assert LOOP_PARAMS.itemsize == 72 and LOOP_STATE.itemsize == 72
ACQ_RESULT = np.dtype([("prn", "<i4"), ("bin", "<i4"), ("tau", "<i4"), ("acquired", "<i4"),
                       ("peak", "<u8"), ("second", "<u8"), ("doppler_hz", "<f8"),
                       ("code_phase_chips", "<f8"), ("metric", "<f8")])
assert ACQ_RESULT.itemsize == 56


class GcError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__("%s: %s (%d)" % (where, gc_strerror(status), status))
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libgnsscorr.so is not built (run __graft_entry__.build() or "
                          "python -m paper_1907_00463_amd.build)")
    lib = C.CDLL(LIB_PATH)
    P, I32, U32, U64, D = C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64, C.c_double
    sig = {
        "gc_strerror": ([I32], C.c_char_p),
        "gc_version": ([P, P], I32),
        "gc_create": ([P, I32], I32),
        "gc_destroy": ([P], I32),
        "gc_nco_init": ([D, D, D, D, D, I32, P], I32),
        "gc_code_table": ([P, I32, P], I32),
        "gc_carrier_f32_error": ([P, U32, U32, P], I32),
        "gc_plan_create": ([P, I32, I32, P, I32, P], I32),
        "gc_plan_destroy": ([P], I32),
        "gc_plan_info": ([P, P, P], I32),
        "gc_correlate": ([P, P, U64, P, P, P, P, P, U32, P], I32),
        "gc_correlate_noalloc": ([P, I32, I32, P, I32, I32, P, U64, P, P, P, P, P, U32, P], I32),
        "gc_plan_timing": ([P, I32], I32),
        "gc_plan_kernel_ms": ([P, I32, P], I32),
        "gc_plan_set_kernels": ([P, I32], I32),
        "gc_batch_create": ([P, P, I32, P, P, I32, P, P, P, P, P, U32, P], I32),
        "gc_batch_configure": ([P, I32, I32, I32], I32),
        "gc_batch_tune": ([P, I32], I32),
        "gc_batch_launch": ([P, P], I32),
        "gc_batch_info": ([P, P, P, P, P, P, P, P], I32),
        "gc_batch_destroy": ([P], I32),
        "gc_server_create": ([P, U64, U64, I32, I32, U32, I32, I32, I32, P], I32),
        "gc_server_open_rx": ([P, I32, P, P, I32, P], I32),
        "gc_server_submit": ([P, I32, P, U64, P], I32),
        "gc_server_hold": ([P, I32], I32),
        "gc_server_poll": ([P, P, I32, P], I32),
        "gc_server_result": ([P, U64, P, P, P, P, P], I32),
        "gc_server_state": ([P, I32, P], I32),
        "gc_server_info": ([P, P, P, P, P, P, P], I32),
        "gc_server_destroy": ([P], I32),
        "gc_server_stats": ([P, P], I32),
        "gc_loop_init": ([D, D, P], I32),
        "gc_track": ([P, P, U64, P, P, P, P, P, P, P, U32, P], I32),
        "gc_acq_create": ([P, I32, I32, D, D, D, I32, P, I32, I32, I32, P], I32),
        "gc_acquire": ([P, P, U64, D, P, P, P], I32),
        "gc_acq_info": ([P, P, P, P, P], I32),
        "gc_acq_destroy": ([P], I32),
        "gc_acq_timing": ([P, I32], I32),
        "gc_acq_kernel_ms": ([P, I32, P], I32),
        "gc_lock_metrics": ([P, P, I32, I32, P, I32, U32, U32, D, D, P, P, P, U32, P, P, P, P,
                             P, U32, P, P], I32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()
EXPORTED = ("gc_strerror", "gc_version", "gc_create", "gc_destroy", "gc_nco_init",
            "gc_code_table", "gc_carrier_f32_error", "gc_plan_create", "gc_plan_destroy", "gc_plan_info",
            "gc_correlate", "gc_correlate_noalloc", "gc_plan_timing", "gc_plan_kernel_ms", "gc_plan_set_kernels",
            "gc_batch_create", "gc_batch_configure", "gc_batch_tune", "gc_batch_launch",
            "gc_batch_info", "gc_batch_destroy", "gc_server_create", "gc_server_open_rx",
            "gc_server_submit", "gc_server_hold", "gc_server_poll", "gc_server_result", "gc_server_state",
            "gc_server_info", "gc_server_destroy", "gc_server_stats", "gc_loop_init",
            "gc_track", "gc_lock_metrics", "gc_acq_create", "gc_acquire", "gc_acq_info",
            "gc_acq_destroy", "gc_acq_timing", "gc_acq_kernel_ms")


def _check(rc: int, where: str):
    if rc != GC_OK:
        raise GcError(rc, where)


def _ptr(a) -> Optional[int]:
    """Address of a numpy array, a torch tensor or an int."""
    if a is None:
        return None
    if isinstance(a, int):
        return a
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


# ------------------------------------------------------------------ C entry points
def gc_strerror(status: int) -> str:
    return _lib.gc_strerror(status).decode()


def gc_version():
    a, b = C.c_int32(), C.c_int32()
    _check(_lib.gc_version(C.byref(a), C.byref(b)), "gc_version")
    return a.value, b.value


def gc_create(device: int = 0) -> int:
    h = C.c_void_p()
    _check(_lib.gc_create(C.byref(h), device), "gc_create")
    return h.value


def gc_destroy(ctx: int) -> None:
    _check(_lib.gc_destroy(ctx), "gc_destroy")


def gc_nco_init(fs_hz, carr_hz, carr_phase_cyc, code_rate_cps, code_phase_chips,
                int_periods) -> np.ndarray:
    st = np.zeros(1, CHAN_STATE)
    _check(_lib.gc_nco_init(fs_hz, carr_hz, carr_phase_cyc, code_rate_cps, code_phase_chips,
                            int_periods, st.ctypes.data), "gc_nco_init")
    return st[0]


def gc_code_table(ctx: int, prn: int) -> np.ndarray:
    out = np.zeros(1023, np.int8)
    _check(_lib.gc_code_table(ctx, prn, out.ctypes.data), "gc_code_table")
    return out


def gc_carrier_f32_error(ctx: int, first_bits: int = 0, count: int = 0x3F800000):
    """Largest |error| (cos, sin) of the float carrier's sin/cos over fp32 phases
    with bit patterns first_bits .. first_bits + count - 1, against fp64."""
    out = np.zeros(2, np.float64)
    _check(_lib.gc_carrier_f32_error(ctx, first_bits, count, out.ctypes.data),
           "gc_carrier_f32_error")
    return float(out[0]), float(out[1])


def gc_plan_create(ctx: int, fmt: int, carrier: int, cfg: np.ndarray) -> int:
    cfg = np.ascontiguousarray(cfg, dtype=CHAN_CFG)
    h = C.c_void_p()
    _check(_lib.gc_plan_create(ctx, fmt, carrier, cfg.ctypes.data, len(cfg), C.byref(h)),
           "gc_plan_create")
    return h.value


def gc_plan_destroy(plan: int) -> None:
    _check(_lib.gc_plan_destroy(plan), "gc_plan_destroy")


def gc_plan_set_kernels(plan: int, mask: int) -> None:
    _check(_lib.gc_plan_set_kernels(plan, mask), "gc_plan_set_kernels")


def gc_plan_info(plan: int):
    a, b = C.c_int32(), C.c_int32()
    _check(_lib.gc_plan_info(plan, C.byref(a), C.byref(b)), "gc_plan_info")
    return a.value, b.value


def gc_correlate(plan: int, samples, n_samples: int, state, out, dump_n, n_dumps, status,
                 max_dumps: int, stream=None) -> int:
    """Enqueue one block; returns the gc_status of the call (per-channel status in ``status``)."""
    return _lib.gc_correlate(plan, _ptr(samples), n_samples, _ptr(state), _ptr(out),
                             _ptr(dump_n), _ptr(n_dumps), _ptr(status), max_dumps,
                             _stream_ptr(stream))


def gc_correlate_noalloc(ctx: int, fmt: int, carrier: int, cfg, n_chan: int, tap_stride: int,
                         samples, n_samples: int, state, out, dump_n, n_dumps, status,
                         max_dumps: int, stream=None) -> int:
    """Enqueue one block without a plan (``cfg`` in device memory); returns the
    gc_status of the call (per-channel status in ``status``)."""
    return _lib.gc_correlate_noalloc(ctx, fmt, carrier, _ptr(cfg), n_chan, tap_stride,
                                     _ptr(samples), n_samples, _ptr(state), _ptr(out),
                                     _ptr(dump_n), _ptr(n_dumps), _ptr(status), max_dumps,
                                     _stream_ptr(stream))


def gc_plan_timing(plan: int, n_slots: int) -> None:
    _check(_lib.gc_plan_timing(plan, n_slots), "gc_plan_timing")


def gc_plan_kernel_ms(plan: int, slot: int) -> float:
    ms = C.c_float()
    _check(_lib.gc_plan_kernel_ms(plan, slot, C.byref(ms)), "gc_plan_kernel_ms")
    return ms.value


def gc_batch_create(ctx: int, rx: np.ndarray, cfg: np.ndarray, chan_rx: np.ndarray, state, out,
                    dump_n, n_dumps, status, max_dumps: int) -> int:
    rx = np.ascontiguousarray(rx, dtype=RX_DESC)
    cfg = np.ascontiguousarray(cfg, dtype=CHAN_CFG)
    chan_rx = np.ascontiguousarray(chan_rx, dtype=np.int32)
    h = C.c_void_p()
    _check(_lib.gc_batch_create(ctx, rx.ctypes.data, len(rx), cfg.ctypes.data,
                                chan_rx.ctypes.data, len(cfg), _ptr(state), _ptr(out),
                                _ptr(dump_n), _ptr(n_dumps), _ptr(status), max_dumps,
                                C.byref(h)), "gc_batch_create")
    return h.value


def gc_batch_configure(batch: int, shape: int, grid: int = 0, periodic_chunk: int = 0) -> None:
    _check(_lib.gc_batch_configure(batch, shape, grid, periodic_chunk), "gc_batch_configure")


def gc_batch_tune(batch: int, reps: int = 3) -> None:
    _check(_lib.gc_batch_tune(batch, reps), "gc_batch_tune")


def gc_batch_launch(batch: int, stream=None) -> None:
    _check(_lib.gc_batch_launch(batch, _stream_ptr(stream)), "gc_batch_launch")


def gc_batch_info(batch: int) -> dict:
    a, b, c, d = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    pc, pi = C.c_int32(), C.c_int32()
    ms = C.c_float()
    _check(_lib.gc_batch_info(batch, C.byref(a), C.byref(b), C.byref(c), C.byref(d), C.byref(ms),
                              C.byref(pc), C.byref(pi)), "gc_batch_info")
    return {"shape": a.value, "grid": b.value, "n_items": c.value, "n_shapes": d.value,
            "tuned_ms": ms.value, "periodic_chunk": pc.value, "periodic_items": pi.value}


def gc_batch_destroy(batch: int) -> None:
    _check(_lib.gc_batch_destroy(batch), "gc_batch_destroy")


def gc_server_create(ctx: int, hbm_budget: int, host_budget: int, max_channels: int,
                     max_receivers: int, max_dumps: int, n_streams: int = 2,
                     max_batch_rx: int = 256, flags: int = 0) -> int:
    h = C.c_void_p()
    _check(_lib.gc_server_create(ctx, hbm_budget, host_budget, max_channels, max_receivers,
                                 max_dumps, n_streams, max_batch_rx, flags, C.byref(h)),
           "gc_server_create")
    return h.value


def gc_server_open_rx(server: int, fmt: int, cfg: np.ndarray, state0: np.ndarray) -> int:
    cfg = np.ascontiguousarray(cfg, dtype=CHAN_CFG)
    state0 = np.ascontiguousarray(state0, dtype=CHAN_STATE)
    assert len(cfg) == len(state0)
    r = C.c_int32()
    _check(_lib.gc_server_open_rx(server, fmt, cfg.ctypes.data, state0.ctypes.data, len(cfg),
                                  C.byref(r)), "gc_server_open_rx")
    return r.value


def gc_server_submit(server: int, rx_id: int, samples: np.ndarray, n_samples: int):
    """Returns the request id, or None when admission is refused (GC_EBUSY)."""
    samples = np.ascontiguousarray(samples, dtype=np.uint8)
    rid = C.c_uint64()
    rc = _lib.gc_server_submit(server, rx_id, samples.ctypes.data, n_samples, C.byref(rid))
    if rc == GC_EBUSY:
        return None
    _check(rc, "gc_server_submit")
    return rid.value


def gc_server_hold(server: int, hold: bool) -> None:
    _check(_lib.gc_server_hold(server, int(bool(hold))), "gc_server_hold")


def gc_server_poll(server: int, max_n: int = 4096) -> np.ndarray:
    ids = np.zeros(max_n, np.uint64)
    n = C.c_int32()
    _check(_lib.gc_server_poll(server, ids.ctypes.data, max_n, C.byref(n)), "gc_server_poll")
    return ids[: n.value]


def gc_server_result(server: int, req_id: int, n_chan: int, max_dumps: int):
    """(out, dump_n, n_dumps, status, service_s) of a finished request, or
    None when it is not finished (GC_EAGAIN)."""
    out = np.zeros((n_chan, max_dumps, 4, 2), np.int32)
    dump_n = np.zeros((n_chan, max_dumps), np.uint32)
    n_dumps = np.zeros(n_chan, np.uint32)
    status = np.zeros(n_chan, np.int32)
    svc = np.zeros(1, np.float64)
    rc = _lib.gc_server_result(server, req_id, out.ctypes.data, dump_n.ctypes.data,
                               n_dumps.ctypes.data, status.ctypes.data, svc.ctypes.data)
    if rc == GC_EAGAIN:
        return None
    _check(rc, "gc_server_result")
    return out, dump_n, n_dumps, status, float(svc[0])


def gc_server_state(server: int, rx_id: int, n_chan: int) -> np.ndarray:
    st = np.zeros(n_chan, CHAN_STATE)
    _check(_lib.gc_server_state(server, rx_id, st.ctypes.data), "gc_server_state")
    return st


def gc_server_info(server: int) -> dict:
    md, ts, fl = C.c_uint32(), C.c_int32(), C.c_int32()
    hb, ln, lr = C.c_uint64(), C.c_uint64(), C.c_uint64()
    _check(_lib.gc_server_info(server, C.byref(md), C.byref(ts), C.byref(fl), C.byref(hb),
                               C.byref(ln), C.byref(lr)), "gc_server_info")
    return {"max_dumps": md.value, "tap_stride": ts.value, "in_flight": fl.value,
            "hbm_in_use": hb.value, "launches": ln.value, "launched_requests": lr.value}


def gc_server_stats(server: int) -> dict:
    t = np.zeros(1, SERVER_TIMING)
    _check(_lib.gc_server_stats(server, t.ctypes.data), "gc_server_stats")
    return {k: t[0][k].item() for k in SERVER_TIMING.names}


def gc_server_destroy(server: int) -> None:
    _check(_lib.gc_server_destroy(server), "gc_server_destroy")


def loop_params(fs_hz, if_hz, dll_bw_hz=2.0, dll_zeta=0.7, dll_gain=1.0, pll_bw_hz=25.0,
                pll_zeta=0.7, pll_gain=0.25, fll_bw_hz=10.0) -> np.ndarray:
    p = np.zeros(1, LOOP_PARAMS)
    p[0] = (fs_hz, if_hz, dll_bw_hz, dll_zeta, dll_gain, pll_bw_hz, pll_zeta, pll_gain, fll_bw_hz)
    return p


def gc_loop_init(carr_hz: float, code_cps: float) -> np.ndarray:
    st = np.zeros(1, LOOP_STATE)
    _check(_lib.gc_loop_init(carr_hz, code_cps, st.ctypes.data), "gc_loop_init")
    return st[0]


def gc_track(plan: int, samples, n_samples: int, params: np.ndarray, state, loop, rows, dump_n,
             n_dumps, status, max_dumps: int, stream=None) -> int:
    """Enqueue closed-loop tracking of one block; returns the gc_status of the call."""
    params = np.ascontiguousarray(params, dtype=LOOP_PARAMS)
    return _lib.gc_track(plan, _ptr(samples), n_samples, params.ctypes.data, _ptr(state),
                         _ptr(loop), _ptr(rows), _ptr(dump_n), _ptr(n_dumps), _ptr(status),
                         max_dumps, _stream_ptr(stream))


def gc_lock_metrics(ctx: int, rows, row_stride: int, prompt_col: int, n_dumps, n_chan: int,
                    max_dumps: int, window: int, dump_s: float, lock_min: float, phase, cn0, lock,
                    max_windows: int, n_windows, lock_fails, hist, edge, bits, max_bits: int,
                    n_bits, stream=None) -> int:
    """Enqueue lock metrics and bit synchronisation; returns the gc_status of the call."""
    return _lib.gc_lock_metrics(ctx, _ptr(rows), row_stride, prompt_col, _ptr(n_dumps), n_chan,
                                max_dumps, window, dump_s, lock_min, _ptr(phase), _ptr(cn0),
                                _ptr(lock), max_windows, _ptr(n_windows), _ptr(lock_fails),
                                _ptr(hist), _ptr(edge), _ptr(bits), max_bits, _ptr(n_bits),
                                _stream_ptr(stream))


def gc_acq_create(ctx: int, fmt: int, samples_per_chip: int, if_hz: float, f_lo_hz: float,
                  f_step_hz: float, n_bins: int, prns, coherent_periods: int, blocks: int) -> int:
    prns = np.ascontiguousarray(prns, dtype=np.int32)
    h = C.c_void_p()
    _check(_lib.gc_acq_create(ctx, fmt, samples_per_chip, if_hz, f_lo_hz, f_step_hz, n_bins,
                              prns.ctypes.data, len(prns), coherent_periods, blocks, C.byref(h)),
           "gc_acq_create")
    return h.value


def gc_acquire(acq: int, samples, n_samples: int, threshold: float, surface, results,
               stream=None) -> int:
    """Enqueue one search; returns the gc_status of the call."""
    return _lib.gc_acquire(acq, _ptr(samples), n_samples, threshold, _ptr(surface),
                           _ptr(results), _stream_ptr(stream))


def gc_acq_info(acq: int) -> dict:
    dg = C.c_int32()
    sb = C.c_uint64()
    ns = C.c_uint64()
    rt = C.c_int32()
    _check(_lib.gc_acq_info(acq, C.byref(dg), C.byref(sb), C.byref(ns), C.byref(rt)),
           "gc_acq_info")
    return {"digits": dg.value, "scratch_bytes": sb.value, "samples_needed": ns.value,
            "row_tile": rt.value}


def gc_acq_timing(acq: int, n_slots: int) -> None:
    _check(_lib.gc_acq_timing(acq, n_slots), "gc_acq_timing")


def gc_acq_kernel_ms(acq: int, slot: int):
    """Durations (ms) of the four kernels of a timed call: sums, contraction,
    reduction, detection."""
    ms = (C.c_float * 4)()
    _check(_lib.gc_acq_kernel_ms(acq, slot, ms), "gc_acq_kernel_ms")
    return [float(v) for v in ms]


def gc_acq_destroy(acq: int) -> None:
    _check(_lib.gc_acq_destroy(acq), "gc_acq_destroy")


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------------------ conveniences
def make_cfg(prn: int, taps_q32: Sequence[int], int_periods: int = 1) -> np.ndarray:
    c = np.zeros((), CHAN_CFG)
    taps = np.asarray(taps_q32, dtype=np.int64)
    c["prn"] = prn
    c["n_taps"] = len(taps)
    c["int_periods"] = int_periods
    c["tap_q32"][: len(taps)] = taps
    return c


def max_dumps_for(n_samples: int, code_step_max: int, int_periods_min: int = 1) -> int:
    """Upper bound on dumps one block can close (phase < W at entry)."""
    W = int_periods_min * 1023 * TWO32
    return (n_samples * code_step_max) // W + 2


class Plan:
    """A plan plus the device buffers one call needs (torch tensors on the plan's device)."""

    def __init__(self, ctx: int, fmt: int, carrier: int, cfgs: np.ndarray, device=None):
        import torch

        self.torch = torch
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self.cfgs = np.ascontiguousarray(cfgs, dtype=CHAN_CFG)
        self.fmt, self.carrier = fmt, carrier
        self.handle = gc_plan_create(ctx, fmt, carrier, self.cfgs)
        self.tap_stride, self.n_chan = gc_plan_info(self.handle)

    def close(self):
        if self.handle:
            gc_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def states_to_device(self, states: np.ndarray):
        b = np.ascontiguousarray(states, dtype=CHAN_STATE).view(np.uint8)
        return self.torch.from_numpy(b.copy()).to(self.device)

    @staticmethod
    def states_from_device(t) -> np.ndarray:
        return t.cpu().numpy().view(CHAN_STATE).copy()

    def outputs(self, max_dumps: int):
        torch = self.torch
        dt = torch.int32 if self.carrier == GC_CARRIER_LUT else torch.float32
        out = torch.zeros((self.n_chan, max_dumps, self.tap_stride, 2), dtype=dt, device=self.device)
        dump_n = torch.zeros((self.n_chan, max_dumps), dtype=torch.int32, device=self.device)
        n_dumps = torch.zeros(self.n_chan, dtype=torch.int32, device=self.device)
        status = torch.zeros(self.n_chan, dtype=torch.int32, device=self.device)
        return out, dump_n, n_dumps, status

    def correlate(self, samples, n_samples: int, state, out, dump_n, n_dumps, status,
                  stream=None):
        max_dumps = out.shape[1]
        rc = gc_correlate(self.handle, samples, n_samples, state, out, dump_n, n_dumps, status,
                          max_dumps, stream if stream is not None
                          else self.torch.cuda.current_stream(self.device))
        _check(rc, "gc_correlate")


class Batch:
    """A batch of receivers bound to its device buffers (torch tensors): the
    receivers' sample blocks, the channel states and the outputs."""

    def __init__(self, ctx: int, blocks, fmts, n_samples, cfgs: np.ndarray, chan_rx,
                 states: np.ndarray, max_dumps: int, device=None):
        import torch

        self.torch = torch
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self.blocks = list(blocks)           # keep the sample tensors alive
        self.cfgs = np.ascontiguousarray(cfgs, dtype=CHAN_CFG)
        n_chan = len(self.cfgs)
        self.tap_stride = int(self.cfgs["n_taps"].max())
        self.max_dumps = max_dumps
        rx = np.zeros(len(self.blocks), RX_DESC)
        for r, (b, f, n) in enumerate(zip(self.blocks, fmts, n_samples)):
            rx[r]["samples"] = b.data_ptr()
            rx[r]["n_samples"] = n
            rx[r]["fmt"] = f
        b = np.ascontiguousarray(states, dtype=CHAN_STATE).view(np.uint8)
        self.state = torch.from_numpy(b.copy()).to(self.device)
        self.out = torch.zeros((n_chan, max_dumps, self.tap_stride, 2), dtype=torch.int32,
                               device=self.device)
        self.dump_n = torch.zeros((n_chan, max_dumps), dtype=torch.int32, device=self.device)
        self.n_dumps = torch.zeros(n_chan, dtype=torch.int32, device=self.device)
        self.status = torch.zeros(n_chan, dtype=torch.int32, device=self.device)
        self.handle = gc_batch_create(ctx, rx, self.cfgs, chan_rx, self.state, self.out,
                                      self.dump_n, self.n_dumps, self.status, max_dumps)

    def configure(self, shape: int, grid: int = 0, periodic_chunk: int = 0):
        gc_batch_configure(self.handle, shape, grid, periodic_chunk)

    def tune(self, reps: int = 3):
        gc_batch_tune(self.handle, reps)

    def launch(self, stream=None):
        gc_batch_launch(self.handle, stream if stream is not None
                        else self.torch.cuda.current_stream(self.device))

    def info(self) -> dict:
        return gc_batch_info(self.handle)

    def states(self) -> np.ndarray:
        return self.state.cpu().numpy().view(CHAN_STATE).copy()

    def close(self):
        if self.handle:
            gc_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
