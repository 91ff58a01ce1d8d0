"""The C ABI: exports, struct layouts, host-side validation and the host NCO
helper.  No compute call is made here (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gnsscorr.h")
LIB = os.path.join(ROOT, "paper_1907_00463_amd", "libgnsscorr.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libgnsscorr.so not built")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gc_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    import ctypes
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    nm = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (gc_\w+)", nm))
    assert set(names) <= exported
    from paper_1907_00463_amd import gnsscorr
    assert set(gnsscorr.EXPORTED) == set(names)


def test_struct_layout_matches_header(tmp_path):
    from paper_1907_00463_amd import gnsscorr
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "gnsscorr.h"
int main(void) {
  printf("%zu %zu\n", sizeof(gc_chan_cfg), sizeof(gc_chan_state));
  printf("%zu %zu %zu\n", offsetof(gc_chan_cfg, tap_q32), offsetof(gc_chan_state, carr_phase_f),
         offsetof(gc_chan_state, acc));
  printf("%zu %zu %zu\n", offsetof(gc_chan_state, acc_f), offsetof(gc_chan_state, acc_n),
         offsetof(gc_chan_state, carr_step));
  printf("%zu %zu %zu %zu\n", sizeof(gc_rx_desc), offsetof(gc_rx_desc, n_samples),
         offsetof(gc_rx_desc, fmt), offsetof(gc_rx_desc, reserved));
  printf("%zu %zu %zu\n", sizeof(gc_server_timing), offsetof(gc_server_timing, enqueue_mean_ms),
         offsetof(gc_server_timing, submit_max_ms));
  printf("%zu %zu %zu %zu %zu\n", sizeof(gc_loop_params), offsetof(gc_loop_params, fll_bw_hz),
         sizeof(gc_loop_state), offsetof(gc_loop_state, prompt_i_prev),
         offsetof(gc_loop_state, have_prev));
  printf("%zu %zu %zu %zu\n", sizeof(gc_acq_result), offsetof(gc_acq_result, peak),
         offsetof(gc_acq_result, doppler_hz), offsetof(gc_acq_result, metric));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    vals = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    cfg, st, rx = gnsscorr.CHAN_CFG, gnsscorr.CHAN_STATE, gnsscorr.RX_DESC
    assert vals == [cfg.itemsize, st.itemsize, cfg.fields["tap_q32"][1],
                    st.fields["carr_phase_f"][1], st.fields["acc"][1],
                    st.fields["acc_f"][1], st.fields["acc_n"][1], st.fields["carr_step"][1],
                    rx.itemsize, rx.fields["n_samples"][1], rx.fields["fmt"][1],
                    rx.fields["reserved"][1], gnsscorr.SERVER_TIMING.itemsize,
                    gnsscorr.SERVER_TIMING.fields["enqueue_mean_ms"][1],
                    gnsscorr.SERVER_TIMING.fields["submit_max_ms"][1],
                    gnsscorr.LOOP_PARAMS.itemsize, gnsscorr.LOOP_PARAMS.fields["fll_bw_hz"][1],
                    gnsscorr.LOOP_STATE.itemsize, gnsscorr.LOOP_STATE.fields["prompt_i_prev"][1],
                    gnsscorr.LOOP_STATE.fields["have_prev"][1],
                    gnsscorr.ACQ_RESULT.itemsize, gnsscorr.ACQ_RESULT.fields["peak"][1],
                    gnsscorr.ACQ_RESULT.fields["doppler_hz"][1],
                    gnsscorr.ACQ_RESULT.fields["metric"][1]]


def test_host_validation_without_a_device():
    from paper_1907_00463_amd import gnsscorr as g
    assert g._lib.gc_plan_create(None, 0, 0, None, 1, None) == g.GC_EINVAL
    assert g._lib.gc_correlate(None, None, 0, None, None, None, None, None, 1, None) == g.GC_EINVAL
    assert g._lib.gc_destroy(None) == g.GC_EINVAL
    assert g._lib.gc_carrier_f32_error(None, 0, 1, None) == g.GC_EINVAL
    # the allocation-free entry point: null context, then sizes past the fixed array
    assert g._lib.gc_correlate_noalloc(None, 0, 0, None, 1, 3, None, 0, None, None, None, None,
                                       None, 1, None) == g.GC_EINVAL
    assert g._lib.gc_plan_destroy(None) == g.GC_EINVAL
    assert g._lib.gc_code_table(None, 1, None) == g.GC_EINVAL
    assert g._lib.gc_batch_create(None, None, 1, None, None, 1, None, None, None, None, None,
                                  1, None) == g.GC_EINVAL
    assert g._lib.gc_batch_destroy(None) == g.GC_EINVAL
    assert g._lib.gc_server_create(None, 1 << 20, 1 << 20, 1, 1, 8, 1, 1, 0,
                                   None) == g.GC_EINVAL
    assert g._lib.gc_server_submit(None, 0, None, 0, None) == g.GC_EINVAL
    assert g._lib.gc_server_poll(None, None, 0, None) == g.GC_EINVAL
    assert g._lib.gc_server_result(None, 1, None, None, None, None, None) == g.GC_EINVAL
    assert g._lib.gc_server_destroy(None) == g.GC_EINVAL
    assert g._lib.gc_server_stats(None, None) == g.GC_EINVAL
    assert g._lib.gc_loop_init(1.0, 1.0, None) == g.GC_EINVAL
    assert g._lib.gc_track(None, None, 0, None, None, None, None, None, None, None, 1,
                           None) == g.GC_EINVAL
    assert g._lib.gc_lock_metrics(None, None, 8, 2, None, 1, 1, 20, 1e-3, 0.5, None, None,
                                  None, 0, None, None, None, None, None, 0, None,
                                  None) == g.GC_EINVAL
    prns = (C.c_int32 * 1)(1)
    assert g._lib.gc_acq_create(None, 0, 4, 0.0, 0.0, 1.0, 1, prns, 1, 1, 1, None) == g.GC_EINVAL
    assert g._lib.gc_acquire(None, None, 0, 2.5, None, None, None) == g.GC_EINVAL
    assert g._lib.gc_acq_info(None, None, None, None, None) == g.GC_EINVAL
    assert g._lib.gc_acq_destroy(None) == g.GC_EINVAL
    ls = g.gc_loop_init(4.0e6, 1.023e6)
    assert ls["carr_hz"] == 4.0e6 and ls["fll_basis_hz"] == 4.0e6 and ls["have_prev"] == 0
    assert g.gc_version() == (1, 0)
    for s in (0, -1, -2, -3, -4, -5, -6, -7):
        assert len(g.gc_strerror(s)) > 0
    with pytest.raises(g.GcError):
        g.gc_nco_init(0.0, 1e6, 0.0, 1.023e6, 0.0, 1)
    with pytest.raises(g.GcError):  # fewer than 2 samples per chip
        g.gc_nco_init(1.5e6, 1e3, 0.0, 1.023e6, 0.0, 1)


@pytest.mark.parametrize("seed", range(20))
def test_nco_init_equals_oracle_words(seed):
    # two implementations of the same written definition (round half even, mod)
    from paper_1907_00463_amd import gnsscorr as g
    rng = np.random.default_rng(seed)
    fs = float(rng.choice([4.092e6, 8.184e6, 16.368e6, 20.46e6, 5e6, 25e6]))
    carr = float(rng.uniform(-fs / 2, fs / 2))
    ph = float(rng.uniform(-3, 3))
    rate = 1.023e6 * (1 + float(rng.uniform(-5e3, 5e3)) / 1575.42e6)
    T = int(rng.choice([1, 4, 20]))
    p0 = float(rng.uniform(-5000, 30000))
    st = g.gc_nco_init(fs, carr, ph, rate, p0, T)
    cp, cs, kp, ks = oracle.nco_words(fs, carr, ph, rate, p0, T)
    assert (int(st["carr_phase"]), int(st["carr_step"]), int(st["code_phase"]),
            int(st["code_step"])) == (cp, cs, kp, ks)
    assert st["acc_n"] == 0 and not st["acc"].any()
    assert abs(st["carr_freq_f"] - carr / fs) == 0.0
    assert 0.0 <= st["carr_phase_f"] < 1.0
