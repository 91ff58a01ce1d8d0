"""The allocation-free entry point gc_correlate_noalloc against gc_correlate
through a plan, on the same channels and blocks: integer results bit for bit
(dumps, sample counts, per-channel status and the final channel states),
float-carrier results within the FP32 tolerance on |P|.  Each case makes two
calls in a row, the second on a smaller block and with fewer channels, so the
fixed device array still holds the first call's records past the second's
channels."""
import numpy as np
import pytest

from gpu_util import TWO32, block_bytes, c10_check

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def g():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1907_00463_amd import gnsscorr
    return gnsscorr


@pytest.fixture(scope="module")
def ctx(g):
    c = g.gc_create(0)
    yield c
    g.gc_destroy(c)


def _dev(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.uint8).copy()).cuda()


def _outputs(g, carrier, n_chan, max_dumps, tap_stride):
    dt = torch.int32 if carrier == g.GC_CARRIER_LUT else torch.float32
    # filled with a pattern, so rows a call must write and leaves unwritten differ
    out = torch.full((n_chan, max_dumps, tap_stride, 2), 7, dtype=dt, device="cuda")
    dump_n = torch.full((n_chan, max_dumps), 7, dtype=torch.int32, device="cuda")
    n_dumps = torch.full((n_chan,), 7, dtype=torch.int32, device="cuda")
    status = torch.full((n_chan,), 7, dtype=torch.int32, device="cuda")
    return out, dump_n, n_dumps, status


def _host(t):
    return tuple(x.cpu().numpy() for x in t)


def _run_plan(g, ctx, fmt, carrier, cfgs, states, buf, n, max_dumps):
    plan = g.Plan(ctx, fmt, carrier, cfgs)
    try:
        st = plan.states_to_device(states)
        o = _outputs(g, carrier, len(cfgs), max_dumps, plan.tap_stride)
        plan.correlate(_dev(buf), n, st, *o)
        torch.cuda.synchronize()
        return _host(o), plan.states_from_device(st), plan.tap_stride
    finally:
        plan.close()


def _run_noalloc(g, ctx, fmt, carrier, cfgs, states, buf, n, max_dumps, tap_stride):
    st = _dev(states)
    cfg_dev = _dev(cfgs)
    o = _outputs(g, carrier, len(cfgs), max_dumps, tap_stride)
    rc = g.gc_correlate_noalloc(ctx, fmt, carrier, cfg_dev, len(cfgs), tap_stride, _dev(buf), n,
                                st, *o, max_dumps, torch.cuda.current_stream())
    assert rc == g.GC_OK, g.gc_strerror(rc)
    torch.cuda.synchronize()
    return _host(o), st.cpu().numpy().view(g.CHAN_STATE).copy()


def _compare(g, carrier, a, b, sa, sb, cfgs, sigma=None):
    (out_a, dn_a, nd_a, st_a), (out_b, dn_b, nd_b, st_b) = a, b
    assert np.array_equal(st_a, st_b)
    assert np.array_equal(nd_a, nd_b)
    for c in range(len(cfgs)):
        nd = int(nd_b[c])
        K = int(cfgs[c]["n_taps"])
        assert np.array_equal(dn_a[c, :nd], dn_b[c, :nd]), c
        if carrier == g.GC_CARRIER_LUT:
            assert np.array_equal(out_a[c, :nd, :K], out_b[c, :nd, :K]), c
        else:
            ok, worst = c10_check(out_a[c, :nd, :K].astype(np.float64),
                                  out_b[c, :nd, :K].astype(np.float64), sigma)
            assert ok.all(), (c, worst)
    for f in ("code_phase", "code_step", "carr_phase", "carr_step", "acc_n"):
        assert np.array_equal(sa[f], sb[f]), f
    if carrier == g.GC_CARRIER_LUT:
        assert np.array_equal(sa["acc"], sb["acc"])
    else:
        assert np.allclose(sa["acc_f"], sb["acc_f"], rtol=1e-5, atol=1e-5 * (sigma or 1.0))


def _two_calls(g, ctx, fmt, carrier, cfgs, states, bufs, ns, k2, sigma=None):
    """Call 1: every channel on block 0.  Call 2: the first k2 channels, from
    the states call 1 left, on block 1 (smaller)."""
    md = [g.max_dumps_for(n, int(states["code_step"].max()), int(cfgs["int_periods"].min()))
          for n in ns]
    p1, ps1, stride = _run_plan(g, ctx, fmt, carrier, cfgs, states, bufs[0], ns[0], md[0])
    a1, as1 = _run_noalloc(g, ctx, fmt, carrier, cfgs, states, bufs[0], ns[0], md[0], stride)
    _compare(g, carrier, a1, p1, as1, ps1, cfgs, sigma)
    c2 = cfgs[:k2].copy()
    s2 = ps1[:k2].copy()
    p2, ps2, stride2 = _run_plan(g, ctx, fmt, carrier, c2, s2, bufs[1], ns[1], md[1])
    a2, as2 = _run_noalloc(g, ctx, fmt, carrier, c2, s2, bufs[1], ns[1], md[1], stride2)
    _compare(g, carrier, a2, p2, as2, ps2, c2, sigma)
    return p1, p2


def _chans(g, rng, n_chan, fs, if_hz, taps, periods=(1,)):
    cfgs = np.zeros(n_chan, g.CHAN_CFG)
    states = np.zeros(n_chan, g.CHAN_STATE)
    prns = rng.choice(np.arange(1, 33), size=n_chan, replace=False)
    for i in range(n_chan):
        T = int(rng.choice(periods))
        fd = float(rng.uniform(-5000.0, 5000.0))
        cfgs[i] = g.make_cfg(int(prns[i]), taps, T)
        states[i] = g.gc_nco_init(fs, if_hz + fd, float(rng.random()),
                                  1.023e6 * (1.0 + fd / 1575.42e6),
                                  float(rng.uniform(0.0, 1023.0 * T)), T)
    return cfgs, states


def test_noalloc_periodic_2bit_equals_plan(g, ctx):
    """2-bit real at 16.368 MHz (half chips of 8 samples): periodic kernel."""
    rng = np.random.default_rng(7001)
    fs = 16.368e6
    cfgs, states = _chans(g, rng, 12, fs, fs / 4, np.array([1 << 31, 0, -(1 << 31)], np.int64),
                          periods=(1, 4, 20))
    ns = [1_636_800, 409_200]
    bufs = [rng.integers(0, 256, size=block_bytes(2, n), dtype=np.uint8) for n in ns]
    p1, _ = _two_calls(g, ctx, 2, g.GC_CARRIER_LUT, cfgs, states, bufs, ns, 5)
    assert np.all(p1[3] == 0) and p1[2].sum() > 100


def test_noalloc_binned_iq_equals_plan(g, ctx):
    """Complex int8 at 5 MHz (the chip-by-chip kernel)."""
    rng = np.random.default_rng(7002)
    fs = 5.0e6
    cfgs, states = _chans(g, rng, 6, fs, 0.0, np.array([1 << 31, 0, -(1 << 31)], np.int64))
    ns = [500_000, 123_457]
    bufs = [rng.integers(0, 256, size=block_bytes(1, n), dtype=np.uint8) for n in ns]
    _two_calls(g, ctx, 1, g.GC_CARRIER_LUT, cfgs, states, bufs, ns, 2)


def test_noalloc_multitap_equals_plan(g, ctx):
    """128 taps at 1/32 chip on complex int8 at 20.46 MHz (the MFMA kernel),
    plus one channel off the 1/32-chip grid (the direct kernel)."""
    rng = np.random.default_rng(7003)
    fs = 20.46e6
    taps = np.array([(-64 + k) << 27 for k in range(128)], np.int64)
    cfgs, states = _chans(g, rng, 4, fs, 0.0, taps)
    off = taps.copy()
    off[5] += 12345
    cfgs[3] = g.make_cfg(int(cfgs[3]["prn"]), off, 1)
    ns = [102_300, 40_920]
    bufs = [rng.integers(0, 256, size=block_bytes(1, n), dtype=np.uint8) for n in ns]
    _two_calls(g, ctx, 1, g.GC_CARRIER_LUT, cfgs, states, bufs, ns, 3)


def test_noalloc_float_carrier_equals_plan(g, ctx):
    """FP32 carrier on real int8 (the chip-by-chip kernel, float atomics)."""
    rng = np.random.default_rng(7004)
    fs = 4.092e6
    cfgs, states = _chans(g, rng, 3, fs, fs / 4, np.array([1 << 31, 0, -(1 << 31)], np.int64))
    ns = [204_600, 40_920]
    bufs = [rng.integers(0, 256, size=block_bytes(0, n), dtype=np.uint8) for n in ns]
    # noise std of one dump component: sqrt(samples per dump * E[x^2] / 2)
    x = bufs[0].view(np.int8).astype(np.float64)
    sigma = float(np.sqrt(4092 * np.mean(x * x) / 2))
    _two_calls(g, ctx, 0, g.GC_CARRIER_F32, cfgs, states, bufs, ns, 1, sigma=sigma)


def test_noalloc_refuses_bad_channels_and_sizes(g, ctx):
    """A cfg a plan would refuse gets GC_EINVAL and is left untouched; the
    others match a plan without it.  Sizes past the fixed array are refused
    before anything is enqueued."""
    rng = np.random.default_rng(7005)
    fs = 8.184e6
    epl = np.array([1 << 31, 0, -(1 << 31)], np.int64)
    cfgs, states = _chans(g, rng, 4, fs, fs / 4, epl)
    bad = cfgs.copy()
    bad[1]["prn"] = 33
    bad[2]["tap_q32"][:4] = [1 << 31, 0, -(1 << 31), 5]   # 4 taps > tap_stride 3
    bad[2]["n_taps"] = 4
    n = 200_000
    buf = rng.integers(0, 256, size=block_bytes(0, n), dtype=np.uint8)
    md = g.max_dumps_for(n, int(states["code_step"].max()))
    a, sa = _run_noalloc(g, ctx, 0, g.GC_CARRIER_LUT, bad, states, buf, n, md, 3)
    out, dn, nd, st = a
    assert list(st) == [0, g.GC_EINVAL, g.GC_EINVAL, 0]
    assert nd[1] == 0 and nd[2] == 0
    assert np.all(out[1] == 7) and np.all(out[2] == 7)       # outputs untouched
    assert np.array_equal(sa[1:3].view(np.uint8), states[1:3].view(np.uint8))
    good = cfgs[[0, 3]]
    p, ps, _ = _run_plan(g, ctx, 0, g.GC_CARRIER_LUT, good, states[[0, 3]], buf, n, md)
    sub = tuple(x[[0, 3]] for x in a)
    _compare(g, g.GC_CARRIER_LUT, sub, p, sa[[0, 3]], ps, good)
    # sizes: one channel past the array, tap_stride 0, format 4 (none)
    big = np.repeat(cfgs[:1], g.GC_NOALLOC_MAX_CHANNELS + 1)
    o = _outputs(g, g.GC_CARRIER_LUT, 1, md, 3)
    dev = _dev(big)
    stt = _dev(np.repeat(states[:1], g.GC_NOALLOC_MAX_CHANNELS + 1))
    sb = _dev(buf)
    assert g.gc_correlate_noalloc(ctx, 0, 0, dev, g.GC_NOALLOC_MAX_CHANNELS + 1, 3, sb, n, stt,
                                  *o, md) == g.GC_EINVAL
    assert g.gc_correlate_noalloc(ctx, 0, 0, dev, 1, 0, sb, n, stt, *o, md) == g.GC_EINVAL
    assert g.gc_correlate_noalloc(ctx, 4, 0, dev, 1, 3, sb, n, stt, *o, md) == g.GC_EINVAL
    torch.cuda.synchronize()
    assert np.all(o[3].cpu().numpy() == 7)                  # nothing was enqueued
