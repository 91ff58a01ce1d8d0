"""GPU parity of the acquisition search (gc_acquire) against the CPU oracle's
FFT-based parallel code-phase search, through the C ABI: the whole power
surface bit for bit and every detection field exactly, for every sample
format, with 2- and 4-digit operands, several blocks and periods, ragged
bin counts, the synthetic signals' satellites and argument errors."""
import numpy as np
import pytest

from oracle import acquire as A

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


def _gpu(g, ctx, fmt, buf, n, R, if_hz, f_lo, f_step, bins, prns, Mc, Knc, threshold=2.5,
         surface=True):
    a = g.gc_acq_create(ctx, fmt, R, if_hz, f_lo, f_step, bins, prns, Mc, Knc)
    try:
        info = g.gc_acq_info(a)
        x = torch.from_numpy(np.ascontiguousarray(buf)).to("cuda")
        N = 1023 * R
        surf = torch.full((len(prns), bins, N), 7, dtype=torch.int64, device="cuda") \
            if surface else None
        res = torch.zeros(len(prns) * g.ACQ_RESULT.itemsize, dtype=torch.uint8, device="cuda")
        rc = g.gc_acquire(a, x, n, threshold, surf, res, torch.cuda.current_stream())
        assert rc == g.GC_OK
        torch.cuda.synchronize()
        r = res.cpu().numpy().view(g.ACQ_RESULT)
        P = surf.cpu().numpy().view(np.uint64) if surface else None
        return P, r, info
    finally:
        g.gc_acq_destroy(a)


def _same_detection(r, want, prns):
    for k, w in enumerate(want):
        got = r[k]
        assert int(got["prn"]) == prns[k]
        assert (int(got["bin"]), int(got["tau"]), int(got["peak"]), int(got["second"])) == \
            (w["bin"], w["tau"], w["peak"], w["second"]), (k, got, w)
        assert float(got["doppler_hz"]) == w["doppler_hz"]
        assert float(got["code_phase_chips"]) == w["code_phase_chips"]
        assert float(got["metric"]) == w["metric"]
        assert bool(got["acquired"]) == w["acquired"]


def _bytes(fmt, n):
    return {0: n, 1: 2 * n, 2: (n + 3) // 4}[fmt]


@pytest.mark.parametrize("fmt,R,Mc,Knc,bins,digits", [
    (2, 4, 1, 2, 7, 2),     # 2-bit real, 2 digits
    (0, 4, 1, 1, 5, 2),     # int8 real at 4 samples per chip: |S| <= 12288
    (0, 4, 2, 2, 3, 4),     # int8 real, 2 periods: 4 digits
    (1, 2, 2, 3, 4, 4),     # int8 I/Q: 4 digits
    (2, 1, 3, 2, 9, 2),     # one sample per chip, 3 periods
    (2, 5, 1, 1, 11, 2),    # an odd R: rows of a bin straddle row tiles
    (1, 1, 1, 1, 1, 2),     # one bin
])
def test_acquire_random_bytes_bit_exact(g, ctx, fmt, R, Mc, Knc, bins, digits):
    rng = np.random.default_rng(100 * R + 10 * fmt + Mc)
    n = Knc * Mc * 1023 * R
    buf = rng.integers(0, 256, _bytes(fmt, n + 8), dtype=np.uint8)
    if_hz = 0.0 if fmt == 1 else 0.25 * R * 1.023e6
    prns = [int(p) for p in rng.choice(np.arange(1, 33), 3, replace=False)] + [4]
    P, r, info = _gpu(g, ctx, fmt, buf, n + 8, R, if_hz, -3000.0, 750.0, bins, prns, Mc, Knc)
    assert info["digits"] == digits and info["samples_needed"] == n
    want = A.search(fmt, buf, R, if_hz, -3000.0, 750.0, bins, prns, Mc, Knc)
    assert np.array_equal(P, want)
    _same_detection(r, A.detect(want, R, -3000.0, 750.0, 2.5), prns)


@pytest.mark.parametrize("fmt,R,Mc,Knc,bins,digits", [
    (1, 20, 1, 2, 3, 4),    # complex int8 at 20.46 MHz: 4 digits
    (2, 32, 1, 1, 2, 2),    # the largest samples-per-chip, 2-bit
    (2, 32, 7, 1, 1, 2),    # 7 periods at R = 32: |S| <= 16128, still 2 digits
])
def test_acquire_large_rates(g, ctx, fmt, R, Mc, Knc, bins, digits):
    rng = np.random.default_rng(7 * R + fmt)
    n = Knc * Mc * 1023 * R
    buf = rng.integers(0, 256, _bytes(fmt, n), dtype=np.uint8)
    if_hz = 0.0 if fmt == 1 else 0.25 * R * 1.023e6
    prns = [11, 28]
    P, r, info = _gpu(g, ctx, fmt, buf, n, R, if_hz, -2500.0, 2500.0, bins, prns, Mc, Knc)
    assert info["digits"] == digits
    want = A.search(fmt, buf, R, if_hz, -2500.0, 2500.0, bins, prns, Mc, Knc)
    assert np.array_equal(P, want)
    _same_detection(r, A.detect(want, R, -2500.0, 2500.0, 2.5), prns)


def test_acquire_128_row_tiles(g, ctx):
    # 32 bins x 4 samples per chip x 4 rows = 512 rows, 32 PRNs: 4 tiles of
    # 128 rows give 512 blocks (one round on 256 compute units), where 6
    # tiles of 96 would need two; both digit counts
    rng = np.random.default_rng(128)
    prns = list(range(1, 33))
    for fmt, Mc, digits in ((2, 1, 2), (1, 1, 4)):
        n = Mc * 1023 * 4
        buf = rng.integers(0, 256, _bytes(fmt, n), dtype=np.uint8)
        if_hz = 0.0 if fmt == 1 else 1.023e6
        P, r, info = _gpu(g, ctx, fmt, buf, n, 4, if_hz, -8000.0, 500.0, 32, prns, Mc, 1)
        assert info["digits"] == digits
        if torch.cuda.get_device_properties(0).multi_processor_count == 256 and digits == 2:
            assert info["row_tile"] == 128
        want = A.search(fmt, buf, 4, if_hz, -8000.0, 500.0, 32, prns, Mc, 1)
        assert np.array_equal(P, want)
        _same_detection(r, A.detect(want, 4, -8000.0, 500.0, 2.5), prns)


def test_acquire_single_channel_signal(g, ctx):
    # PRN 7 at +1.5 kHz, 300.25 chips, 45 dB-Hz, int8 at 4.092 MHz; a search
    # of 8 PRNs over +-5 kHz in 500 Hz bins, 1 ms coherent, 4 blocks
    from paper_1907_00463_amd import synth
    st, chans, rng = synth.workload_single_channel(seconds=0.005)
    buf = synth.synth_samples(st, rng)
    prns = [7, 1, 2, 3, 8, 19, 25, 32]
    P, r, _ = _gpu(g, ctx, st.fmt, buf, st.n, 4, st.if_hz, -5000.0, 500.0, 21, prns, 1, 4)
    want = A.search(st.fmt, buf, 4, st.if_hz, -5000.0, 500.0, 21, prns, 1, 4)
    assert np.array_equal(P, want)
    det = A.detect(want, 4, -5000.0, 500.0, 2.5)
    _same_detection(r, det, prns)
    assert r[0]["acquired"] and int(r[0]["bin"]) == 13 and abs(int(r[0]["tau"]) - 1201) <= 1
    assert not np.any(r["acquired"][1:])


def test_acquire_twelve_channel_cold_start(g, ctx):
    # cold start on the 2-bit 16.368 MHz stream: all 32 PRNs over +-10 kHz in
    # 500 Hz bins (41), 1 ms coherent, 2 blocks; the surface is compared on
    # sampled rows (the oracle's full surface is 172 MB), every detection
    # exactly, and the satellites in the stream are found
    from paper_1907_00463_amd import synth
    st, chans, rng = synth.workload_twelve_channels(seconds=0.0021)
    buf = synth.synth_samples(st, rng)
    prns = list(range(1, 33))
    P, r, info = _gpu(g, ctx, st.fmt, buf, st.n, 16, st.if_hz, -10000.0, 500.0, 41, prns, 1, 2)
    assert info["digits"] == 2
    # 2624 rows: 28 tiles of 96 x 4 x 32 = 3584 blocks fill 7 rounds of 512
    # exactly, where 21 tiles of 128 would leave a quarter round
    assert info["row_tile"] == (96 if torch.cuda.get_device_properties(0).multi_processor_count == 256
                                else info["row_tile"])
    want = A.search(st.fmt, buf, 16, st.if_hz, -10000.0, 500.0, 41, prns, 1, 2)
    sel = np.random.default_rng(3).integers(0, 32 * 41, 64)
    for s in sel:
        p, d = divmod(int(s), 41)
        assert np.array_equal(P[p, d], want[p, d]), (p, d)
    det = A.detect(want, 16, -10000.0, 500.0, 2.5)
    _same_detection(r, det, prns)
    strong = [s for s in st.sats if s.cn0_dbhz >= 46.0]
    for s in strong:
        k = s.prn - 1
        assert r[k]["acquired"], s.prn
        assert abs(float(r[k]["doppler_hz"]) - s.doppler_hz) < 500.0
    absent = [p for p in prns if p not in [s.prn for s in st.sats]]
    assert not any(r[p - 1]["acquired"] for p in absent)


def test_acquire_bench_configuration(g, ctx):
    # the benchmark's search (32 PRNs x 41 bins x 16368 phases, 10 blocks of
    # 1 ms on the 12-channel stream): sampled (PRN, bin) rows against the
    # oracle, one bin at a time; every detection against the GPU's own full
    # surface (peak, its place, the second peak's chip rule) and, for the
    # PRNs whose peak row was sampled, against the oracle's row
    from paper_1907_00463_amd import synth
    st, chans, rng = synth.workload_twelve_channels(seconds=0.0101)
    buf = synth.synth_samples(st, rng)
    prns = list(range(1, 33))
    R, f_lo, f_step, bins, knc = 16, -10000.0, 500.0, 41, 10
    P, r, info = _gpu(g, ctx, st.fmt, buf, st.n, R, st.if_hz, f_lo, f_step, bins, prns, 1, knc)
    assert info["samples_needed"] == knc * 16368
    pick = np.random.default_rng(11).integers(0, 32 * bins, 10).tolist()
    pick += [(int(x["prn"]) - 1) * bins + int(x["bin"]) for x in r if x["acquired"]][:4]
    for sidx in pick:
        p, d = divmod(int(sidx), bins)
        row = A.search(st.fmt, buf, R, st.if_hz, f_lo + float(d) * f_step, f_step, 1, [p + 1], 1,
                       knc)
        assert np.array_equal(P[p, d], row[0, 0]), (p, d)
    N = 16368
    chips = np.arange(N) // R
    for k, x in enumerate(r):
        flat = int(np.argmax(P[k].reshape(-1)))
        d, tau = divmod(flat, N)
        assert (int(x["bin"]), int(x["tau"]), int(x["peak"])) == (d, tau, int(P[k, d, tau]))
        j = tau // R
        dist = np.minimum((chips - j) % 1023, (j - chips) % 1023)
        assert int(x["second"]) == int(P[k, d][dist >= 2].max())
        assert float(x["metric"]) == float(int(x["peak"])) / float(int(x["second"]))
    assert sum(int(x["acquired"]) for x in r) >= 10


def test_acquire_without_surface_and_repeated(g, ctx):
    # no surface requested: the same detections; a plan runs again on new data
    rng = np.random.default_rng(8)
    R, n = 2, 2 * 1023 * 2
    prns = [3, 17]
    a = g.gc_acq_create(ctx, 2, R, 0.5e6, -1000.0, 1000.0, 3, prns, 1, 2)
    try:
        for it in range(2):
            buf = rng.integers(0, 256, n // 4, dtype=np.uint8)
            x = torch.from_numpy(buf).to("cuda")
            res = torch.zeros(2 * g.ACQ_RESULT.itemsize, dtype=torch.uint8, device="cuda")
            assert g.gc_acquire(a, x, n, 1.5, None, res) == g.GC_OK
            torch.cuda.synchronize()
            r = res.cpu().numpy().view(g.ACQ_RESULT)
            want = A.search(2, buf, R, 0.5e6, -1000.0, 1000.0, 3, prns, 1, 2)
            _same_detection(r, A.detect(want, R, -1000.0, 1000.0, 1.5), prns)
    finally:
        g.gc_acq_destroy(a)


def test_acquire_argument_errors(g, ctx):
    with pytest.raises(g.GcError):
        g.gc_acq_create(ctx, 2, 33, 0.0, 0.0, 1.0, 1, [1], 1, 1)          # R too large
    with pytest.raises(g.GcError):
        g.gc_acq_create(ctx, 2, 4, 0.0, 0.0, 1.0, 1, [0], 1, 1)           # PRN 0
    with pytest.raises(g.GcError):
        g.gc_acq_create(ctx, 1, 20, 0.0, 0.0, 1.0, 1, [1], 1000, 1)       # power past uint64
    with pytest.raises(g.GcError):
        g.gc_acq_create(ctx, 2, 4, 0.0, 0.0, 1.0, 0, [1], 1, 1)           # no bins
    a = g.gc_acq_create(ctx, 0, 1, 0.0, 0.0, 1.0, 1, [1], 1, 1)     # int8: zero bytes are 0
    try:
        x = torch.zeros(1024, dtype=torch.uint8, device="cuda")
        res = torch.zeros(g.ACQ_RESULT.itemsize, dtype=torch.uint8, device="cuda")
        assert g.gc_acquire(a, x, 1022, 2.5, None, res) == g.GC_EINVAL    # too few samples
        assert g.gc_acquire(a, x, 1023, 2.5, None, None) == g.GC_EINVAL   # no results
        assert g.gc_acquire(a, x, 1023, 2.5, None, res) == g.GC_OK
        torch.cuda.synchronize()
        r = res.cpu().numpy().view(g.ACQ_RESULT)[0]
        # all-zero input: every power is 0, the peak is bin 0, tau 0, metric inf
        assert (int(r["peak"]), int(r["tau"]), int(r["second"])) == (0, 0, 0)
        assert float(r["metric"]) == float("inf")
    finally:
        g.gc_acq_destroy(a)
