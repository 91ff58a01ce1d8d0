"""GPU parity of the dense multi-tap path (taps on the 1/32-chip grid, int8
MFMA form) against the CPU oracle, through the C ABI: bit-exact int32 dumps,
sample counts and final NCO state."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from gpu_util import TWO32, assert_exact, block_bytes, c10_check, run_library, run_oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TAPS_128 = np.array([(k - 64) << 27 for k in range(128)], np.int64)  # -2 + k/32 chips


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


def _channels(g, rng, fs, n_chan, taps, periods=(1, 4, 1, 20), rates=None):
    cfgs = np.zeros(n_chan, g.CHAN_CFG)
    states = np.zeros(n_chan, g.CHAN_STATE)
    for i in range(n_chan):
        T = periods[i % len(periods)]
        cfgs[i] = g.make_cfg(int(rng.integers(1, 33)), taps, T)
        fd = float(rng.uniform(-5000, 5000))
        rate = 1.023e6 * (1 + fd / 1575.42e6) if rates is None else rates[i % len(rates)]
        states[i] = g.gc_nco_init(fs, float(rng.uniform(-0.3, 0.3)) * fs, float(rng.random()), rate,
                                  float(rng.uniform(0, 1023 * T)), T)
    return cfgs, states


def _blocks(rng, fmt, lens):
    return [rng.integers(0, 256, size=block_bytes(fmt, n), dtype=np.uint8) for n in lens]


@pytest.mark.parametrize("fmt", [1, 0, 2, 3])
def test_128_taps_bit_exact(g, ctx, fmt):
    # 128 taps at -2 + k/32 chips, 20.46 MHz, dumps of 1/4/20 periods, blocks
    # that split chunks and dumps anywhere
    rng = np.random.default_rng(700 + fmt)
    cfgs, states = _channels(g, rng, 20.46e6, 4, TAPS_128)
    lens = [61_000, 7040 * 3 + 12, 4 * 997]
    blocks = _blocks(rng, fmt, lens)
    lib, lst = run_library(torch, ctx, fmt, g.GC_CARRIER_LUT, cfgs, states, blocks, lens)
    orc, ost = run_oracle(fmt, cfgs, states, blocks, lens)
    assert_exact(lib, lst, orc, ost, cfgs)


def test_mfma_path_equals_direct_path(g, ctx):
    # the same plan with the MFMA family switched off runs the direct kernel
    rng = np.random.default_rng(711)
    cfgs, states = _channels(g, rng, 20.46e6, 3, TAPS_128)
    lens = [40_000]
    blocks = _blocks(rng, 1, lens)
    a, sa = run_library(torch, ctx, 1, g.GC_CARRIER_LUT, cfgs, states, blocks, lens)
    b, sb = run_library(torch, ctx, 1, g.GC_CARRIER_LUT, cfgs, states, blocks, lens, kernels=0)
    assert np.array_equal(a[0][0], b[0][0])
    assert np.array_equal(a[0][1], b[0][1])
    assert np.array_equal(sa.view(np.uint8), sb.view(np.uint8))


def test_fp32_carrier_128_taps_within_tolerance(g, ctx):
    # the FP32-carrier variant of the multi-correlator (complex int8, 128
    # taps at 1/32 chip) against the FP64 oracle, every tap to the |P| bound
    rng = np.random.default_rng(720)
    cfgs, states = _channels(g, rng, 20.46e6, 3, TAPS_128, periods=(1, 4, 1))
    states["code_phase"] %= np.uint64(1023 * TWO32)
    lens = [44_000, 20_460]
    blocks = _blocks(rng, 1, lens)
    lib, lst = run_library(torch, ctx, 1, g.GC_CARRIER_F32, cfgs, states, blocks, lens)
    orc, ost = run_oracle(1, cfgs, states, blocks, lens, f64=True)
    worst = 0.0
    for (out, dump_n, n_dumps, status), (dumps, dns) in zip(lib, orc):
        assert np.all(status == 0)
        for i in range(len(cfgs)):
            nd = int(n_dumps[i])
            assert nd == len(dumps[i])
            assert np.array_equal(dump_n[i, :nd], dns[i])
            if nd == 0:
                continue
            sigma = np.sqrt(dns[i].astype(np.float64) * (2 * 128 ** 2 / 3) / 2)[:, None]
            ok, w = c10_check(out[i, :nd, :128].astype(np.float64), dumps[i], sigma)
            assert ok.all(), w
            worst = max(worst, w)
    for i in range(len(cfgs)):
        assert int(lst[i]["code_phase"]) == ost[i].code_phase
        assert abs(float(lst[i]["carr_phase_f"]) - ost[i].carr_phase_f) < 1e-9
    print("worst relative |P| error", worst)


def test_epl_columns_equal_the_three_tap_correlator(g, ctx):
    # columns 48, 64, 80 of the 128-tap grid are -1/2, 0, +1/2 chip
    rng = np.random.default_rng(712)
    cfgs, states = _channels(g, rng, 20.46e6, 2, TAPS_128, periods=(1,))
    lens = [50_000]
    blocks = _blocks(rng, 1, lens)
    lib, _ = run_library(torch, ctx, 1, g.GC_CARRIER_LUT, cfgs, states, blocks, lens)
    epl = cfgs.copy()
    for i in range(len(epl)):
        epl[i] = g.make_cfg(int(cfgs[i]["prn"]), [1 << 31, 0, -(1 << 31)], 1)
    orc, _ = run_oracle(1, epl, states, blocks, lens)
    out, dump_n, n_dumps, status = lib[0]
    for i in range(len(cfgs)):
        nd = int(n_dumps[i])
        got = out[i, :nd][:, [80, 64, 48], :].astype(np.int64)
        assert np.array_equal(got, orc[0][0][i]), i


def test_mixed_taps_rates_and_fallback(g, ctx):
    # complex E/P/L (3 taps on the grid), an off-grid tap set and a channel
    # with more than 32 samples per chip in one plan: the last two go to the
    # direct kernel, the rest to the MFMA kernel
    rng = np.random.default_rng(713)
    fs = 20.46e6
    tap_sets = [np.array([1 << 31, 0, -(1 << 31)], np.int64),
                np.array([0, 5 << 27, -(3 << 27), 1 << 20], np.int64),
                TAPS_128[::3].copy(),
                TAPS_128[10:90].copy()]
    n = len(tap_sets)
    cfgs = np.zeros(n, g.CHAN_CFG)
    states = np.zeros(n, g.CHAN_STATE)
    for i, t in enumerate(tap_sets):
        cfgs[i] = g.make_cfg(int(rng.integers(1, 33)), t, 1)
        rate = 0.5e6 if i == 2 else 1.023e6 * (1 + float(rng.uniform(-3e-6, 3e-6)))
        states[i] = g.gc_nco_init(fs, 2.1e6, float(rng.random()), rate,
                                  float(rng.uniform(0, 1023)), 1)
    lens = [33_333, 21_000]
    blocks = _blocks(rng, 1, lens)
    lib, lst = run_library(torch, ctx, 1, g.GC_CARRIER_LUT, cfgs, states, blocks, lens)
    orc, ost = run_oracle(1, cfgs, states, blocks, lens)
    assert_exact(lib, lst, orc, ost, cfgs)


def test_more_channels_than_one_block(g, ctx):
    rng = np.random.default_rng(714)
    cfgs, states = _channels(g, rng, 20.46e6, 21, TAPS_128[::2].copy(), periods=(1, 4))
    lens = [25_000]
    blocks = _blocks(rng, 1, lens)
    lib, lst = run_library(torch, ctx, 1, g.GC_CARRIER_LUT, cfgs, states, blocks, lens)
    orc, ost = run_oracle(1, cfgs, states, blocks, lens)
    assert_exact(lib, lst, orc, ost, cfgs)


def test_multicorrelator_workload_sampled_channels(g, ctx):
    # the 256-channel, 128-tap, 2 s complex workload in the benchmark's launch
    # configuration; every dump of 6 channels (spread over the channel groups
    # and the PRN hypotheses) against the oracle
    from paper_1907_00463_amd import synth
    st, chans, rng = synth.workload_multicorrelator()
    buf = synth.synth_samples(st, rng)
    cfgs = np.zeros(len(chans), g.CHAN_CFG)
    states = np.zeros(len(chans), g.CHAN_STATE)
    for i, ch in enumerate(chans):
        cfgs[i] = g.make_cfg(ch.prn, synth.taps_to_q32(ch.taps_chips), ch.int_periods)
        states[i] = g.gc_nco_init(st.fs, ch.carr_hz, ch.carr_phase0, ch.code_rate,
                                  ch.code_phase0, ch.int_periods)
    lib, lst = run_library(torch, ctx, st.fmt, g.GC_CARRIER_LUT, cfgs, states, [buf], [st.n])
    out, dump_n, n_dumps, status = lib[0]
    assert np.all(status == 0)
    assert int(n_dumps.min()) >= 1999
    pick = [0, 37, 100, 131, 200, 255]

    def one(i):
        r, s = run_oracle(st.fmt, cfgs[i: i + 1], states[i: i + 1], [buf], [st.n])
        return i, r[0][0][0], r[0][1][0], s[0]

    with ThreadPoolExecutor(max_workers=len(pick)) as ex:
        for i, dumps, dns, s in ex.map(one, pick):
            nd = int(n_dumps[i])
            assert nd == len(dumps), i
            assert np.array_equal(out[i, :nd].astype(np.int64), dumps), i
            assert np.array_equal(dump_n[i, :nd], dns), i
            assert int(lst[i]["code_phase"]) == s.code_phase
            assert int(lst[i]["acc_n"]) == s.acc_n
            assert np.array_equal(lst[i]["acc"].reshape(-1).astype(np.int64), s.acc)


@pytest.mark.parametrize("rate_scale", [1.0, 1.0 + 2e-6])
def test_32_samples_per_chip_edge(g, ctx, rate_scale):
    # code step exactly 2^27 (32 samples per chip: every cell row of a chip
    # written, 1,024-sample windows) and just above it, complex int8 at
    # 32.736 MHz; 128 taps, dumps of 1 and 4 periods
    rng = np.random.default_rng(730)
    fs = 32.736e6
    rates = (1.023e6 * rate_scale,)
    cfgs, states = _channels(g, rng, fs, 3, TAPS_128, periods=(1, 4, 1), rates=rates)
    assert int(states["code_step"].min()) >= 1 << 27
    lens = [70_000, 33_000]
    blocks = _blocks(rng, 1, lens)
    lib, lst = run_library(torch, ctx, 1, g.GC_CARRIER_LUT, cfgs, states, blocks, lens)
    orc, ost = run_oracle(1, cfgs, states, blocks, lens)
    assert_exact(lib, lst, orc, ost, cfgs)


@pytest.mark.parametrize("fs, rate_scale", [
    (10.7415e6, 1.0 + 2e-6),     # 10.5 samples per chip: whole samples per two chips
    (20.46e6, 1.0 + 3.05e-5),    # drift per two chips just below the direct form's bound
    (20.46e6, 1.0 + 3.10e-5),    # just above it: every window by the scatter
    (16.368e6, 1.0 - 1.5e-5),    # frequent row crossings, negative drift
])
@pytest.mark.parametrize("fmt", [1, 3])
def test_direct_cells_rates_bit_exact(g, ctx, fs, rate_scale, fmt):
    # Rates that exercise the multi-tap kernel's direct-cell form and its
    # fallback: half-integer samples per chip, drifts near the bound on
    # |D2 dp - 2^33| (many row crossings, windows switching between the two
    # forms), both signs of the drift; 128 taps, dumps of 1/4/1/20 periods,
    # blocks that cut windows and dumps anywhere.
    rng = np.random.default_rng(740 + fmt)
    cfgs, states = _channels(g, rng, fs, 4, TAPS_128, rates=(1.023e6 * rate_scale,))
    lens = [90_000, 7040 * 3 + 12, 33_001]
    blocks = _blocks(rng, fmt, lens)
    lib, lst = run_library(torch, ctx, fmt, g.GC_CARRIER_LUT, cfgs, states, blocks, lens)
    orc, ost = run_oracle(fmt, cfgs, states, blocks, lens)
    assert_exact(lib, lst, orc, ost, cfgs)
