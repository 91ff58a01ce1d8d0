"""GPU parity of batches (many receivers, one persistent graph-captured
launch) against the CPU oracle, through the C ABI: every channel of every
receiver bit-exact in dumps, sample counts and final NCO state; graph
replays, every block shape and the autotuner give the same results."""
import numpy as np
import pytest

from gpu_util import block_bytes, oracle_state, run_oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

EPL = [1 << 31, 0, -(1 << 31)]


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


def _receivers(g, seed, n_rx=6):
    rng = np.random.default_rng(seed)
    rates = [4.092e6, 8.184e6, 16.368e6]
    rx, cfgs, states, chan_rx = [], [], [], []
    for r in range(n_rx):
        fs = rates[r % 3]
        fmt = (0, 2, 1, 3)[(r + r // 4) % 4]   # real int8, 2-bit, complex int8, complex 2-bit
        n = int(rng.integers(50_000, 400_000))
        buf = rng.integers(0, 256, size=block_bytes(fmt, n), dtype=np.uint8)
        rx.append((fmt, n, buf))
        for c in range(int(rng.integers(1, 5))):
            T = int(rng.choice([1, 4, 20]))
            taps = EPL if (r, c) != (1, 1) else [0, 1 << 30]  # one 2-tap channel
            cfgs.append(g.make_cfg(int(rng.integers(1, 33)), taps, T))
            fd = float(rng.uniform(-5000, 5000))
            states.append(g.gc_nco_init(fs, fs / 4 + fd, float(rng.random()),
                                        1.023e6 * (1 + fd / 1575.42e6),
                                        float(rng.uniform(0, 1023 * T)), T))
            chan_rx.append(r)
    return rx, np.array(cfgs, g.CHAN_CFG), np.array(states, g.CHAN_STATE), np.array(chan_rx)


def _make_batch(g, ctx, rx, cfgs, states, chan_rx):
    blocks = [torch.from_numpy(b).to("cuda") for (_, _, b) in rx]
    max_dumps = max(g.max_dumps_for(n, int(states["code_step"].max()), 1) for (_, n, _) in rx)
    return g.Batch(ctx, blocks, [f for (f, _, _) in rx], [n for (_, n, _) in rx], cfgs, chan_rx,
                   states, max_dumps)


def _oracle_all(rx, cfgs, states, chan_rx):
    res = []
    for i in range(len(cfgs)):
        fmt, n, buf = rx[int(chan_rx[i])]
        r, s = run_oracle(fmt, cfgs[i: i + 1], states[i: i + 1], [buf], [n])
        res.append((r[0][0][0], r[0][1][0], s[0]))
    return res


def _check(batch, cfgs, expect):
    torch.cuda.synchronize()
    out = batch.out.cpu().numpy()
    dump_n = batch.dump_n.cpu().numpy().astype(np.uint32)
    n_dumps = batch.n_dumps.cpu().numpy()
    status = batch.status.cpu().numpy()
    st = batch.states()
    assert np.all(status == 0), status
    for i, (dumps, dns, s) in enumerate(expect):
        K = int(cfgs[i]["n_taps"])
        nd = int(n_dumps[i])
        assert nd == len(dumps), (i, nd, len(dumps))
        assert np.array_equal(out[i, :nd, :K].astype(np.int64), dumps), i
        assert np.array_equal(dump_n[i, :nd], dns), i
        assert int(st[i]["code_phase"]) == s.code_phase, i
        assert int(st[i]["carr_phase"]) == s.carr_phase, i
        assert int(st[i]["acc_n"]) == s.acc_n, i
        assert np.array_equal(st[i]["acc"][:K].reshape(-1).astype(np.int64), s.acc), i


def test_batch_bit_exact_mixed_receivers(g, ctx):
    rx, cfgs, states, chan_rx = _receivers(g, 901)
    b = _make_batch(g, ctx, rx, cfgs, states, chan_rx)
    try:
        b.launch()
        _check(b, cfgs, _oracle_all(rx, cfgs, states, chan_rx))
    finally:
        b.close()


def test_batch_graph_replays_match_eager_restores(g, ctx):
    # the captured graph replayed three times, the channel states restored
    # by eager copies between the replays; every replay checked
    rx, cfgs, states, chan_rx = _receivers(g, 902, n_rx=4)
    expect = _oracle_all(rx, cfgs, states, chan_rx)
    b = _make_batch(g, ctx, rx, cfgs, states, chan_rx)
    try:
        s0 = b.state.clone()
        for _ in range(3):
            b.state.copy_(s0)
            b.out.fill_(7)                       # stale values must be overwritten
            b.launch()
            _check(b, cfgs, expect)
    finally:
        b.close()


def test_batch_every_shape_and_the_tuner(g, ctx):
    rx, cfgs, states, chan_rx = _receivers(g, 903, n_rx=5)
    expect = _oracle_all(rx, cfgs, states, chan_rx)
    b = _make_batch(g, ctx, rx, cfgs, states, chan_rx)
    try:
        s0 = b.state.clone()
        for shape in range(b.info()["n_shapes"]):
            for grid, chunk in ((0, 0), (7, -1), (0, 2), (7, 8)):
                b.configure(shape, grid, chunk)
                b.state.copy_(s0)
                b.launch()
                _check(b, cfgs, expect)
        b.state.copy_(s0)
        torch.cuda.synchronize()
        b.tune(reps=1)
        info = b.info()
        assert info["tuned_ms"] > 0 and 0 <= info["shape"] < info["n_shapes"]
        # tuning leaves the bound states as they were
        assert torch.equal(b.state, s0)
        b.launch()
        _check(b, cfgs, expect)
    finally:
        b.close()


def test_batch_equals_plans(g, ctx):
    # the same receivers through one plan per receiver
    from gpu_util import run_library
    rx, cfgs, states, chan_rx = _receivers(g, 904, n_rx=3)
    b = _make_batch(g, ctx, rx, cfgs, states, chan_rx)
    try:
        b.launch()
        torch.cuda.synchronize()
        out = b.out.cpu().numpy()
        for r, (fmt, n, buf) in enumerate(rx):
            idx = np.nonzero(chan_rx == r)[0]
            lib, _ = run_library(torch, ctx, fmt, g.GC_CARRIER_LUT, cfgs[idx], states[idx],
                                 [buf], [n], max_dumps=b.max_dumps)
            o = lib[0][0]
            for j, i in enumerate(idx):
                K = int(cfgs[i]["n_taps"])
                nd = int(lib[0][2][j])
                assert np.array_equal(out[i, :nd, :K], o[j, :nd, :K]), i
    finally:
        b.close()


def test_batch_wide_receivers_share_waves(g, ctx):
    # receivers of 9, 11, 12, 14, 16 and 17 channels: groups below three
    # quarters of a block's 16 waves share their channels' bins over all 16
    # (two channel pieces for some waves), fuller groups run one wave per
    # channel; the 17-channel receiver spans two groups; items come from the
    # device queue in size order.  Every channel bit-exact against the oracle.
    rng = np.random.default_rng(905)
    rates = [16.368e6, 8.184e6, 4.092e6, 16.368e6, 8.184e6, 16.368e6]
    counts = [9, 11, 12, 14, 16, 17]
    rx, cfgs, states, chan_rx = [], [], [], []
    for r, (fs, nc) in enumerate(zip(rates, counts)):
        fmt = (2, 0)[r % 2]
        n = int(rng.integers(120_000, 260_000))
        rx.append((fmt, n, rng.integers(0, 256, size=block_bytes(fmt, n), dtype=np.uint8)))
        for c in range(nc):
            T = int(rng.choice([1, 4, 20]))
            cfgs.append(g.make_cfg(int(rng.integers(1, 33)), EPL, T))
            fd = float(rng.uniform(-5000, 5000))
            states.append(g.gc_nco_init(fs, fs / 4 + fd, float(rng.random()),
                                        1.023e6 * (1 + fd / 1575.42e6),
                                        float(rng.uniform(0, 1023 * T)), T))
            chan_rx.append(r)
    cfgs = np.array(cfgs, g.CHAN_CFG)
    states = np.array(states, g.CHAN_STATE)
    chan_rx = np.array(chan_rx)
    b = _make_batch(g, ctx, rx, cfgs, states, chan_rx)
    try:
        b.launch()
        _check(b, cfgs, _oracle_all(rx, cfgs, states, chan_rx))
    finally:
        b.close()


def test_batch_full_workload_sampled(g, ctx):
    # The 64-receiver batched workload at full size (708 channels, 1 s per
    # receiver at 4.092/8.184/16.368 MHz, int8 and 2-bit, 1/4/20-period dumps)
    # in the launch configuration the benchmark times: one batch, tuned, the
    # graph launched once.  The receivers' channels and NCO words are the
    # workload's; the sample bytes are uniform random (bit-exactness does not
    # depend on the signal, and this keeps the test fast).  Checked against
    # the oracle: one channel of every (rate, format, period) class, the first
    # and last channel of the widest receiver, and the receivers' last
    # channels, which close the work queue's items.
    from paper_1907_00463_amd import synth
    work = synth.workload_batched(seconds=1.0)
    rng = np.random.default_rng(1303)
    rx, cfgs, states, chan_rx = [], [], [], []
    for r, (st, chans, _) in enumerate(work):
        rx.append((st.fmt, st.n, rng.integers(0, 256, size=block_bytes(st.fmt, st.n),
                                              dtype=np.uint8)))
        for ch in chans:
            cfgs.append(g.make_cfg(ch.prn, synth.taps_to_q32(ch.taps_chips), ch.int_periods))
            states.append(g.gc_nco_init(st.fs, ch.carr_hz, ch.carr_phase0, ch.code_rate,
                                        ch.code_phase0, ch.int_periods))
            chan_rx.append(r)
    cfgs = np.array(cfgs, g.CHAN_CFG)
    states = np.array(states, g.CHAN_STATE)
    chan_rx = np.array(chan_rx)
    assert len(work) == 64 and len(cfgs) == 708
    pick = {}
    for i in range(len(cfgs)):
        st = work[int(chan_rx[i])][0]
        pick.setdefault((st.fs, st.fmt, int(cfgs[i]["int_periods"])), i)
    assert len(pick) == 18
    sel = set(pick.values())
    widest = max(range(64), key=lambda r: int(np.sum(chan_rx == r)))
    idx = np.nonzero(chan_rx == widest)[0]
    sel |= {int(idx[0]), int(idx[-1])}
    for r in range(0, 64, 9):
        sel.add(int(np.nonzero(chan_rx == r)[0][-1]))
    sel = sorted(sel)
    b = _make_batch(g, ctx, rx, cfgs, states, chan_rx)
    try:
        s0 = b.state.clone()
        b.tune(reps=1)
        assert torch.equal(b.state, s0)
        b.launch()
        torch.cuda.synchronize()
        out = b.out.cpu().numpy()
        dump_n = b.dump_n.cpu().numpy().astype(np.uint32)
        n_dumps = b.n_dumps.cpu().numpy()
        status = b.status.cpu().numpy()
        st_fin = b.states()
        assert np.all(status == 0)
        for i in sel:
            fmt, n, buf = rx[int(chan_rx[i])]
            r, s = run_oracle(fmt, cfgs[i: i + 1], states[i: i + 1], [buf], [n])
            dumps, dns, so = r[0][0][0], r[0][1][0], s[0]
            nd = int(n_dumps[i])
            assert nd == len(dumps), (i, nd, len(dumps))
            assert np.array_equal(out[i, :nd, :3].astype(np.int64), dumps), i
            assert np.array_equal(dump_n[i, :nd], dns), i
            assert int(st_fin[i]["code_phase"]) == so.code_phase, i
            assert int(st_fin[i]["carr_phase"]) == so.carr_phase, i
            assert int(st_fin[i]["acc_n"]) == so.acc_n, i
            assert np.array_equal(st_fin[i]["acc"][:3].reshape(-1).astype(np.int64), so.acc), i
        # every channel: dump counts and sample counts follow from the NCO words alone
        for i in range(len(cfgs)):
            n = rx[int(chan_rx[i])][1]
            W = int(cfgs[i]["int_periods"]) * 1023 << 32
            u_end = int(states[i]["code_phase"]) + n * int(states[i]["code_step"])
            assert int(n_dumps[i]) == u_end // W, i
            nd = int(n_dumps[i])
            assert int(dump_n[i, :nd].astype(np.int64).sum()) + int(st_fin[i]["acc_n"]) == n, i
    finally:
        b.close()


def test_batch_many_receivers_item_selection(g, ctx):
    # 300 receivers (more than one pass of the set-up's item selection over
    # receivers), some with no channel at all, complex ones (their channels
    # take the chip-by-chip kernel, so their tiles must be selected) spread
    # over every pass, real ones at periodic rates (periodic kernel only):
    # every channel bit-exact against the oracle, with the periodic kernel on
    # (selection) and off (every item).
    rng = np.random.default_rng(907)
    rates = [4.092e6, 8.184e6, 16.368e6]
    rx, cfgs, states, chan_rx = [], [], [], []
    for r in range(300):
        fs = rates[r % 3]
        fmt = 1 if r % 37 == 5 else (3 if r % 53 == 7 else (0, 2)[r % 2])
        n = int(rng.integers(2_000, 9_000))
        rx.append((fmt, n, rng.integers(0, 256, size=block_bytes(fmt, n), dtype=np.uint8)))
        if r % 11 == 3:
            continue   # a receiver with no channel
        for c in range(int(rng.integers(1, 3))):
            T = int(rng.choice([1, 4]))
            cfgs.append(g.make_cfg(int(rng.integers(1, 33)), EPL, T))
            fd = float(rng.uniform(-5000, 5000))
            states.append(g.gc_nco_init(fs, fs / 4 + fd, float(rng.random()),
                                        1.023e6 * (1 + fd / 1575.42e6),
                                        float(rng.uniform(0, 1023 * T)), T))
            chan_rx.append(r)
    cfgs = np.array(cfgs, g.CHAN_CFG)
    states = np.array(states, g.CHAN_STATE)
    chan_rx = np.array(chan_rx)
    assert len(set(chan_rx.tolist())) < 300 and max(chan_rx) > 256
    expect = _oracle_all(rx, cfgs, states, chan_rx)
    b = _make_batch(g, ctx, rx, cfgs, states, chan_rx)
    try:
        s0 = b.state.clone()
        for grid, chunk in ((0, 0), (0, -1), (5, 2)):
            b.configure(0, grid, chunk)
            b.state.copy_(s0)
            b.out.fill_(7)
            b.launch()
            _check(b, cfgs, expect)
    finally:
        b.close()
