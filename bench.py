"""Benchmark: correlation throughput of libgnsscorr on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Default workload ("twelve"): 12 channels, 2-bit real samples at fs = 16.368
MHz, IF = 4.092 MHz, 10 s of data, 12 PRNs with seeded Doppler / code phase /
C/N0, 1 ms dumps, early/prompt/late at +-1/2 chip.  One step = one
correlation of the whole block for all channels (all hot-path stages),
starting from the same initial channel state, inputs already resident in
HBM.  Other workloads: "single" (1 channel, int8 real at 4.092 MHz, 1 s) and
"multicorrelator" (256 channels x 128 taps at 1/32 chip, complex int8 at
20.46 MHz, 2 s).

Prints ONE JSON line.  ``value`` is G sample*taps/s (one sample correlated
against one tap, I and Q counted together).  ``roofline`` prices the main
kernel's algorithmic work against the VALU peak (256 CUs * 64 lanes *
2.4 GHz): 6 32-bit lane-ops per sample per channel for E/P/L (carrier NCO
add, table lookup, two multiplies, two adds), 14 for the first stage of the
multi-tap form; the kernel duration comes from HIP events the library
records around that kernel on the launch stream.  ``cpu_baseline`` is the
CPU oracle on a bounded sample of the same stream; ``plain`` is one plan and
one direct-kernel launch per channel on the same GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "G sample·taps/s E/P/L correlation vs plain; real-time channels; served p99 latency"
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12     # 32-bit lane-ops/s, T
INT8_MFMA_PEAK_TOPS = 5000.0                 # dense int8 MFMA, T ops/s (2 ops per MAC)
OPS_PER_SAMPLE_CHANNEL = 6
HBM_PEAK_GBS = 8000.0
KERNEL_SETS = {"auto": None, "binned": 2, "direct": 0}
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_pbin_i2_12ch_10s_counters.md")


def realtime_channels(channels: int, data_seconds: float, wall_seconds: float) -> float:
    """Channels that could run in real time: sum(channels x data time) / wall time
    (the definition behind the paper's Table 5, 1 ms / time per epoch per channel)."""
    return channels * data_seconds / wall_seconds


# ---------------------------------------------------------------- workloads
WORKLOADS = {
    "twelve": dict(
        describe="12 channels, 2-bit real, fs 16.368 MHz, IF 4.092 MHz, %g s, 1 ms dumps, "
                 "E/P/L at +-1/2 chip", seconds=10.0, ops=6, fmt_name="i2_real",
        cpu_seconds=10.0),
    "single": dict(
        describe="1 channel (PRN 7), int8 real, fs 4.092 MHz, IF 1.023 MHz, %g s, 1 ms dumps, "
                 "E/P/L at +-1/2 chip", seconds=1.0, ops=6, fmt_name="i8_real",
        cpu_seconds=1.0),
    "multicorrelator": dict(
        describe="256 channels x 128 taps (-2 + k/32 chips), complex int8, fs 20.46 MHz, IF 0, "
                 "%g s, 1 ms dumps", seconds=2.0, ops=14, fmt_name="i8_iq",
        cpu_seconds=0.05),
}


def build_inputs(workload: str, seconds: float):
    from paper_1907_00463_amd import gnsscorr as g
    from paper_1907_00463_amd import synth

    make = {"twelve": synth.workload_twelve_channels, "single": synth.workload_single_channel,
            "multicorrelator": synth.workload_multicorrelator}[workload]
    st, chans, rng = make(seconds=seconds)
    buf = synth.synth_samples(st, rng)
    cfgs = np.zeros(len(chans), g.CHAN_CFG)
    states = np.zeros(len(chans), g.CHAN_STATE)
    for i, ch in enumerate(chans):
        cfgs[i] = g.make_cfg(ch.prn, synth.taps_to_q32(ch.taps_chips), ch.int_periods)
        states[i] = g.gc_nco_init(st.fs, ch.carr_hz, ch.carr_phase0, ch.code_rate,
                                  ch.code_phase0, ch.int_periods)
    return st, chans, buf, cfgs, states


def cpu_baseline(st, buf, cfgs, states, seconds: float = 10.0):
    """The oracle as it stands, host threads over channels, on the first
    `seconds` of the same stream."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    bytes_per = {0: 1.0, 1: 2.0, 2: 0.25}[st.fmt]
    n = int(round(seconds * st.fs))
    n -= n % 4
    n = min(n, st.n)
    sub = buf[: int(np.ceil(n * bytes_per))]
    threads = min(len(cfgs), os.cpu_count() or 1)

    def one(i):
        s = states[i]
        os_ = oracle.OracleState(int(s["carr_phase"]), int(s["carr_step"]), int(s["code_phase"]),
                                 int(s["code_step"]), int(cfgs[i]["n_taps"]))
        K = int(cfgs[i]["n_taps"])
        return oracle.correlate_lut(st.fmt, sub, n, int(cfgs[i]["prn"]), cfgs[i]["tap_q32"][:K],
                                    int(cfgs[i]["int_periods"]), os_)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(one, range(len(cfgs))))
    dt = time.perf_counter() - t0
    taps = int(cfgs["n_taps"].sum())
    return {"value": n * taps / dt / 1e9, "unit": "G sample·taps/s", "cores": threads,
            "kind": "oracle",
            "sample": "first %.3f s (%d samples) of the same stream, all %d channels, "
                      "%d threads over channels; %.2f s wall; real-time channels %.1f"
                      % (n / st.fs, n, len(cfgs), threads, dt,
                         realtime_channels(len(cfgs), n / st.fs, dt))}


def kernel_source_tag(name: str = "gc_pbin.hip") -> str:
    import hashlib
    src = os.path.join(ROOT, "paper_1907_00463_amd", "csrc", name)
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def recorded_traffic():
    """HBM bytes per launch of the periodic kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a copy of known size), or
    None when the kernel source has changed since those counters were taken."""
    try:
        with open(TRAFFIC_PROFILE) as f:
            text = f.read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_source_sha256_16") != kernel_source_tag():
        return None
    try:
        return int(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_steps(torch, step, steps, warmup):
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def plain_baseline(torch, g, ctx, st, cfgs, states, samples, n, max_dumps, stream, steps, warmup):
    """Plain per-channel launches: one plan and one launch per channel, each
    with the direct per-sample kernel, on the same stream and inputs."""
    plans, bufs = [], []
    for i in range(len(cfgs)):
        p = g.Plan(ctx, st.fmt, g.GC_CARRIER_LUT, cfgs[i: i + 1])
        g.gc_plan_set_kernels(p.handle, 0)
        s0 = p.states_to_device(states[i: i + 1])
        plans.append(p)
        bufs.append((s0, s0.clone()) + p.outputs(max_dumps))

    def step():
        for p, (s0, s, out, dn, nd, stt) in zip(plans, bufs):
            s.copy_(s0)
            p.correlate(samples, n, s, out, dn, nd, stt, stream=stream)

    dt = time_steps(torch, step, steps, warmup)
    for p in plans:
        p.close()
    return dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=list(WORKLOADS), default="twelve")
    ap.add_argument("--seconds", type=float, default=None, help="data per step")
    ap.add_argument("--kernels", choices=list(KERNEL_SETS), default="auto",
                    help="kernel families the plan may use (auto: all)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the per-channel launch baseline")
    ap.add_argument("--cpu-seconds", type=float, default=None)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before timing, copy a buffer of this many MiB once (a kernel of known "
                         "traffic that scales the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the correlator shards by receiver or channel "
              "with no exchange, and no multi-GPU figure is produced here (--gpus 1).",
              file=sys.stderr)
        sys.exit(2)
    wl = WORKLOADS[args.workload]
    seconds = args.seconds if args.seconds is not None else wl["seconds"]
    cpu_seconds = args.cpu_seconds if args.cpu_seconds is not None else wl["cpu_seconds"]

    import torch

    from paper_1907_00463_amd import gnsscorr as g

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    print("bench: generating %.3f s of the %s workload" % (seconds, args.workload),
          file=sys.stderr, flush=True)
    st, chans, buf, cfgs, states = build_inputs(args.workload, seconds)
    n = st.n
    ctx = g.gc_create(0)
    plan = g.Plan(ctx, st.fmt, g.GC_CARRIER_LUT, cfgs)
    if KERNEL_SETS[args.kernels] is not None:
        g.gc_plan_set_kernels(plan.handle, KERNEL_SETS[args.kernels])
    samples = torch.from_numpy(buf).to(dev)
    state0 = plan.states_to_device(states)
    state = state0.clone()
    max_dumps = g.max_dumps_for(n, int(states["code_step"].max()),
                                int(cfgs["int_periods"].min()))
    out, dump_n, n_dumps, status = plan.outputs(max_dumps)
    stream = torch.cuda.current_stream(dev)

    def step():
        state.copy_(state0)
        plan.correlate(samples, n, state, out, dump_n, n_dumps, status, stream=stream)

    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    print("bench: warmup %d" % args.warmup, file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    g.gc_plan_timing(plan.handle, args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [g.gc_plan_kernel_ms(plan.handle, i) for i in range(args.steps)]
    g.gc_plan_timing(plan.handle, 0)
    assert int(status.abs().sum()) == 0, "channel refused"
    nd = n_dumps.cpu().numpy()
    print("bench: timed %d steps, %.3f ms/step, kernel %.3f ms" % (
        args.steps, 1e3 * wall / args.steps, float(np.mean(kern_ms))), file=sys.stderr, flush=True)

    ms_step = 1e3 * wall / args.steps
    taps = int(cfgs["n_taps"].sum())
    sample_taps = n * taps
    value = sample_taps / (wall / args.steps) / 1e9
    k_s = float(np.mean(kern_ms)) / 1e3
    achieved = wl["ops"] * n * len(cfgs) / k_s / 1e12
    taps_per = sorted(set(int(t) for t in cfgs["n_taps"]))
    res = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "G sample·taps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": wl["describe"] % seconds,
                   "channels": len(cfgs),
                   "taps_per_channel": taps_per[0] if len(taps_per) == 1 else taps_per,
                   "samples": n, "format": wl["fmt_name"], "kernels": args.kernels,
                   "dumps_per_channel": int(nd.max()),
                   "realtime_channels": round(realtime_channels(len(cfgs), n / st.fs,
                                                                wall / args.steps), 1)},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                     "peak": round(VALU_PEAK_TOPS, 2), "unit": "T lane-ops/s",
                     "frac": round(achieved / VALU_PEAK_TOPS, 4),
                     "traffic": recorded_traffic()
                     if (args.kernels == "auto" and args.workload == "twelve") else None,
                     "kernel_ms": round(k_s * 1e3, 4),
                     "ops_per_sample_channel": wl["ops"]},
    }
    if args.workload == "multicorrelator" and args.kernels == "auto":
        # stage 2: 128 rows (I/Q x lo/hi x 32 cells) x 16 shifts per chip
        chips = n * float(np.mean(states["code_step"].astype(np.float64))) / 2 ** 32
        macs = 128 * 16 * chips * len(cfgs)
        tops = 2 * macs / k_s / 1e12
        res["roofline_stage2"] = {"bound": "mfma", "achieved": round(tops, 3),
                                  "peak": INT8_MFMA_PEAK_TOPS, "unit": "T int8 ops/s",
                                  "frac": round(tops / INT8_MFMA_PEAK_TOPS, 5),
                                  "macs": round(macs),
                                  "note": "int8 MFMA work over the whole kernel time "
                                          "(stage 1 dominates)"}
    if not args.no_plain:
        print("bench: plain per-channel launches", file=sys.stderr, flush=True)
        psteps = 1 if args.workload == "multicorrelator" else max(1, min(args.steps, 5))
        dt = plain_baseline(torch, g, ctx, st, cfgs, states, samples, n, max_dumps, stream,
                            psteps, 1)
        res["plain"] = {"value": round(sample_taps / dt / 1e9, 3), "unit": "G sample·taps/s",
                        "ms_per_step": round(dt * 1e3, 4),
                        "kind": "one plan and one direct-kernel launch per channel",
                        "speedup": round(dt / (wall / args.steps), 2)}
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(st, buf, cfgs, states, cpu_seconds)
    plan.close()
    g.gc_destroy(ctx)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
