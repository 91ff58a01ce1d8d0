"""Helpers for the GPU parity tests: run the library and the oracle on the
same blocks and compare what they return."""
from __future__ import annotations

import numpy as np

import oracle

TWO32 = 1 << 32


def block_bytes(fmt: int, n: int) -> int:
    return {0: n, 1: 2 * n, 2: (n + 3) // 4, 3: (n + 1) // 2}[fmt]


def oracle_state(st_rec, K: int, f64: bool = False) -> oracle.OracleState:
    s = oracle.OracleState(int(st_rec["carr_phase"]), int(st_rec["carr_step"]),
                           int(st_rec["code_phase"]), int(st_rec["code_step"]), K,
                           carr_phase_f=float(st_rec["carr_phase_f"]),
                           carr_freq_f=float(st_rec["carr_freq_f"]))
    s.acc_n = int(st_rec["acc_n"])
    if f64:
        s.acc = st_rec["acc_f"][:K].reshape(-1).astype(np.float64)
    else:
        s.acc = st_rec["acc"][:K].reshape(-1).astype(np.int64)
    return s


def run_library(torch, ctx, fmt, carrier, cfgs, states, blocks, ns, max_dumps=None, stream=None,
                kernels=None):
    """Run consecutive blocks through one plan; returns per-block host results
    [(out, dump_n, n_dumps, status)] and the final host states.  ``kernels``:
    GC_KERNEL_* mask for the plan (None: the library default)."""
    from paper_1907_00463_amd import gnsscorr as g

    plan = g.Plan(ctx, fmt, carrier, cfgs)
    try:
        if kernels is not None:
            g.gc_plan_set_kernels(plan.handle, kernels)
        st_dev = plan.states_to_device(states)
        res = []
        for buf, n in zip(blocks, ns):
            md = max_dumps or g.max_dumps_for(n, int(states["code_step"].max()),
                                              int(cfgs["int_periods"].min()))
            out, dump_n, n_dumps, status = plan.outputs(md)
            sbuf = torch.from_numpy(np.ascontiguousarray(buf)).to("cuda") if len(buf) else \
                torch.zeros(1, dtype=torch.uint8, device="cuda")
            plan.correlate(sbuf, n, st_dev, out, dump_n, n_dumps, status, stream=stream)
            torch.cuda.synchronize()
            res.append((out.cpu().numpy(), dump_n.cpu().numpy().astype(np.uint32),
                        n_dumps.cpu().numpy(), status.cpu().numpy()))
        return res, plan.states_from_device(st_dev)
    finally:
        plan.close()


def run_oracle(fmt, cfgs, states, blocks, ns, f64=False):
    """Same blocks through the oracle; returns per-block [(list of dumps, list of dump_n)]
    and the oracle states."""
    sts = [oracle_state(states[i], int(cfgs[i]["n_taps"]), f64) for i in range(len(cfgs))]
    res = []
    for buf, n in zip(blocks, ns):
        dumps, dns = [], []
        for i, c in enumerate(cfgs):
            K = int(c["n_taps"])
            taps = c["tap_q32"][:K]
            if f64:
                d, dn = oracle.correlate_f64(fmt, buf, n, int(c["prn"]), taps, int(c["int_periods"]), sts[i])
            else:
                d, dn = oracle.correlate_lut(fmt, buf, n, int(c["prn"]), taps, int(c["int_periods"]), sts[i])
            dumps.append(d)
            dns.append(dn)
        res.append((dumps, dns))
    return res, sts


def assert_exact(lib_res, lib_states, orc_res, orc_states, cfgs):
    for (out, dump_n, n_dumps, status), (dumps, dns) in zip(lib_res, orc_res):
        assert np.all(status == 0), status
        for i, c in enumerate(cfgs):
            K = int(c["n_taps"])
            nd = int(n_dumps[i])
            assert nd == len(dumps[i]), (i, nd, len(dumps[i]))
            assert np.array_equal(out[i, :nd, :K, :].astype(np.int64), dumps[i]), i
            assert np.array_equal(dump_n[i, :nd], dns[i]), i
    for i, c in enumerate(cfgs):
        K = int(c["n_taps"])
        s, o = lib_states[i], orc_states[i]
        assert int(s["carr_phase"]) == o.carr_phase
        assert int(s["code_phase"]) == o.code_phase
        assert int(s["acc_n"]) == o.acc_n
        assert np.array_equal(s["acc"][:K].reshape(-1).astype(np.int64), o.acc)


def c10_check(p_lib, p_ref, sigma):
    """FP32 variant tolerance on |P| per dump: ||P| - |P_ref|| <= 1e-5 * max(|P_ref|, 3 sigma)."""
    a = np.abs(p_lib[..., 0] + 1j * p_lib[..., 1])
    b = np.abs(p_ref[..., 0] + 1j * p_ref[..., 1])
    tol = 1e-5 * np.maximum(b, 3.0 * sigma)
    return np.abs(a - b) <= tol, np.max(np.abs(a - b) / np.maximum(b, 3.0 * sigma))
