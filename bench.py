"""Benchmark: 30-qubit complex128 random circuit, fused + LDS-blocked vs gate-by-gate.

Workload: 30 qubits (16 GiB complex128 state), depth 40; every layer is U3
(angles U[0, 2pi)) on all qubits then CZ on a random perfect matching
(1,800 gates, seed 30002).  One timed step = |0...0> initialisation, the
whole fused/blocked plan (kmax = 5), and a Pauli-expectation readout, all
on the GPU through the C ABI.  The plan is built once beforehand (its host
time is reported as plan_seconds, like the paper's separate optimiser time).

Printed: one JSON line with gate-applications/s, the dominant kernel's
roofline figures (per-launch device time from events around every launch),
the gate-by-gate path's throughput on the same circuit, and the CPU oracle
timed on a bounded sample of the same workload.
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

HBM_PEAK_GBS = 8000.0        # MI355X published HBM3E bandwidth
FP64_PEAK_TFLOPS = 78.6      # MI355X published FP64 vector (= matrix) rate
WORKLOAD = dict(n=30, depth=40, seed=30002, kmax=5)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(circ, max_gates, budget_s):
    """The oracle as it stands, on the host, on the first gates of the same
    30-qubit circuit (a bounded sample), in gate-applications/s."""
    from oracle import sim
    L = sim.lib()
    n = circ.n
    t0 = time.perf_counter()
    psi = np.empty(1 << n, dtype=np.complex128)
    L.or_init_zero(psi.ctypes.data_as(sim.C.POINTER(sim.C.c_double)), n)
    t_init = time.perf_counter() - t0
    done = 0
    t1 = time.perf_counter()
    for g in circ.gates[:max_gates]:
        sim.apply_gate(psi, g.targets, g.matrix, L)
        done += 1
        if time.perf_counter() - t1 > budget_s:
            break
    dt = time.perf_counter() - t1
    del psi
    return {"value": done / dt, "unit": "gate-applications/s", "cores": sim.num_threads(L), "kind": "oracle",
            "sample": "first %d gates of the 30-qubit depth-40 U3+CZ circuit (of %d), complex128 on the host; "
                      "init %.1f s excluded" % (done, len(circ), t_init),
            "seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-gbg", action="store_true", help="skip the gate-by-gate comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--n", type=int, default=WORKLOAD["n"])
    ap.add_argument("--chunk", type=int, default=0, help="chunk qubits C (0 = library default)")
    ap.add_argument("--reg-qubits", type=int, default=0, help="register qubits per thread r (0 = default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no collectives); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2406_14084_amd import inputs as I
    from paper_2406_14084_amd import qs

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    n, depth, seed, kmax = args.n, WORKLOAD["depth"], WORKLOAD["seed"], WORKLOAD["kmax"]
    circ = I.random_u3_2q(n=n, depth=depth, seed=seed)
    log("circuit: %d qubits, %d gates" % (n, len(circ)))

    t0 = time.perf_counter()
    plan = qs.Plan(circ, kmax=kmax, chunk_qubits=args.chunk, reg_qubits=args.reg_qubits)
    plan_s = time.perf_counter() - t0
    st_plan = plan.stats()
    log("plan: %d blocks + %d swap passes, %.3f s" % (st_plan["blocks"], st_plan["swap_passes"], plan_s))

    state = qs.State(n, "c128")
    terms = [(0, 1, 1.0), (0, 3, 0.5)]           # <Z0> + 0.5 <Z0 Z1>
    stream = torch.cuda.current_stream()

    def step():
        state.init_zero()
        state.apply_plan(plan)
        return state.expect(terms)

    for i in range(args.warmup):
        step()
        log("warmup %d done" % i)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    e0.record(stream)
    val = None
    for i in range(args.steps):
        val = step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    log("timed %d steps: %.2f ms/step (wall %.2f s)" % (args.steps, ms_step, wall))

    # per-launch device times of the dominant kernel (the blocked pass)
    ms_steps, kinds = state.apply_plan_timed(plan)
    torch.cuda.synchronize()
    blk = ms_steps[kinds == 1]
    swp = ms_steps[kinds == 0]
    amp_bytes = 16.0
    pass_bytes = 2.0 * (1 << n) * amp_bytes
    flops_total = st_plan["flops_per_amp"] * float(1 << n)
    nblk = len(blk)
    avg_ms = float(blk.mean()) if nblk else float("nan")
    flops_per_launch = flops_total / max(1, nblk)
    t_hbm = pass_bytes / (HBM_PEAK_GBS * 1e9)
    t_alu = flops_per_launch / (FP64_PEAK_TFLOPS * 1e12)
    ach_gbs = pass_bytes / (avg_ms * 1e-3) / 1e9
    ach_tf = flops_per_launch / (avg_ms * 1e-3) / 1e12
    if t_alu > t_hbm:
        roof = {"bound": "alu", "achieved": round(ach_tf, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach_tf / FP64_PEAK_TFLOPS, 4), "traffic": None}
    else:
        roof = {"bound": "hbm", "achieved": round(ach_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach_gbs / HBM_PEAK_GBS, 4), "traffic": None}
    roof["kernel"] = "k_block (blocked pass)"
    roof["launches"] = nblk
    roof["avg_launch_ms"] = round(avg_ms, 4)
    roof["algorithmic_bytes_per_launch"] = pass_bytes
    roof["algorithmic_flops_per_launch"] = flops_per_launch
    roof["hbm_gbs_per_launch"] = round(ach_gbs, 1)
    roof["fp64_tflops_per_launch"] = round(ach_tf, 2)

    out = {
        "metric": "gate-applications/s (30q complex128 random U3+CZ depth 40, fused kmax=5 + LDS-blocked)",
        "value": round(len(circ) / (ms_step * 1e-3), 2),
        "unit": "gate-applications/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (seeded random circuit, explicit FP64 gate matrices)",
        "config": {"workload": "random U3 + CZ(random perfect matching), %d qubits, depth %d, seed %d, "
                               "complex128 state, fused kmax=%d, chunk %d qubits, %d register qubits"
                               % (n, depth, seed, kmax, st_plan["chunk_qubits"], st_plan["reg_qubits"]),
                   "n": n, "gates": len(circ), "blocks": st_plan["blocks"], "swap_passes": st_plan["swap_passes"],
                   "step": "init |0..0> + apply_plan + <Z0 + 0.5 Z0Z1>"},
        "roofline": roof,
        "hbm_gbs_effective": round((st_plan["blocks"] + st_plan["swap_passes"]) * pass_bytes
                                   / (float(ms_steps.sum()) * 1e-3) / 1e9, 1),
        "plan_seconds": round(plan_s, 4),
        "swap_pass_avg_ms": round(float(swp.mean()), 4) if len(swp) else None,
        "readout_value": val,
    }

    if not args.no_gbg:
        # gate-by-gate comparison on the same circuit: one pass per gate
        state.init_zero()
        torch.cuda.synchronize()
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g0.record(stream)
        for i, g in enumerate(circ.gates):
            state.apply_gate(g.targets, g.matrix)
            if i % 300 == 299:
                log("gbg %d/%d gates" % (i + 1, len(circ)))
        g1.record(stream)
        torch.cuda.synchronize()
        gms = g0.elapsed_time(g1)
        gval = state.expect(terms)
        out["gbg"] = {"value": round(len(circ) / (gms * 1e-3), 2), "unit": "gate-applications/s",
                      "ms": round(gms, 1), "hbm_gbs": round(len(circ) * pass_bytes / (gms * 1e-3) / 1e9, 1),
                      "speedup_fused_vs_gbg": round(gms / ms_step, 2),
                      "readout_abs_diff_vs_fused": abs(gval - val)}
    del state
    torch.cuda.empty_cache()

    if not args.no_cpu:
        log("cpu oracle baseline (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(circ, max_gates=64, budget_s=args.cpu_budget)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
