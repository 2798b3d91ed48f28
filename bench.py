"""Benchmark: 30-qubit complex128 random circuit, fused + LDS-blocked vs gate-by-gate.

Workload: 30 qubits (16 GiB complex128 state), depth 40; every layer is U3
(angles U[0, 2pi)) on all qubits then CZ on a random perfect matching
(1,800 gates, seed 30002).  One timed step = |0...0> initialisation, the
whole fused/blocked plan (kmax = 5), and a Pauli-expectation readout, all
on the GPU through the C ABI.  The plan is built once beforehand (its host
time is reported as plan_seconds, like the paper's separate optimiser time).

Printed: one JSON line with gate-applications/s, the dominant kernel's
roofline figures (per-launch device time from events around every launch;
HBM traffic per launch from the committed hardware-counter summary when it
was taken on the current kernel and planner sources), the gate-by-gate
path's throughput on the same circuit, the CPU oracle timed on a bounded
sample of the same workload, and the variants compared with the plain fused
path: complex64 with matrix-core ops (32 qubits), 512 batched QAOA
instances in one launch vs 512 launches, and (with --learned) the learned
planner on a 33-qubit complex128 circuit.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X published HBM3E bandwidth
FP64_PEAK_TFLOPS = 78.6      # MI355X published FP64 vector (= matrix) rate
WORKLOAD = dict(n=30, depth=40, seed=30002, kmax=5)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_block_traffic_u3cz30.txt")
TRAFFIC_SOURCES = ("paper_2406_14084_amd/csrc/k_block.hip", "paper_2406_14084_amd/csrc/planner.cpp")


def sources_sha256():
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(n):
    """HBM bytes per k_block launch from the counter summary (FETCH_SIZE and
    WRITE_SIZE per dispatch, each scaled by the same counter's reading for a
    copy of known size); None if absent, for another size, or taken on other
    kernel/planner sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv.get("sources_sha256") != sources_sha256() or int(kv["n"]) != n:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


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


def _ms(torch, fn, reps=2):
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def bench_c64(torch, I, qs):
    """32-qubit complex64 U3 + CX depth 60: matrix-core ops vs vector FMA only;
    the rigorous state-error bound of the plan beside it."""
    n = 32
    c = I.random_u3_2q(n=n, depth=60, seed=32003, two="CX")
    st = qs.State(n, "c64")
    res = {"workload": "random U3 + CX(random perfect matching), 32 qubits, depth 60, seed 32003, complex64",
           "gates": len(c)}
    u = 2.0 ** -24
    gam = lambda m: m * u / (1 - m * u)
    for name, mf in (("mfma", True), ("vector", False)):
        p = qs.Plan(c, kmax=5, dtype="c64", mfma=mf)
        s = p.stats()
        ms = _ms(torch, lambda: (st.init_zero(), st.apply_plan(p)))
        phi = (1 + math.sqrt(5)) / 2
        bound = sum(s["ops_dense"][k] * (math.sqrt(2) * gam(2 ** (k + 1)) + u) * 2 ** (k / 2) for k in range(1, 6)) \
            + s["ops_diag"] * (math.sqrt(2) * gam(2) + u) \
            + s["ops_rot"] * (3 * phi ** 2 * (1 + math.sqrt(2)) * u * (1 + 1e-4) + 2e-14)
        res[name] = {"ms": round(ms, 2), "gate_applications_per_s": round(len(c) / (ms * 1e-3), 1),
                     "ops_mfma": s["ops_mfma"], "ops_dense": s["ops_dense"], "blocks": s["blocks"],
                     "swap_passes": s["swap_passes"], "flops_per_amp": s["flops_per_amp"],
                     "state_error_bound_l2": bound}
        log("complex64 32q %s: %.1f ms" % (name, ms))
    res["speedup_mfma_vs_vector"] = round(res["vector"]["ms"] / res["mfma"]["ms"], 3)
    del st
    return res


def bench_qaoa(torch, I, qs):
    """512 MaxCut QAOA instances (3-regular, 10-20 qubits, p = 4, complex64):
    one graph-captured persistent launch vs 512 sequential launches."""
    insts = I.qaoa_batch(count=512, p=4, seed=512004)
    b = qs.QaoaBatch(insts, "c64")
    choice, tune_ms = b.autotune()
    b.run(graph=True)
    batched = _ms(torch, lambda: b.run(graph=True), reps=3)
    seq = _ms(torch, lambda: b.run_sequential(), reps=3)
    err = b.error()
    gates = sum(len(q.circuit()) for q in insts)
    log("qaoa batch: %.2f ms batched, %.2f ms sequential" % (batched, seq))
    return {"workload": "512 QAOA MaxCut instances, random 3-regular graphs, 10-20 qubits, p=4, seed 512004, complex64",
            "batched_ms": round(batched, 3), "sequential_ms": round(seq, 3),
            "speedup_batched_vs_sequential": round(seq / batched, 2), "autotune_choice": choice,
            "gate_applications_per_s_batched": round(gates / (batched * 1e-3), 1), "spin_error_flag": err}


def bench_qft31(torch, I, qs):
    """Context only: the 31-qubit QFT (496 gates, complex128, 32 GiB) that the paper times on one
    A100 (3.6 s there, another machine); here from |0...0> through the fused, blocked path."""
    c = I.qft(31)
    p = qs.Plan(c, kmax=5)
    st = qs.State(31, "c128")
    ms = _ms(torch, lambda: (st.init_zero(), st.apply_plan(p)))
    s = p.stats()
    del st
    log("qft31: %.1f ms" % ms)
    return {"workload": "QFT, 31 qubits, complex128 (496 gates: 31 H + 465 controlled phases)", "ms": round(ms, 2),
            "blocks": s["blocks"], "swap_passes": s["swap_passes"],
            "paper_a100_seconds": 3.6, "note": "the paper's number is on another machine (one A100): context, not a target"}


def bench_learned(torch, I, qs):
    """33-qubit complex128 (128 GiB) depth-60 Haar SU(4) circuit: learned vs heuristic planner."""
    from paper_2406_14084_amd import costmodel
    n = 33
    c = I.random_su4(n=n, depth=60, seed=33005)
    model = costmodel.load_default()
    ph = qs.Plan(c, kmax=5)
    pl = qs.Plan(c, kmax=5, planner=1, cost_model=model)
    pp = qs.Plan(c, kmax=5, planner=3)
    st = qs.State(n, "c128")
    th = _ms(torch, lambda: (st.init_zero(), st.apply_plan(ph)), reps=1)
    tl = _ms(torch, lambda: (st.init_zero(), st.apply_plan(pl)), reps=1)
    tp = _ms(torch, lambda: (st.init_zero(), st.apply_plan(pp)), reps=1)
    s, sp = pl.stats(), pp.stats()
    log("learned 33q: heuristic %.0f ms, learned %.0f ms, fewest passes %.0f ms" % (th, tl, tp))
    del st
    keys = ("planner", "chunk_qubits", "reg_qubits", "low_qubits", "blocks", "swap_passes", "candidates",
            "predicted_ms", "predicted_heuristic_ms")
    return {"workload": "Haar SU(4) on random pairs, 33 qubits, depth 60, seed 33005, complex128",
            "heuristic_ms": round(th, 1), "learned_ms": round(tl, 1), "fewest_passes_ms": round(tp, 1),
            "gain_vs_heuristic": round((th - tl) / th, 4), "gain_vs_fewest_passes": round((tp - tl) / tp, 4),
            "learned_choice": {k: s[k] for k in keys}, "fewest_passes_choice": {k: sp[k] for k in keys}}


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
    ap.add_argument("--no-split", action="store_true",
                    help="keep single-qubit gates whole (no phase * rotation * phase split)")
    ap.add_argument("--no-variants", action="store_true", help="skip the complex64 and batched-QAOA comparisons")
    ap.add_argument("--learned", action="store_true", help="also compare the learned planner at 33 qubits (128 GiB)")
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
    plan = qs.Plan(circ, kmax=kmax, chunk_qubits=args.chunk, reg_qubits=args.reg_qubits, split=not args.no_split)
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
                "frac": round(ach_tf / FP64_PEAK_TFLOPS, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(ach_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach_gbs / HBM_PEAK_GBS, 4)}
    tr = measured_traffic(n) if (args.chunk == 0 and args.reg_qubits == 0 and not args.no_split) else None
    roof["traffic"] = tr
    if tr is not None:
        roof["traffic_over_algorithmic"] = round(tr / pass_bytes, 4)
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

    if not args.no_variants:
        out["complex64_32q"] = bench_c64(torch, I, qs)
        torch.cuda.empty_cache()
        out["qaoa_batch"] = bench_qaoa(torch, I, qs)
        torch.cuda.empty_cache()
        out["context_qft31"] = bench_qft31(torch, I, qs)
        torch.cuda.empty_cache()
    if args.learned:
        out["learned_planner_33q"] = bench_learned(torch, I, qs)
        torch.cuda.empty_cache()

    if not args.no_cpu:
        log("cpu oracle baseline (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(circ, max_gates=64, budget_s=args.cpu_budget)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
