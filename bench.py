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
instances in one launch vs 512 launches, the 31-qubit headline circuits, the
H-gate and Table I micro-benchmarks, and the learned planner against the
tuned heuristic and the fewest-passes plan on a 33-qubit complex128 circuit.
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
FP32_PEAK_TFLOPS = 157.3     # MI355X published FP32 rate
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_C1_SCRIPT = r"""
import sys, time, json
sys.path.insert(0, %r)
from oracle import sim
from paper_2406_14084_amd import inputs as I
c = I.layered_rotations(n=16, layers=20, seed=16001)
L = sim.lib()
psi = sim.zero_state(16)
t = time.perf_counter()
sim.apply_circuit(psi, c, L)
dt = time.perf_counter() - t
print(json.dumps({"seconds": dt, "gates": len(c), "threads": sim.num_threads(L)}))
"""


def cpu_c1_full():
    """The oracle on the whole 16-qubit layered circuit (470 gates), in a
    child process with one OpenMP thread and with the default (all)."""
    import subprocess
    out = {}
    for label, env_threads in (("one_thread", "1"), ("all_threads", None)):
        env = dict(os.environ)
        if env_threads:
            env["OMP_NUM_THREADS"] = env_threads
        r = subprocess.run([sys.executable, "-c", _C1_SCRIPT % ROOT], capture_output=True, text=True, env=env,
                           timeout=300)
        d = json.loads(r.stdout.strip().splitlines()[-1])
        out[label] = {"gate_applications_per_s": round(d["gates"] / d["seconds"], 1), "seconds": round(d["seconds"], 4),
                      "threads": d["threads"]}
    return out


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
    each with its roofline fraction (HBM bytes at 8 TB/s vs its arithmetic at
    the FP32 peak, per pass) and its measured error against the same circuit
    run in complex128 on the GPU (||delta psi||_2, max |delta amp|, 1 - F),
    beside the rigorous bound and the typical estimate of the plan."""
    from tests import c64_bounds as B
    n = 32
    c = I.random_u3_2q(n=n, depth=60, seed=32003, two="CX")
    res = {"workload": "random U3 + CX(random perfect matching), 32 qubits, depth 60, seed 32003, complex64",
           "gates": len(c)}
    ref = qs.State(n, "c128")
    ref.init_zero()
    ref.apply_plan(qs.Plan(c, kmax=5))
    st = qs.State(n, "c64")
    pass_bytes = 2.0 * (1 << n) * 8
    for name, mf in (("mfma", True), ("vector", False)):
        p = qs.Plan(c, kmax=5, dtype="c64", mfma=mf)
        s = p.stats()
        ms = _ms(torch, lambda: (st.init_zero(), st.apply_plan(p)))
        ms_steps, kinds = st.apply_plan_timed(p)
        passes = s["blocks"] + s["swap_passes"]
        t_roof = max(passes * pass_bytes / (HBM_PEAK_GBS * 1e9), s["flops_per_amp"] * (1 << n) / (FP32_PEAK_TFLOPS * 1e12))
        st.init_zero()
        st.apply_plan(p)
        d2, dmax, ov, nrm = 0.0, 0.0, 0.0 + 0.0j, 0.0
        step = 1 << 28
        for i in range(0, 1 << n, step):
            a = st.tensor[i:i + step].to(torch.complex128)
            b = ref.tensor[i:i + step]
            diff = (a - b).abs()
            d2 += float((diff ** 2).sum().item())
            dmax = max(dmax, float(diff.max().item()))
            ov += complex(torch.vdot(b, a).item())
            nrm += float((a.abs() ** 2).sum().item())
        rig, typ = B.bound_for(p)
        res[name] = {"ms": round(ms, 2), "gate_applications_per_s": round(len(c) / (ms * 1e-3), 1),
                     "ops_mfma": s["ops_mfma"], "ops_dense": s["ops_dense"], "blocks": s["blocks"],
                     "swap_passes": s["swap_passes"], "flops_per_amp": s["flops_per_amp"],
                     "roofline_frac": round(t_roof / (float(ms_steps.sum()) * 1e-3), 3),
                     "hbm_gbs": round(passes * pass_bytes / (float(ms_steps.sum()) * 1e-3) / 1e9, 1),
                     "fp32_tflops": round(s["flops_per_amp"] * (1 << n) / (float(ms_steps.sum()) * 1e-3) / 1e12, 2),
                     "vs_complex128": {"l2": math.sqrt(d2), "max_abs": dmax, "one_minus_fidelity": 1 - abs(ov) ** 2 / nrm},
                     "state_error_bound_l2": rig, "typical_estimate_l2": typ}
        log("complex64 32q %s: %.1f ms, ||d||2 %.3e" % (name, ms, math.sqrt(d2)))
    res["speedup_mfma_vs_vector"] = round(res["vector"]["ms"] / res["mfma"]["ms"], 3)
    del st, ref
    torch.cuda.empty_cache()
    # dense two-qubit gates, where 4-5-qubit fused ops do reach the matrix cores
    n2 = 30
    c2 = I.random_su4(n=n2, depth=20, seed=30020)
    st2 = qs.State(n2, "c64")
    pb2 = 2.0 * (1 << n2) * 8
    su = {"workload": "Haar SU(4) on random pairs, 30 qubits, depth 20, seed 30020, complex64", "gates": len(c2)}
    for name, mf in (("mfma", True), ("vector", False)):
        p = qs.Plan(c2, kmax=5, dtype="c64", mfma=mf)
        s = p.stats()
        ms = _ms(torch, lambda: (st2.init_zero(), st2.apply_plan(p)))
        ms_steps, kinds = st2.apply_plan_timed(p)
        passes = s["blocks"] + s["swap_passes"]
        su[name] = {"ms": round(ms, 2), "ops_mfma": s["ops_mfma"], "ops_dense": s["ops_dense"], "blocks": s["blocks"],
                    "swap_passes": s["swap_passes"], "flops_per_amp": s["flops_per_amp"],
                    "hbm_gbs": round(passes * pb2 / (float(ms_steps.sum()) * 1e-3) / 1e9, 1),
                    "fp32_tflops": round(s["flops_per_amp"] * (1 << n2) / (float(ms_steps.sum()) * 1e-3) / 1e12, 2)}
        log("complex64 30q SU(4) %s: %.1f ms (%d matrix-core ops)" % (name, ms, s["ops_mfma"]))
    su["speedup_mfma_vs_vector"] = round(su["vector"]["ms"] / su["mfma"]["ms"], 3)
    res["su4_30q"] = su
    del st2
    return res


def bench_qaoa(torch, I, qs):
    """512 MaxCut QAOA instances (3-regular, 10-20 qubits, p = 4, complex64):
    one graph-captured persistent launch vs 512 sequential launches.  The
    batch is bound by on-chip arithmetic and launch/queue latency, not HBM
    (instances of <= 13 qubits never leave LDS): its roofline line is the
    algorithmic FP32 rate (per layer and amplitude, the cost phase 6 flops and
    each RX a dense 2x2 product, 16) against the FP32 peak."""
    insts = I.qaoa_batch(count=512, p=4, seed=512004)
    b = qs.QaoaBatch(insts, "c64")
    choice, tune_ms = b.autotune()
    b.run(graph=True)
    batched = _ms(torch, lambda: b.run(graph=True), reps=3)
    seq = _ms(torch, lambda: b.run_sequential(), reps=3)
    err = b.error()
    gates = sum(len(q.circuit()) for q in insts)
    flops = sum(float(1 << q.n) * len(q.gammas) * (6 + 16 * q.n) for q in insts)
    log("qaoa batch: %.2f ms batched, %.2f ms sequential" % (batched, seq))
    return {"workload": "512 QAOA MaxCut instances, random 3-regular graphs, 10-20 qubits, p=4, seed 512004, complex64",
            "batched_ms": round(batched, 3), "sequential_ms": round(seq, 3),
            "speedup_batched_vs_sequential": round(seq / batched, 2), "autotune_choice": choice,
            "gate_applications_per_s_batched": round(gates / (batched * 1e-3), 1), "spin_error_flag": err,
            "roofline": {"kernel": "k_qaoa", "bound": "alu", "algorithmic_flops": flops,
                         "achieved_tflops": round(flops / (batched * 1e-3) / 1e12, 2), "peak_tflops": FP32_PEAK_TFLOPS,
                         "frac": round(flops / (batched * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4)}}


TABLE1 = ("H", "U", "X", "CX", "CP", "SWAP", "RX", "RY", "RZ", "RZZ")


def _table1_circuit(I, name, n, seed=71):
    """One gate of the given type on every qubit (two-qubit gates on (q, q+1 mod n))."""
    rng = np.random.default_rng(seed)
    c = I.Circuit(n)
    for q in range(n):
        a = float(rng.uniform(0, 2 * math.pi))
        if name == "H":
            c.add("H", (q,), I.g_h())
        elif name == "U":
            c.add("U", (q,), I.g_u3(*(float(v) for v in rng.uniform(0, 2 * math.pi, 3))))
        elif name == "X":
            c.add("X", (q,), I.g_x())
        elif name in ("RX", "RY", "RZ"):
            c.add(name, (q,), {"RX": I.g_rx, "RY": I.g_ry, "RZ": I.g_rz}[name](a))
        else:
            m = {"CX": I.g_cx(), "CP": I.g_cp(a), "SWAP": I.g_swap(), "RZZ": I.g_rzz(a)}[name]
            c.add(name, (q, (q + 1) % n), m)
    return c


def _touched_fraction(c):
    """Fraction of the state a gate-by-gate pass of each gate reads and
    writes: the rows of its matrix that are not unit diagonal rows (the
    diagonal and permutation kinds touch only those; a control's 0 half is
    such rows)."""
    fr = []
    for g in c.gates:
        m = g.matrix
        unit = sum(1 for r in range(m.shape[0]) if m[r, r] == 1 and np.count_nonzero(m[r]) == 1)
        fr.append((m.shape[0] - unit) / m.shape[0])
    return fr


def bench_micro(torch, I, qs, amp_bytes=16.0):
    """The paper's micro-benchmarks on MI355X: the H-gate qubit sweep (an H
    on every qubit, 24..33 qubits) and the Table I gate set at 31 qubits (one
    gate per qubit), gate by gate (one pass per gate, op kinds) vs fused and
    blocked; time per gate and HBM roofline fraction per point."""
    res = {"h_sweep": [], "table1_31q": []}
    for n in range(24, 34):
        c = _table1_circuit(I, "H", n)
        st = qs.State(n, "c128")
        p = qs.Plan(c, kmax=5)
        s = p.stats()
        pass_bytes = 2.0 * (1 << n) * amp_bytes
        tb = _ms(torch, lambda: st.apply_plan(p))
        tg = _ms(torch, lambda: st.apply_circuit_gbg(c), reps=1)
        passes = s["blocks"] + s["swap_passes"]
        res["h_sweep"].append({
            "n": n, "gates": len(c), "fused_ms": round(tb, 3), "fused_ms_per_gate": round(tb / len(c), 4),
            "fused_passes": passes, "fused_hbm_frac": round(passes * pass_bytes / (tb * 1e-3) / 1e9 / HBM_PEAK_GBS, 3),
            "gbg_ms": round(tg, 3), "gbg_ms_per_gate": round(tg / len(c), 4),
            "gbg_hbm_frac": round(len(c) * pass_bytes / (tg * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)})
        del st
        torch.cuda.empty_cache()
        log("h sweep %d: fused %.2f ms, gbg %.2f ms" % (n, tb, tg))
    n = 31
    st = qs.State(n, "c128")
    st.init_zero()
    pass_bytes = 2.0 * (1 << n) * amp_bytes
    for name in TABLE1:
        c = _table1_circuit(I, name, n)
        p = qs.Plan(c, kmax=5)
        s = p.stats()
        tb = _ms(torch, lambda: st.apply_plan(p))
        tg = _ms(torch, lambda: st.apply_circuit_gbg(c), reps=1)
        touched = sum(_touched_fraction(c))
        passes = s["blocks"] + s["swap_passes"]
        res["table1_31q"].append({
            "gate": name, "gates": len(c), "fused_ms_per_gate": round(tb / len(c), 4), "fused_passes": passes,
            "fused_hbm_frac": round(passes * pass_bytes / (tb * 1e-3) / 1e9 / HBM_PEAK_GBS, 3),
            "gbg_ms_per_gate": round(tg / len(c), 4), "gbg_kind": qs.gate_class(c.gates[0].targets, c.gates[0].matrix)[0],
            "gbg_touched_state_fraction": round(touched / len(c), 3),
            "gbg_hbm_frac": round(touched * pass_bytes / (tg * 1e-3) / 1e9 / HBM_PEAK_GBS, 3),
            "speedup_fused_vs_gbg": round(tg / tb, 2)})
        log("table1 %s: fused %.3f ms/gate, gbg %.3f ms/gate" % (name, tb / len(c), tg / len(c)))
    del st
    res["note"] = ("roofline fractions: algorithmic bytes (a full read+write pass per fused pass; the touched "
                   "fraction of the state per gate-by-gate pass) / time / 8 TB/s")
    return res


def bench_headline31(torch, I, qs):
    """The paper's headline circuits at 31 qubits (Table II): QFT (496 gates)
    and QAOA p = 5 on the complete graph (2,511 gates), complex128, fused and
    blocked, from |0...0>; the paper's single-A100 times are context only."""
    out = {}
    n = 31
    pass_bytes = 2.0 * (1 << n) * 16
    st = qs.State(n, "c128")
    for key, c, paper_s in (("qft31", I.qft(n), 3.6), ("qaoa31_p5", I.qaoa_complete(n=n, p=5, seed=31005), 17.5)):
        t0 = time.perf_counter()
        p = qs.Plan(c, kmax=5)
        plan_s = time.perf_counter() - t0
        s = p.stats()
        ms = _ms(torch, lambda: (st.init_zero(), st.apply_plan(p)))
        ms_steps, kinds = st.apply_plan_timed(p)
        passes = s["blocks"] + s["swap_passes"]
        out[key] = {"gates": len(c), "ms": round(ms, 2), "gate_applications_per_s": round(len(c) / (ms * 1e-3), 1),
                    "blocks": s["blocks"], "swap_passes": s["swap_passes"], "plan_seconds": round(plan_s, 3),
                    "roofline": {"bound": "hbm", "achieved_gbs": round(passes * pass_bytes / (float(ms_steps.sum()) * 1e-3) / 1e9, 1),
                                 "frac": round(passes * pass_bytes / (float(ms_steps.sum()) * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)},
                    "paper_a100_seconds": paper_s}
        log("%s: %.1f ms (%d passes)" % (key, ms, passes))
    del st
    out["note"] = "the paper's numbers are one A100 (another machine, raw circuits): context, not a target"
    return out


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
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-planner comparison at 33 qubits (128 GiB)")
    ap.add_argument("--no-micro", action="store_true", help="skip the H-gate sweep and Table I gate benchmark")
    ap.add_argument("--only", choices=("c64", "qaoa", "headline31", "micro", "learned"), default=None,
                    help="run just this comparison and print its JSON object (for profiling one path)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no collectives); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2406_14084_amd import inputs as I
    from paper_2406_14084_amd import qs

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.only:
        legs = {"c64": bench_c64, "qaoa": bench_qaoa, "headline31": bench_headline31, "micro": bench_micro,
                "learned": bench_learned}
        print(json.dumps({"only": args.only, args.only: legs[args.only](torch, I, qs)}), flush=True)
        return
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
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t_wall = time.perf_counter()
    ev[0].record(stream)
    val = None
    for i in range(args.steps):
        val = step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms_total = ev[0].elapsed_time(ev[-1])
    ms_step = ms_total / args.steps
    per_step = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
    ms_median = float(np.median(per_step))
    log("timed %d steps: %.2f ms/step mean, %.2f median (wall %.2f s)" % (args.steps, ms_step, ms_median, wall))

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
        "ms_per_step_median": round(ms_median, 3),
        "ms_per_step_min_max": [round(min(per_step), 3), round(max(per_step), 3)],
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
        out["headline_31q"] = bench_headline31(torch, I, qs)
        torch.cuda.empty_cache()
    if not args.no_micro:
        out["micro"] = bench_micro(torch, I, qs)
        torch.cuda.empty_cache()
    if not args.no_learned:
        out["learned_planner_33q"] = bench_learned(torch, I, qs)
        torch.cuda.empty_cache()

    if not args.no_cpu:
        log("cpu oracle baseline (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(circ, max_gates=64, budget_s=args.cpu_budget)
        out["cpu_baseline"]["cpu_model"] = cpu_model()
        out["cpu_baseline"]["c1_16q_full_circuit"] = cpu_c1_full()

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
