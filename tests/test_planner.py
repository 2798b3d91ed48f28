"""Host-only tests of the planner behind qs_fuse (no GPU needed).

What is checked is the validity of a plan, which the paper's artifact checks
by replaying swaps and comparing per-qubit gate order (its
validate_circuit_order step): every gate runs exactly once, inside a block
whose chunk holds all of its qubits at that point of the qubit reordering,
and the per-qubit order of gates is the input's.  Which valid plan is chosen
is not unique; plan amplitudes are pinned by the GPU parity tests.
"""
from __future__ import annotations

import math
import re

import numpy as np
import pytest

from paper_2406_14084_amd import inputs as I
from paper_2406_14084_amd import qs


def _replay_check(circ, plan):
    st = plan.stats()
    blocks = plan.blocks()
    layouts = plan.layouts()
    dump = plan.dump()
    # per step kind, in order
    kinds = re.findall(r"^(BLOCK|SWAP) ", dump, flags=re.M)
    assert len(kinds) == len(layouts) - 1
    assert layouts[-1] == list(range(circ.n)), "final layout is not canonical"
    seen = []
    bi = 0
    per_qubit = {q: [] for q in range(circ.n)}
    for s, kind in enumerate(kinds):
        if kind == "SWAP":
            continue
        phys, ids = blocks[bi]
        bi += 1
        l2p = layouts[s]
        chunk = set(phys)
        assert len(chunk) == st["chunk_qubits"]
        # the lowest L physical qubits are always part of the chunk
        assert set(range(st["low_qubits"])) <= chunk
        for g in ids:
            for q in circ.gates[g].targets:
                assert l2p[q] in chunk, (g, q)
                per_qubit[q].append(g)
            seen.append(g)
    assert bi == len(blocks) == st["blocks"]
    assert sorted(seen) == list(range(len(circ))), "every gate exactly once"
    for q in range(circ.n):
        want = [i for i, g in enumerate(circ.gates) if q in g.targets]
        assert per_qubit[q] == want, q
    return st


@pytest.mark.parametrize("n,seed", [(10, 1), (16, 2), (20, 3), (30, 4)])
@pytest.mark.parametrize("swaps", [True, False])
def test_plan_replay_random(n, seed, swaps):
    c = I.random_dense(n, 300, seed, kmax=3)
    p = qs.Plan(c, kmax=4, swaps=swaps)
    _replay_check(c, p)


@pytest.mark.parametrize("gen", ["c1", "c2", "su4", "qft"])
def test_plan_replay_workloads(gen):
    c = {"c1": lambda: I.layered_rotations(),
         "c2": lambda: I.random_u3_2q(n=30, depth=10, seed=30002),
         "su4": lambda: I.random_su4(n=33, depth=8, seed=1),
         "qft": lambda: I.qft(20)}[gen]()
    p = qs.Plan(c, kmax=5)
    st = _replay_check(c, p)
    assert st["blocks"] < len(c)


def test_worked_example_replay():
    """The paper's 14-gate example, chunk of 4 qubits (its finder argument)."""
    c = I.worked_example()
    p = qs.Plan(c, kmax=4, chunk_qubits=4)
    st = _replay_check(c, p)
    # the paper's plan needs 4 gate blocks for these 14 gates at C = 4; gathered
    # chunks need no more than that
    assert st["blocks"] <= 4


def test_worked_example_fused_diagonal_value():
    """RZZ gates with IDs 2, 3, 9 on physical (0,2), (1,3), (0,3) of a 4-qubit
    chunk fuse into one diagonal whose entry |0000> has real part cos(7) =
    0.75390225434330471, the first value the paper prints for its first D4."""
    golden = {}
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "worked_example_d4.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                golden[k] = float(v)
    for key, gates in (("d4_first", [((0, 2), 2.0), ((1, 3), 3.0), ((0, 3), 9.0)]),
                       ("d4_second", [((1, 3), 12.0), ((0, 2), 8.0)])):
        c = I.Circuit(4)
        for tg, th in gates:
            c.add("RZZ", tg, I.g_rzz(th))
        p = qs.Plan(c, kmax=4, chunk_qubits=4)
        st = p.stats()
        assert st["ops"] == 1 and st["ops_diag"] == 1, p.dump()
        line = [ln for ln in p.dump().splitlines() if ln.startswith("D")][0]
        parts = line.split()
        kq = int(parts[0][1:])
        re0 = float(parts[1 + kq])
        assert abs(re0 - golden[key]) <= 2e-16, (line, golden[key])


def test_fusion_reduces_or_keeps_cost():
    """Fusion never adds ops or arithmetic; splitting single-qubit gates into
    phase * rotation * phase may add (cheap diagonal) ops but lowers the
    arithmetic further."""
    c = I.random_u3_2q(n=20, depth=20, seed=5)
    on = qs.Plan(c, kmax=4, fusion=True, split=False).stats()
    off = qs.Plan(c, kmax=4, fusion=False).stats()
    sp = qs.Plan(c, kmax=4, fusion=True).stats()
    assert on["ops"] <= off["ops"]
    assert on["flops_per_amp"] <= off["flops_per_amp"] + 1e-9
    assert sp["ops_rot"] > 0 and sp["ops_dense"][1] == 0
    assert sp["flops_per_amp"] < 0.6 * on["flops_per_amp"]


def test_gbg_planner_one_block_per_gate():
    c = I.random_dense(12, 40, 9, kmax=2)
    p = qs.Plan(c, kmax=2, planner=2)
    st = _replay_check(c, p)
    assert st["blocks"] == len(c)


def test_small_n_single_block():
    for n in (1, 2, 3, 5):
        c = I.random_dense(n, 20, n, kmax=min(3, n))
        p = qs.Plan(c, kmax=3)
        st = _replay_check(c, p)
        assert st["blocks"] == 1


def test_planner_time_small():
    """Planning stays far below simulation time (the paper keeps its optimiser
    under 1 % of the simulation)."""
    c = I.random_u3_2q(n=30, depth=40, seed=30002)
    p = qs.Plan(c, kmax=5)
    assert p.stats()["plan_seconds"] < 2.0


@pytest.mark.parametrize("bad", ["k0", "k6", "dup", "range"])
def test_fuse_rejects_bad_gates(bad):
    c = I.Circuit(6)
    c.add("H", (0,), I.g_h())
    k, t, m = c.arrays()
    if bad == "k0":
        k[0] = 0
    elif bad == "k6":
        k[0] = 6
    elif bad == "dup":
        k[0] = 2
        t[0:2] = [1, 1]
        m = np.zeros(32)
    else:
        t[0] = 6

    class Raw:
        n = 6

        def arrays(self):
            return k, t, m

    with pytest.raises(qs.QSError) as e:
        qs.Plan(Raw(), kmax=3)
    assert e.value.code == -1


@pytest.mark.parametrize("gen,opts", [
    (lambda: I.random_su4(n=24, depth=10, seed=3), dict(kmax=5)),
    (lambda: I.random_dense(22, 200, 8, kmax=3), dict(kmax=4, reg_qubits=3)),
    (lambda: I.qft(20), dict(kmax=3, chunk_qubits=11, low_qubits=5)),
    (lambda: I.layered_rotations(n=26, layers=6, seed=5), dict(kmax=5, dtype="c64")),
])
def test_block_features_consistent(gen, opts):
    """The cost model's step features agree with the plan they describe:
    one row per step, the swap-pass flag, and op counts and flops that add
    up to the plan's own statistics."""
    p = qs.Plan(gen(), **opts)
    f = p.features()
    s = p.stats()
    assert f.shape == (p.nsteps(), qs.COST_FEATURES) and np.all(np.isfinite(f))
    assert int(round(f[:, 0].sum())) == s["swap_passes"]
    assert np.all(f[:, 1] == (1.0 if opts.get("dtype") == "c64" else 0.0))
    cnt = lambda col, scale: int(round(float((f[:, col].astype(np.float64) * scale).sum())))
    for k in range(2, 6):
        assert cnt(10 + k, 8) == s["ops_dense"][k], k
    # single-qubit gates: ungrouped dense ops plus grouped ones (dense 2x2 or split-off rotations)
    assert cnt(11, 8) + cnt(21, 16) == s["ops_dense"][1] + s["ops_rot"]
    assert cnt(16, 8) + cnt(17, 8) + cnt(18, 8) + cnt(19, 8) == s["ops_diag"]
    sign_ops = cnt(18, 8) + cnt(19, 8)
    # stats price every diagonal at 6 flops per amplitude; +-1 diagonals cost none in the features
    assert abs(float((f[:, 22].astype(np.float64) * 256).sum()) + 6 * sign_ops - s["flops_per_amp"]) < 1e-3 * s["flops_per_amp"] + 1


def test_learned_planner_needs_model():
    with pytest.raises(qs.QSError) as e:
        qs.Plan(I.random_su4(n=12, depth=4, seed=1), kmax=5, planner=1)
    assert e.value.code == -1


def test_pass_count_planner_minimises_passes():
    """planner=3 (the paper's objective over the candidate geometries) returns
    a plan with no more passes than any single candidate it searched."""
    c = I.random_su4(n=24, depth=16, seed=9)
    p = qs.Plan(c, kmax=5, planner=3)
    s = p.stats()
    assert s["planner"] == 3 and s["candidates"] > 1
    passes = lambda st: st["blocks"] + st["swap_passes"]
    cands = []
    for C in (11, 12, 13):
        for r in (3, 4, 5):
            for L in (3, 4, 5):
                for k in (2, 3, 4, 5):
                    cands.append(passes(qs.Plan(c, kmax=k, chunk_qubits=C, reg_qubits=r, low_qubits=L).stats()))
    assert passes(s) == min(cands + [passes(qs.Plan(c, kmax=5).stats())])


def test_planner_value_checked():
    with pytest.raises(qs.QSError):
        qs.Plan(I.random_su4(n=8, depth=2, seed=1), kmax=3, planner=7)
