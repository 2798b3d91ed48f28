"""The paper's circuit text formats and planning model (artifact appendix):
raw-circuit reader, the optimised-circuit writer, the order check, and the
worked example of Fig. 5 at chunk size 4 (host only)."""
from __future__ import annotations

import os

import numpy as np
import pytest

from oracle import sim
from paper_2406_14084_amd import inputs as I
from paper_2406_14084_amd import paper_format as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    with open(os.path.join(GOLD, name)) as f:
        return f.read()


def _lines(text):
    return [ln.split() for ln in text.splitlines() if ln.split() and not ln.startswith("#")]


def _steps(text):
    """[(kind, sorted lines)] per step; a block's lines as a multiset."""
    f = _lines(text)
    out, i = [], 0
    while i < len(f):
        cnt = int(f[i][0])
        body = [" ".join(x) for x in f[i + 1:i + 1 + cnt]]
        i += 1 + cnt
        kind = body[0].split()[0] if body and body[0].split()[0] in ("SQS", "CSQS") else "BLOCK"
        out.append((kind, sorted(body) if kind == "BLOCK" else body))
    return out


def example():
    return P.parse_raw(_read("worked_example_raw.txt"), angle_from_id=True)


def test_parse_worked_example():
    gates, n = example()
    assert n == 10 and len(gates) == 14
    assert [g.gid for g in gates] == list(range(14))
    assert gates[2].name == "RZZ" and gates[2].targets == (2, 4) and gates[2].params == [2.0]
    again, n2 = P.parse_raw(P.raw_text(gates))
    assert n2 == n and [(g.name, g.targets, g.gid) for g in again] == [(g.name, g.targets, g.gid) for g in gates]
    c = P.to_circuit(gates, n)
    ref = I.worked_example()
    assert all(np.array_equal(a.matrix, b.matrix) and a.targets == b.targets for a, b in zip(c.gates, ref.gates))


def test_parse_rejects_bad_lines():
    for bad in ("FOO 1 0", "H 0", "RZZ 1 1 3 0.5", "RX 0 4"):
        with pytest.raises(ValueError):
            P.parse_raw(bad)


def test_printed_plan_passes_order_check():
    """Fig. 5(b) as printed replays: every gate once, targets inside the
    4-qubit chunk and mapping back to the raw targets, per-qubit order kept."""
    gates, n = example()
    res = P.validate(gates, n, _read("worked_example_optimized_fig5b.txt"), 4)
    assert res["blocks"] == 4 and res["sqs"] == 5 and res["csqs"] == 1


def test_worked_example_plan_matches_printed():
    """finder raw.txt 4 8 10 1 1 0 0: the same steps, swaps and block
    contents as the printed Fig. 5(b) (independent gates of a block may be
    listed in another order)."""
    gates, n = example()
    text = P.write_optimized(P.plan_paper(gates, n, 4, R=8, swaps=True, cswaps=True))
    assert _steps(text) == _steps(_read("worked_example_optimized_fig5b.txt"))
    P.validate(gates, n, text, 4)


def test_worked_example_fused_values():
    """finder raw.txt 4 8 10 1 1 4 1: RZZ 2, 3, 9 and RZZ 12, 8 merge into two
    D4 lines whose first entries have the printed real parts (cos 7 and
    cos 10); the fused plan passes the order check with its values."""
    gates, n = example()
    gold = dict(ln.split() for ln in _read("worked_example_d4.txt").splitlines()
                if ln.strip() and not ln.startswith("#"))
    text = P.write_optimized(P.plan_paper(gates, n, 4, R=8, F=4, fusion=True))
    d = [f for f in _lines(text) if f[0] == "D4"]
    assert len(d) == 2
    assert [sorted(int(x) for x in f[f.index("ID") + 1:]) for f in d] == [[2, 3, 9], [8, 12]]
    assert abs(float(d[0][5]) - float(gold["d4_first"])) <= 2e-16
    assert abs(float(d[1][5]) - float(gold["d4_second"])) <= 2e-16
    res = P.validate(gates, n, text, 4)
    assert res["fused"] == 2


def _execute(text, gates, n, C):
    """Run an optimised circuit with the oracle: gates on their physical
    targets, swaps as Eq. 4 bit exchanges; returns the state in logical order."""
    by_id = {g.gid: g for g in gates}
    psi = sim.zero_state(n)
    p2l = list(range(n))
    f = _lines(text)
    i = 0
    while i < len(f):
        cnt = int(f[i][0])
        for ln in f[i + 1:i + 1 + cnt]:
            if ln[0] in ("SQS", "CSQS"):
                s = int(ln[1])
                a, b = [int(x) for x in ln[2:2 + s]], [int(x) for x in ln[2 + s:2 + 2 * s]]
                sim.swap_qubits(psi, a, b)
                for x, y in zip(a, b):
                    p2l[x], p2l[y] = p2l[y], p2l[x]
            elif ln[0].startswith("D"):
                k = int(ln[0][1:])
                phys = [int(x) for x in ln[1:1 + k]]
                v = np.array([float(x) for x in ln[1 + k:1 + k + 2 * (1 << k)]])
                sim.apply_gate(psi, phys, np.diag(v[0::2] + 1j * v[1::2]))
            else:
                g = by_id[int(ln[1 + P.ARITY[ln[0]]])]
                phys = [int(x) for x in ln[1:1 + P.ARITY[ln[0]]]]
                # printed targets of symmetric gates may be sorted: apply in raw order
                l2p = {p2l[p]: p for p in phys}
                sim.apply_gate(psi, [l2p[q] for q in g.targets], g.matrix)
        i += 1 + cnt
    # undo the final layout: logical q sits at physical position l2p[q]
    out = np.empty_like(psi)
    idx = np.arange(1 << n)
    log = np.zeros(1 << n, dtype=np.int64)
    for p in range(n):
        log |= ((idx >> p) & 1) << p2l[p]
    out[log] = psi
    return out


@pytest.mark.parametrize("fusion", [False, True])
def test_optimised_text_executes_to_the_oracle_state(fusion, oracle_lib):
    """Executing the written plan line by line (physical targets, SQS/CSQS
    exchanges, fused diagonals from their printed values) gives the raw
    circuit's state: the worked example, and random circuits with rank
    qubits."""
    cases = [(example(), 4, 8)]
    rng = np.random.default_rng(5)
    for seed in range(3):
        lines = []
        names = ["H", "RZZ", "CX", "RX", "CZ", "SWAP", "CP", "T"]
        for gid in range(60):
            nm = names[rng.integers(len(names))]
            tg = rng.choice(11, P.ARITY[nm], replace=False)
            ps = " ".join("%.6f" % x for x in rng.uniform(0, 6, P.NPARAM.get(nm, 0)))
            lines.append("%s %s %d %s" % (nm, " ".join(map(str, tg)), gid, ps))
        cases.append((P.parse_raw("\n".join(lines), n=11), 5, 9))
    for (gates, n), C, R in cases:
        text = P.write_optimized(P.plan_paper(gates, n, C, R=R, F=C if fusion else 0, fusion=fusion))
        P.validate(gates, n, text, C)
        want = sim.run(P.to_circuit(gates, n))
        got = _execute(text, gates, n, C)
        assert np.max(np.abs(got - want)) <= 1e-12


def test_order_check_catches_mistakes():
    gates, n = example()
    good = P.write_optimized(P.plan_paper(gates, n, 4, R=8, F=4, fusion=True))
    P.validate(gates, n, good, 4)
    L = good.splitlines()
    muts = []
    # two dependent gates of the first block swapped with a later one: H 13 before the D4
    j = next(i for i, ln in enumerate(L) if ln.startswith("D4"))
    m = list(L)
    m[j], m[j + 1] = m[j + 1], m[j]
    muts.append(m)
    # a swap line with a wrong partner
    m = list(L)
    k = next(i for i, ln in enumerate(L) if ln.startswith("SQS 3"))
    m[k] = m[k].replace("4 5 7", "4 5 6")
    muts.append(m)
    # a changed fused value
    m = list(L)
    parts = m[j].split()
    parts[5] = "0.7539"
    m[j] = " ".join(parts)
    muts.append(m)
    # a target outside the chunk
    m = list(L)
    m[1] = "H 5 0"
    muts.append(m)
    for m in muts:
        with pytest.raises(ValueError):
            P.validate(gates, n, "\n".join(m) + "\n", 4)


def test_cli(tmp_path, capsys):
    raw = tmp_path / "raw.txt"
    raw.write_text(_read("worked_example_raw.txt"))
    assert P.main(["finder", str(raw), "4", "8", "10", "1", "1", "4", "1"]) == 0
    opt = tmp_path / "opt.txt"
    opt.write_text(capsys.readouterr().out)
    assert P.main(["validate", str(raw), str(opt), "4"]) == 0
    assert "Passed" in capsys.readouterr().out
