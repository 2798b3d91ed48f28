"""The paper's circuit text formats and its planning model (artifact
appendix of arXiv 2406.14084: the raw circuit read by its optimiser, the
optimised circuit it writes, and the order check run on the result).

Raw circuit: one gate per line, "TYPE t1 [t2 ...] ID [parameters]".  The
worked example (Fig. 5a) gives no parameters; `angle_from_id` reads a missing
angle as the gate ID, the reading under which the printed fused-diagonal
values come out (cos 7 and cos 10).

Optimised circuit (Fig. 5b/5c): a sequence of steps, each a count line and
that many lines:
  - a gate block: gate lines "TYPE p1 [p2 ...] ID" with the *physical*
    targets (all below the chunk size C: a block runs on the lowest C
    physical qubits), or fused diagonal lines
    "D<k> p1 ... pk re_0 im_0 ... re_{2^k-1} im_{2^k-1} ID i1 i2 ..."
    (entries in local-index order, first listed target = most significant
    bit, as in Eq. 3; the trailing IDs name the merged gates -- the paper
    elides this "remaining information");
  - an in-memory swap (Eq. 4, Alg. 4): "SQS s a1 .. as b1 .. bs" exchanges
    physical qubits a_j <-> b_j;
  - a cross-rank swap (Alg. 5): "CSQS s a1 .. as b1 .. bs", the s highest
    local qubits a_j with rank qubits b_j (one GPU executes it like SQS).

`plan_paper` is the paper's model of Sec. IV (Eq. 5-7, Alg. 1-2): the chunk
is the lowest C physical qubits, the chunk set of each gate block is chosen
greedily to run as many pending gates (in dependency order) as possible
once the current chunk can run none, from the local qubits while they can
run a gate, and swaps bring the chosen qubits in; with rank qubits (local qubits R < n) a qubit above R comes
in through the top local positions (SQS, CSQS, SQS), as in the worked
example.  Inside a block, diagonal gates merge into one D_k over at most F
qubits (Alg. 2 third level, the artifact's diagonal fusion).  Plans are not
unique: `validate` checks what any valid plan must satisfy (the artifact's
validate_circuit_order): every gate once, physical targets inside the chunk
mapping back to the raw targets through the replayed swaps, per-qubit gate
order preserved, and fused diagonal values equal to the product of their
members' diagonals.

This module is host tooling around the library (the library's own planner,
qs_fuse, plans for the MI355X kernels: gathered chunks, folded swaps); run as
`python -m paper_2406_14084_amd.paper_format finder RAW C R n swaps cswaps F
fusion` (the paper's argument order) or `... validate RAW OPT C`.
"""
from __future__ import annotations

import sys

import numpy as np

from . import inputs as I

ARITY = {"H": 1, "X": 1, "Y": 1, "Z": 1, "S": 1, "T": 1, "RX": 1, "RY": 1, "RZ": 1, "U3": 1,
         "CX": 2, "CNOT": 2, "CZ": 2, "CP": 2, "SWAP": 2, "RZZ": 2}
NPARAM = {"RX": 1, "RY": 1, "RZ": 1, "U3": 3, "CP": 1, "RZZ": 1}
SYMMETRIC = {"CZ", "CP", "SWAP", "RZZ"}


def gate_matrix(name, params):
    if name == "H":
        return I.g_h()
    if name == "X":
        return I.g_x()
    if name == "Y":
        return I.g_y()
    if name == "Z":
        return I.g_z()
    if name == "S":
        return np.diag([1, 1j]).astype(np.complex128)
    if name == "T":
        return np.diag([1, np.exp(0.25j * np.pi)]).astype(np.complex128)
    if name == "RX":
        return I.g_rx(params[0])
    if name == "RY":
        return I.g_ry(params[0])
    if name == "RZ":
        return I.g_rz(params[0])
    if name == "U3":
        return I.g_u3(*params)
    if name in ("CX", "CNOT"):
        return I.g_cx()
    if name == "CZ":
        return I.g_cz()
    if name == "CP":
        return I.g_cp(params[0])
    if name == "SWAP":
        return I.g_swap()
    if name == "RZZ":
        return I.g_rzz(params[0])
    raise ValueError("unknown gate type %r" % name)


class RawGate:
    def __init__(self, name, targets, gid, params, matrix):
        self.name, self.targets, self.gid, self.params, self.matrix = name, tuple(targets), gid, params, matrix

    @property
    def diag(self):
        m = self.matrix
        return bool(np.all(m == np.diag(np.diag(m))))


def parse_raw(text, n=None, angle_from_id=False):
    """[RawGate] from raw-circuit text, and n (given, or 1 + the largest target)."""
    gates = []
    for ln, line in enumerate(text.splitlines(), 1):
        f = line.split("#")[0].split()
        if not f:
            continue
        name = f[0].upper()
        if name not in ARITY:
            raise ValueError("line %d: unknown gate type %r" % (ln, f[0]))
        k = ARITY[name]
        if len(f) < k + 2:
            raise ValueError("line %d: expected %d targets and an ID" % (ln, k))
        tg = [int(x) for x in f[1:1 + k]]
        gid = int(f[1 + k])
        rest = [float(x) for x in f[2 + k:2 + k + NPARAM.get(name, 0)]]
        if len(rest) < NPARAM.get(name, 0):
            if not angle_from_id:
                raise ValueError("line %d: %s needs %d parameter(s)" % (ln, name, NPARAM[name]))
            rest = [float(gid)] * NPARAM[name]
        if len(set(tg)) != k:
            raise ValueError("line %d: repeated target" % ln)
        gates.append(RawGate(name, tg, gid, rest, gate_matrix(name, rest)))
    nn = max((max(g.targets) for g in gates), default=-1) + 1
    if n is None:
        n = nn
    elif nn > n:
        raise ValueError("a target exceeds n = %d" % n)
    return gates, n


def to_circuit(gates, n):
    """inputs.Circuit of the raw gates (explicit matrices), for qs_fuse and the oracle."""
    c = I.Circuit(n)
    for g in gates:
        c.add(g.name, g.targets, g.matrix)
    return c


def raw_text(gates):
    out = []
    for g in gates:
        ps = "".join(" %.17g" % p for p in g.params)
        out.append("%s %s %d%s" % (g.name, " ".join(map(str, g.targets)), g.gid, ps))
    return "\n".join(out) + "\n"


# ---------------------------------------------------------------------------
# planning in the paper's model
# ---------------------------------------------------------------------------
def _executable(gates, rem, inS):
    """Pending gates (indices into gates, in order) that run with the chunk
    holding the logical qubits inS: a gate runs when all its qubits are in the
    chunk and no earlier pending gate that did not run shares a qubit."""
    blocked = set()
    take = []
    for i in rem:
        q = gates[i].targets
        if all(inS[x] for x in q) and not any(x in blocked for x in q):
            take.append(i)
        else:
            blocked.update(q)
    return take


def _choose_chunk(gates, rem, n, C, current, allowed):
    """Chunk set grown gate by gate: scan the pending gates in order; a gate
    whose qubits are allowed, not blocked by an earlier skipped gate, and fit
    (with the qubits taken so far) in C joins and brings its qubits; any other
    gate blocks its qubits.  Free places are then filled with qubits already in
    the chunk (no swap), then the lowest others."""
    S, blocked = set(), set()
    for i in rem:
        q = set(gates[i].targets)
        if (q & blocked) or not q <= allowed or len(S | q) > C:
            blocked |= q
            continue
        S |= q
    # (current members highest logical index first: the reading under which the
    # worked example's printed swaps come out)
    for q in sorted(current, reverse=True) + [x for x in sorted(allowed) if x not in current] + list(range(n)):
        if len(S) >= C:
            break
        S.add(q)
    inS = [False] * n
    for q in S:
        inS[q] = True
    return inS


def _fuse_block(lines, F):
    """Merge diagonal gate lines of one block into D_k lines over at most F
    physical qubits; a merged line sits where its first member was, so a later
    member joins only if no gate placed since then shares a qubit with it."""
    out = []
    group = None          # index into out of the open group
    blocked = set()
    for ln in lines:
        kind, name, phys, g = ln
        if g.diag:
            if group is not None:
                U = set(out[group]["phys"]) | set(phys)
                if len(U) <= F and not (set(phys) & blocked):
                    out[group]["members"].append(ln)
                    out[group]["phys"] = sorted(U)
                    continue
            out.append({"members": [ln], "phys": sorted(phys)})
            group = len(out) - 1
            blocked = set()
        else:
            out.append({"members": [ln], "phys": list(phys)})
            if group is not None:
                blocked.update(phys)
    res = []
    for item in out:
        if len(item["members"]) == 1:
            res.append(item["members"][0])
        else:
            res.append(("D", item["phys"], item["members"]))
    return res


def fused_diagonal(phys, members):
    """Entries of the merged diagonal on physical qubits phys (first = MSB):
    the product of every member's diagonal entry at that index."""
    k = len(phys)
    d = np.ones(1 << k, dtype=np.complex128)
    pos = {p: k - 1 - i for i, p in enumerate(phys)}
    for _, _, mp, g in members:
        e = np.diag(g.matrix)
        km = len(mp)
        for idx in range(1 << k):
            li = 0
            for j, p in enumerate(mp):
                li |= ((idx >> pos[p]) & 1) << (km - 1 - j)
            d[idx] *= e[li]
    return d


def plan_paper(gates, n, C, R=None, swaps=True, cswaps=True, F=0, fusion=False):
    """Steps of a plan in the paper's model: ("BLOCK", lines) with lines
    ("G", name, phys targets, gate) or ("D", phys, members); ("SQS", a, b);
    ("CSQS", a, b)."""
    R = n if R is None else R
    if not (1 <= C <= R <= n):
        raise ValueError("need 1 <= cache size <= local qubits <= n")
    l2p = list(range(n))
    p2l = list(range(n))
    rem = list(range(len(gates)))
    steps = []

    def swap(kind, a, b):
        for x, y in zip(a, b):
            qa, qb = p2l[x], p2l[y]
            p2l[x], p2l[y] = qb, qa
            l2p[qa], l2p[qb] = y, x
        steps.append((kind, list(a), list(b)))

    while rem:
        current = {p2l[p] for p in range(C)}
        inS = [False] * n
        for q in current:
            inS[q] = True
        take = _executable(gates, rem, inS)
        if swaps and not take:
            # the current chunk is spent: choose the next chunk set, from the
            # local qubits while they can run a gate (no cross-rank swap), else
            # from all qubits
            local = {p2l[p] for p in range(R)}
            inS = _choose_chunk(gates, rem, n, C, current, local)
            take = _executable(gates, rem, inS)
            if not take and R < n:
                inS = _choose_chunk(gates, rem, n, C, current, set(range(n)))
                take = _executable(gates, rem, inS)
        if not take:
            raise ValueError("no gate fits a chunk of %d qubits" % C)
        want = {q for q in range(n) if inS[q]}
        incoming = sorted((l2p[q] for q in want if l2p[q] >= C))
        vacate = sorted(p for p in range(C) if p2l[p] not in want)
        local_in = [b for b in incoming if b < R]
        rank_in = [b for b in incoming if b >= R]
        if rank_in:
            if not cswaps:
                raise ValueError("a block needs a rank qubit but cross-rank swaps are off")
            s = len(rank_in)
            low = vacate[:s]
            top = list(range(R - s, R))
            swap("SQS", low, top)
            swap("CSQS", top, rank_in)
            swap("SQS", low, top)
            vacate = vacate[s:]
        if local_in:
            swap("SQS", vacate[:len(local_in)], local_in)
        lines = [("G", gates[i].name, [l2p[q] for q in gates[i].targets], gates[i]) for i in take]
        assert all(p < C for ln in lines for p in ln[2])
        if fusion and F > 1:
            lines = _fuse_block(lines, F)
        steps.append(("BLOCK", lines))
        done = set(take)
        rem = [i for i in rem if i not in done]
    return steps


def write_optimized(steps):
    out = []
    for st in steps:
        if st[0] == "BLOCK":
            out.append(str(len(st[1])))
            for ln in st[1]:
                if ln[0] == "G":
                    _, name, phys, g = ln
                    if name in SYMMETRIC:
                        phys = sorted(phys)
                    out.append("%s %s %d" % (name, " ".join(map(str, phys)), g.gid))
                else:
                    _, phys, members = ln
                    d = fused_diagonal(phys, members)
                    vals = " ".join("%.17g %.17g" % (z.real, z.imag) for z in d)
                    ids = " ".join(str(m[3].gid) for m in members)
                    out.append("D%d %s %s ID %s" % (len(phys), " ".join(map(str, phys)), vals, ids))
        else:
            kind, a, b = st
            out.append("1")
            out.append("%s %d %s %s" % (kind, len(a), " ".join(map(str, a)), " ".join(map(str, b))))
    return "\n".join(out) + "\n"


# ---------------------------------------------------------------------------
# order check (the artifact's validate_circuit_order, restated)
# ---------------------------------------------------------------------------
def validate(gates, n, opt_text, C, require_values=True):
    """Replay an optimised circuit against the raw gates; returns a summary
    dict, raises ValueError naming the first violation."""
    by_id = {g.gid: g for g in gates}
    if len(by_id) != len(gates):
        raise ValueError("raw gate IDs are not unique")
    p2l = list(range(n))
    seen = []
    per_qubit = {q: [] for q in range(n)}
    lines = [ln.split("#")[0].split() for ln in opt_text.splitlines()]
    lines = [f for f in lines if f]
    i = 0
    nblocks = nswaps = ncswaps = nfused = 0
    while i < len(lines):
        cnt = int(lines[i][0])
        body = lines[i + 1:i + 1 + cnt]
        if len(body) != cnt:
            raise ValueError("step at line %d is short" % (i + 1))
        i += 1 + cnt
        if body and body[0][0] in ("SQS", "CSQS"):
            for f in body:
                s = int(f[1])
                a, b = [int(x) for x in f[2:2 + s]], [int(x) for x in f[2 + s:2 + 2 * s]]
                if len(set(a + b)) != 2 * s:
                    raise ValueError("%s exchanges a qubit twice" % f[0])
                for x, y in zip(a, b):
                    p2l[x], p2l[y] = p2l[y], p2l[x]
                nswaps += f[0] == "SQS"
                ncswaps += f[0] == "CSQS"
            continue
        nblocks += 1
        for f in body:
            if f[0].startswith("D") and f[0][1:].isdigit():
                k = int(f[0][1:])
                phys = [int(x) for x in f[1:1 + k]]
                vals = [float(x) for x in f[1 + k:1 + k + 2 * (1 << k)]]
                ids = [int(x) for x in f[f.index("ID") + 1:]] if "ID" in f else []
                if not ids:
                    raise ValueError("fused line without member IDs cannot be order-checked")
                if any(p >= C for p in phys):
                    raise ValueError("D line reaches outside the chunk")
                members = []
                for gid in ids:
                    g = by_id[gid]
                    logical = {p2l[p] for p in phys}
                    if not set(g.targets) <= logical or not g.diag:
                        raise ValueError("gate %d is not a diagonal on the D line's qubits" % gid)
                    members.append(("G", g.name, [phys[[p2l[p] for p in phys].index(q)] for q in g.targets], g))
                    for q in g.targets:
                        per_qubit[q].append(gid)
                    seen.append(gid)
                if require_values and vals:
                    want = fused_diagonal(phys, members)
                    got = np.array(vals[0::2]) + 1j * np.array(vals[1::2])
                    if got.size != want.size or np.max(np.abs(got - want)) > 1e-12:
                        raise ValueError("D line values differ from the product of its members")
                nfused += 1
                continue
            name = f[0].upper()
            k = ARITY[name]
            phys = [int(x) for x in f[1:1 + k]]
            gid = int(f[1 + k])
            g = by_id.get(gid)
            if g is None or g.name.upper() != name:
                raise ValueError("unknown gate ID %d or wrong type" % gid)
            if any(p >= C for p in phys):
                raise ValueError("gate %d has a physical target outside the chunk" % gid)
            logical = [p2l[p] for p in phys]
            ok = logical == list(g.targets) or (name in SYMMETRIC and sorted(logical) == sorted(g.targets))
            if not ok:
                raise ValueError("gate %d maps to qubits %s, raw targets %s" % (gid, logical, g.targets))
            for q in g.targets:
                per_qubit[q].append(gid)
            seen.append(gid)
    if sorted(seen) != sorted(by_id):
        raise ValueError("gates missing or repeated")
    for q in range(n):
        want = [g.gid for g in gates if q in g.targets]
        if per_qubit[q] != want:
            raise ValueError("qubit %d: order %s, raw %s" % (q, per_qubit[q], want))
    return {"blocks": nblocks, "sqs": nswaps, "csqs": ncswaps, "fused": nfused,
            "final_layout_canonical": p2l == list(range(n))}


def main(argv):
    if len(argv) >= 9 and argv[0] == "finder":
        raw, C, Rk, n, sw, cs, F, fu = argv[1], *map(int, argv[2:9])
        gates, n = parse_raw(open(raw).read(), n=n, angle_from_id=True)
        steps = plan_paper(gates, n, C, R=Rk, swaps=bool(sw), cswaps=bool(cs), F=F, fusion=bool(fu))
        sys.stdout.write(write_optimized(steps))
        return 0
    if len(argv) == 4 and argv[0] == "validate":
        gates, n = parse_raw(open(argv[1]).read(), angle_from_id=True)
        res = validate(gates, n, open(argv[2]).read(), int(argv[3]))
        print("Passed the circuit order validation:", res)
        return 0
    print("usage: python -m paper_2406_14084_amd.paper_format finder RAW cache rank qubits swaps cswaps fusion_size fusion\n"
          "       python -m paper_2406_14084_amd.paper_format validate RAW OPTIMISED cache", file=sys.stderr)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
