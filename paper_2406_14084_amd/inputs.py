"""Seeded synthetic inputs: gate matrices and circuit generators.

This module is shared by the HIP path (bench, binding callers) and the CPU
oracle's tests.  It holds no part of the simulation method itself -- no state
vector is touched here, nothing is fused, blocked or reordered.  It only
writes down circuits: ordered gate lists, each with its target qubits and an
explicit FP64 matrix, so that both sides see bit-identical inputs.

Gate matrices follow the OpenQASM 2 / Qiskit definitions (the paper's gate
table, Sec. VI-A Table I, names the gates without giving matrices):
  RX(t) = exp(-i t X/2), RY(t) = exp(-i t Y/2), RZ(t) = exp(-i t Z/2),
  U3(t, p, l) = [[cos t/2, -e^{il} sin t/2], [e^{ip} sin t/2, e^{i(p+l)} cos t/2]],
  CP(l) = diag(1, 1, 1, e^{il}), RZZ(t) = exp(-i t Z(x)Z/2).
The half angle of RZZ matches the fused-diagonal values printed in the
paper's artifact appendix (the D4 entries equal cos(7) and cos(10)).

Multi-qubit matrices use the paper's Eq. 3 index order: for targets
(t0, t1, ...), t0 is the most significant bit of the local row/column index
(for CX, t0 is the control).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

# ----------------------------------------------------------------------------
# gate matrices (complex128)
# ----------------------------------------------------------------------------
_S2 = 1.0 / math.sqrt(2.0)


def g_h():
    return np.array([[_S2, _S2], [_S2, -_S2]], dtype=np.complex128)


def g_x():
    return np.array([[0, 1], [1, 0]], dtype=np.complex128)


def g_y():
    return np.array([[0, -1j], [1j, 0]], dtype=np.complex128)


def g_z():
    return np.array([[1, 0], [0, -1]], dtype=np.complex128)


def g_rx(t):
    c, s = math.cos(t / 2), math.sin(t / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def g_ry(t):
    c, s = math.cos(t / 2), math.sin(t / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def g_rz(t):
    return np.array([[np.exp(-0.5j * t), 0], [0, np.exp(0.5j * t)]], dtype=np.complex128)


def g_u3(t, p, l):
    c, s = math.cos(t / 2), math.sin(t / 2)
    return np.array([[c, -np.exp(1j * l) * s],
                     [np.exp(1j * p) * s, np.exp(1j * (p + l)) * c]], dtype=np.complex128)


def g_cx():
    m = np.eye(4, dtype=np.complex128)
    m[2:, 2:] = [[0, 1], [1, 0]]
    return m


def g_cz():
    return np.diag([1, 1, 1, -1]).astype(np.complex128)


def g_cp(l):
    return np.diag([1, 1, 1, np.exp(1j * l)]).astype(np.complex128)


def g_swap():
    m = np.zeros((4, 4), dtype=np.complex128)
    m[0, 0] = m[1, 2] = m[2, 1] = m[3, 3] = 1
    return m


def g_rzz(t):
    a, b = np.exp(-0.5j * t), np.exp(0.5j * t)
    return np.diag([a, b, b, a]).astype(np.complex128)


def g_cut_phase(gamma):
    """exp(-i gamma [z_u != z_v]) on one edge: diag(1, e^{-ig}, e^{-ig}, 1)."""
    e = np.exp(-1j * gamma)
    return np.diag([1, e, e, 1]).astype(np.complex128)


def g_haar(rng: np.random.Generator, dim: int):
    """Haar-random SU(dim): QR of a complex Gaussian matrix, R-diagonal phase
    fix (Mezzadri's recipe), then divided by det^(1/dim).  Draw order: the
    real parts (dim*dim normals), then the imaginary parts."""
    re = rng.standard_normal((dim, dim))
    im = rng.standard_normal((dim, dim))
    z = (re + 1j * im) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    q = q * (d / np.abs(d))[None, :]
    det = np.linalg.det(q)
    q = q / det ** (1.0 / dim)
    return q.astype(np.complex128)


# ----------------------------------------------------------------------------
# circuits
# ----------------------------------------------------------------------------
@dataclass
class Gate:
    name: str
    targets: tuple
    matrix: np.ndarray  # (2^k, 2^k) complex128

    @property
    def k(self):
        return len(self.targets)


@dataclass
class Circuit:
    n: int
    gates: list = field(default_factory=list)

    def add(self, name, targets, matrix):
        targets = tuple(int(t) for t in targets)
        m = np.ascontiguousarray(matrix, dtype=np.complex128)
        assert m.shape == (1 << len(targets),) * 2, (name, targets, m.shape)
        assert len(set(targets)) == len(targets) and all(0 <= t < self.n for t in targets)
        self.gates.append(Gate(name, targets, m))
        return self

    def __len__(self):
        return len(self.gates)

    def arrays(self):
        """Flat arrays in the C layout: k[g] (int32), targets[5*g + j] (int32,
        unused slots -1) and the matrices concatenated row-major as
        interleaved (re, im) float64, 2 * 4^k[g] values per gate."""
        ng = len(self.gates)
        k = np.array([g.k for g in self.gates], dtype=np.int32)
        t = np.full((ng, 5), -1, dtype=np.int32)
        for i, g in enumerate(self.gates):
            t[i, :g.k] = g.targets
        if ng:
            mats = np.concatenate([g.matrix.reshape(-1).view(np.float64) for g in self.gates])
        else:
            mats = np.zeros(0, dtype=np.float64)
        return k, t.reshape(-1).copy(), np.ascontiguousarray(mats, dtype=np.float64)

    def inverse(self):
        """U^dagger of the whole circuit: reversed order, conjugate transposes."""
        inv = Circuit(self.n)
        for g in reversed(self.gates):
            inv.add(g.name + "_dg", g.targets, g.matrix.conj().T)
        return inv

    def counts(self):
        out = {}
        for g in self.gates:
            out[g.name] = out.get(g.name, 0) + 1
        return out


# --- seeded workload recipes (draw order documented per function) -----------

def layered_rotations(n=16, layers=20, seed=16001):
    """Random layered circuit: per layer, on every qubit q (ascending) draw a
    gate index uniform in {H, RX, RY, RZ} and then an angle U[0, 2pi) (the
    angle is drawn for H too, and ignored, so the stream does not depend on
    the choice); then CX on brickwork pairs: even layers (0,1),(2,3),...,
    odd layers (1,2),(3,4),...; the control is the lower qubit."""
    rng = np.random.default_rng(seed)
    c = Circuit(n)
    for layer in range(layers):
        for q in range(n):
            kind = int(rng.integers(0, 4))
            ang = float(rng.uniform(0.0, 2 * math.pi))
            if kind == 0:
                c.add("H", (q,), g_h())
            elif kind == 1:
                c.add("RX", (q,), g_rx(ang))
            elif kind == 2:
                c.add("RY", (q,), g_ry(ang))
            else:
                c.add("RZ", (q,), g_rz(ang))
        start = layer % 2
        for a in range(start, n - 1, 2):
            c.add("CX", (a, a + 1), g_cx())
    return c


def _random_pairs(rng, n):
    """A seeded random perfect matching: permutation of range(n), paired
    consecutively; floor(n/2) pairs, the first element of each pair first."""
    perm = rng.permutation(n)
    return [(int(perm[2 * i]), int(perm[2 * i + 1])) for i in range(n // 2)]


def random_u3_2q(n=30, depth=40, seed=30002, two="CZ"):
    """Depth-`depth` random circuit: per layer, U3(t, p, l) on every qubit
    (ascending q; t, p, l drawn in that order, each U[0, 2pi)), then the
    two-qubit gate `two` (CZ or CX) on a random perfect matching."""
    rng = np.random.default_rng(seed)
    c = Circuit(n)
    g2 = {"CZ": g_cz, "CX": g_cx}[two]
    for _ in range(depth):
        for q in range(n):
            t, p, l = (float(v) for v in rng.uniform(0.0, 2 * math.pi, size=3))
            c.add("U3", (q,), g_u3(t, p, l))
        for a, b in _random_pairs(rng, n):
            c.add(two, (a, b), g2())
    return c


def random_su4(n=33, depth=60, seed=33005):
    """Per layer, a random perfect matching (odd n leaves one qubit idle),
    then a Haar SU(4) on each pair in matching order."""
    rng = np.random.default_rng(seed)
    c = Circuit(n)
    for _ in range(depth):
        for a, b in _random_pairs(rng, n):
            c.add("SU4", (a, b), g_haar(rng, 4))
    return c


def random_dense(n, ngates, seed, kmax=3, kinds=("dense", "diag", "perm")):
    """Test circuits: gates of 1..kmax qubits on random distinct (unsorted)
    targets; dense = Haar unitary, diag = random phases, perm = X/CX/SWAP."""
    rng = np.random.default_rng(seed)
    c = Circuit(n)
    for _ in range(ngates):
        k = int(rng.integers(1, min(kmax, n) + 1))
        tg = tuple(int(v) for v in rng.choice(n, size=k, replace=False))
        kind = kinds[int(rng.integers(0, len(kinds)))]
        if kind == "dense":
            c.add("U%d" % k, tg, g_haar(rng, 1 << k))
        elif kind == "diag":
            ph = rng.uniform(0, 2 * math.pi, size=1 << k)
            c.add("D%d" % k, tg, np.diag(np.exp(1j * ph)))
        else:
            if k == 1:
                c.add("X", tg, g_x())
            elif k == 2:
                c.add("CX" if rng.integers(0, 2) else "SWAP", tg, g_cx() if rng.integers(0, 2) else g_swap())
            else:
                p = rng.permutation(1 << k)
                c.add("P%d" % k, tg, np.eye(1 << k, dtype=np.complex128)[p])
    return c


def qft(n):
    """Textbook QFT without the final qubit-reversal swaps: for q from the top
    qubit down, H on q then CP(pi / 2^(q-j)) controlled by each lower qubit j.
    n H gates + n(n-1)/2 CP gates (496 at n = 31, the paper's Table II)."""
    c = Circuit(n)
    for q in range(n - 1, -1, -1):
        c.add("H", (q,), g_h())
        for j in range(q - 1, -1, -1):
            c.add("CP", (j, q), g_cp(math.pi / (1 << (q - j))))
    return c


def qaoa_complete(n=31, p=5, seed=31005):
    """QAOA on the complete graph with the paper's Table II gate count: H on
    every qubit, then per layer l RZZ(gamma_l) on every pair (j, k), j < k
    (ascending j, then k), and RX(beta_l) on every qubit: n + p (n(n-1)/2 + n)
    gates (2,511 at n = 31, p = 5).  gamma_l, beta_l ~ U[0, 2pi), drawn gamma
    then beta per layer."""
    rng = np.random.default_rng(seed)
    c = Circuit(n)
    for q in range(n):
        c.add("H", (q,), g_h())
    for _ in range(p):
        gamma, beta = (float(v) for v in rng.uniform(0.0, 2 * math.pi, size=2))
        for j in range(n):
            for k in range(j + 1, n):
                c.add("RZZ", (j, k), g_rzz(gamma))
        for q in range(n):
            c.add("RX", (q,), g_rx(beta))
    return c


def qaoa_complete_angles(p=5, seed=31005):
    """The (gamma_l, beta_l) that qaoa_complete draws."""
    rng = np.random.default_rng(seed)
    return [tuple(float(v) for v in rng.uniform(0.0, 2 * math.pi, size=2)) for _ in range(p)]


def ghz(n):
    """H on qubit 0, then CX(0 -> i) for i = 1..n-1."""
    c = Circuit(n)
    c.add("H", (0,), g_h())
    for i in range(1, n):
        c.add("CX", (0, i), g_cx())
    return c


def worked_example():
    """The 14-gate, 10-qubit circuit of the paper's Fig. 5(a), as listed in
    its artifact appendix: lines "type targets ID".  The raw format carries no
    angle, so RZZ uses theta = ID (the reading that reproduces the printed
    fused-diagonal values)."""
    lines = [("H", (0,), 0), ("H", (1,), 1), ("RZZ", (2, 4), 2), ("RZZ", (5, 7), 3),
             ("H", (8,), 4), ("H", (9,), 5), ("H", (3,), 6), ("H", (6,), 7),
             ("RZZ", (0, 2), 8), ("RZZ", (4, 7), 9), ("H", (9,), 10), ("RZZ", (1, 8), 11),
             ("RZZ", (3, 6), 12), ("H", (5,), 13)]
    c = Circuit(10)
    for name, tg, gid in lines:
        c.add(name, tg, g_h() if name == "H" else g_rzz(float(gid)))
    return c


# --- QAOA MaxCut batch --------------------------------------------------------

def random_3regular(rng, n, max_tries=10000):
    """Random simple 3-regular graph on n (even) vertices by the pairing
    model with rejection: 3n half-edges, random permutation, paired
    consecutively; reject on self-loops or multi-edges.  Edges (u < v),
    sorted."""
    assert n % 2 == 0 and n >= 4
    for _ in range(max_tries):
        stubs = np.repeat(np.arange(n), 3)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        ok = True
        seen = set()
        for u, v in pairs:
            u, v = int(u), int(v)
            if u == v:
                ok = False
                break
            e = (min(u, v), max(u, v))
            if e in seen:
                ok = False
                break
            seen.add(e)
        if ok:
            return sorted(seen)
    raise RuntimeError("no 3-regular graph found")


@dataclass
class QaoaInstance:
    n: int
    edges: list
    gammas: np.ndarray
    betas: np.ndarray

    def circuit(self):
        """H on all qubits, then per layer: the cut phase on every edge
        (diag(1, e^{-i g}, e^{-i g}, 1)) and RX(2 b) on every qubit."""
        c = Circuit(self.n)
        for q in range(self.n):
            c.add("H", (q,), g_h())
        for g, b in zip(self.gammas, self.betas):
            for u, v in self.edges:
                c.add("CUT", (u, v), g_cut_phase(float(g)))
            for q in range(self.n):
                c.add("RX", (q,), g_rx(2.0 * float(b)))
        return c


def qaoa_batch(count=512, p=4, seed=512004, sizes=(10, 12, 14, 16, 18, 20)):
    """`count` MaxCut QAOA instances.  Instance i uses its own generator
    default_rng([seed, i]): n uniform from `sizes` (3-regular graphs need an
    even vertex count), then the graph, then gammas (p values U[0, pi)), then
    betas (p values U[0, pi))."""
    out = []
    for i in range(count):
        rng = np.random.default_rng([seed, i])
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        edges = random_3regular(rng, n)
        gam = rng.uniform(0.0, math.pi, size=p)
        bet = rng.uniform(0.0, math.pi, size=p)
        out.append(QaoaInstance(n, edges, gam, bet))
    return out
