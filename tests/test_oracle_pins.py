"""Pins for the CPU oracle: values fixed by the paper or by mathematics.

Each check takes the loaded oracle library as an argument so that the same
checks can be run against deliberately broken copies of the oracle (see
test_oracle_mutants.py): a plausible mistake anywhere in the oracle must
make at least one of them fail.
"""
from __future__ import annotations

import math
import os

import numpy as np
import pytest

from oracle import sim
from paper_2406_14084_amd import inputs as I
from tests import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# -- checks (return None or raise AssertionError) ------------------------------

def check_kron_bruteforce(L):
    """Oracle == sum-of-Kronecker-products full unitary on random circuits,
    n <= 7, k <= 3, unsorted targets, dense / diagonal / permutation gates."""
    for n, ng, seed in ((1, 6, 1), (2, 10, 2), (3, 14, 3), (5, 20, 4), (7, 24, 5)):
        c = I.random_dense(n, ng, seed, kmax=min(3, n))
        want = bf.run(c)
        got = sim.run(c, L)
        assert np.max(np.abs(got - want)) <= 1e-12, (n, np.max(np.abs(got - want)))


def check_h_all(L):
    """H on every qubit of |0...0> -> 2^{-n/2} on every basis state."""
    n = 11
    c = I.Circuit(n)
    for q in range(n):
        c.add("H", (q,), I.g_h())
    psi = sim.run(c, L)
    assert np.max(np.abs(psi - 2 ** (-n / 2))) <= 1e-14


def check_ghz(L):
    """H q0, CX 0->i: (|0..0> + |1..1>)/sqrt(2), all else 0."""
    n = 12
    psi = sim.run(I.ghz(n), L)
    want = np.zeros(1 << n, dtype=np.complex128)
    want[0] = want[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(psi - want)) <= 1e-15


def check_x_all(L):
    n = 9
    c = I.Circuit(n)
    for q in range(n):
        c.add("X", (q,), I.g_x())
    psi = sim.run(c, L)
    want = np.zeros(1 << n, dtype=np.complex128)
    want[-1] = 1
    assert np.array_equal(psi, want)


def check_cnot_orientation(L):
    """Eq. 3: the first listed qubit is the control / MSB.  |q1 q0> = |01>
    (index 1) with CX(control 0, target 1) -> |11> (index 3); CX(1, 0) leaves
    it unchanged."""
    psi = np.zeros(4, dtype=np.complex128)
    psi[1] = 1
    sim.apply_gate(psi, (0, 1), I.g_cx(), L)
    assert psi[3] == 1 and np.sum(np.abs(psi)) == 1
    psi = np.zeros(4, dtype=np.complex128)
    psi[1] = 1
    sim.apply_gate(psi, (1, 0), I.g_cx(), L)
    assert psi[1] == 1 and np.sum(np.abs(psi)) == 1


def check_rotation_expectations(L):
    """RY(t)|0>: <Z> = cos t, <X> = sin t, <Y> = 0; RX(t)|0>: <Y> = -sin t."""
    for t in (0.3, 1.7, 4.1):
        psi = np.array([1, 0], dtype=np.complex128)
        sim.apply_gate(psi, (0,), I.g_ry(t), L)
        assert abs(sim.expect_pauli(psi, 0, 1, L).real - math.cos(t)) <= 1e-15
        assert abs(sim.expect_pauli(psi, 1, 0, L).real - math.sin(t)) <= 1e-15
        assert abs(sim.expect_pauli(psi, 1, 1, L)) <= 1e-15
        psi = np.array([1, 0], dtype=np.complex128)
        sim.apply_gate(psi, (0,), I.g_rx(t), L)
        assert abs(sim.expect_pauli(psi, 1, 1, L).real + math.sin(t)) <= 1e-15


def check_norm_and_inverse(L):
    """Norm preserved (1e-13) along the 16-qubit layered circuit; the circuit
    followed by its inverse returns |0...0> (1e-12)."""
    c = I.layered_rotations(n=12, layers=10, seed=7)
    psi = sim.run(c, L)
    assert abs(sim.norm2(psi, L) - 1.0) <= 1e-13
    sim.apply_circuit(psi, c.inverse(), L)
    e0 = np.zeros_like(psi)
    e0[0] = 1
    assert np.max(np.abs(psi - e0)) <= 1e-12


def check_qft_closed_form(L):
    """QFT without final swaps maps |x> to 2^{-n/2} sum_y e^{2 pi i x y / 2^n}
    |bitrev(y)>."""
    n = 7
    N = 1 << n
    for x in (0, 1, 5, 77, 127):
        psi = np.zeros(N, dtype=np.complex128)
        psi[x] = 1
        sim.apply_circuit(psi, I.qft(n), L)
        y = np.arange(N)
        rev = np.array([int(format(v, "0%db" % n)[::-1], 2) for v in y])
        want = np.zeros(N, dtype=np.complex128)
        want[rev] = np.exp(2j * np.pi * x * y / N) / math.sqrt(N)
        assert np.max(np.abs(psi - want)) <= 1e-13, x


def check_swap_tensor(L):
    """Eq. 4 swap == swapping tensor axes (several disjoint pairs)."""
    rng = np.random.default_rng(11)
    n = 8
    for a, b in (((0,), (7,)), ((1, 2), (5, 3)), ((0, 4, 6), (1, 2, 7))):
        psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
        want = bf.tensor_swap(psi, a, b)
        got = psi.copy()
        sim.swap_qubits(got, a, b, L)
        assert np.array_equal(got, want)


def check_pauli_bruteforce(L):
    """<P> == psi^dag (kron of Pauli matrices) psi, all 4^3 strings on 3 qubits
    and random strings on 6."""
    rng = np.random.default_rng(3)
    for n, masks in ((3, list(bf.all_pauli_masks(3))),
                     (6, [(int(rng.integers(64)), int(rng.integers(64))) for _ in range(20)])):
        psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
        psi /= np.linalg.norm(psi)
        for x, z in masks:
            want = np.vdot(psi, bf.pauli_matrix(n, x, z) @ psi)
            got = sim.expect_pauli(psi, x, z, L)
            assert abs(got - want) <= 1e-13, (n, x, z)


def check_probs(L):
    """Closed forms of p_i = |a_i|^2 (Eq. 1): H on every qubit gives 2^-n on
    every basis state; GHZ gives 1/2 at |0..0> and |1..1> and 0 elsewhere;
    a basis state gives a one-hot vector; a state scaled by a phase keeps its
    probabilities; a hand-computed 2-amplitude case (3+4i)/5, 0 -> 1, 0."""
    n = 10
    c = I.Circuit(n)
    for q in range(n):
        c.add("H", (q,), I.g_h())
    p = sim.probs(sim.run(c, L), L)
    assert np.max(np.abs(p - 2.0 ** -n)) <= 1e-15
    assert abs(float(np.sum(p)) - 1.0) <= 1e-13
    p = sim.probs(sim.run(I.ghz(9), L), L)
    want = np.zeros(1 << 9)
    want[0] = want[-1] = 0.5
    assert np.max(np.abs(p - want)) <= 1e-15
    psi = np.zeros(32, dtype=np.complex128)
    psi[13] = 1j
    p = sim.probs(psi, L)
    assert p[13] == 1.0 and np.count_nonzero(p) == 1
    p = sim.probs(np.array([0.6 + 0.8j, 0.0], dtype=np.complex128), L)
    assert abs(p[0] - 1.0) <= 2e-16 and p[1] == 0.0
    rng = np.random.default_rng(5)
    psi = rng.standard_normal(64) + 1j * rng.standard_normal(64)
    ph = np.exp(0.37j)
    assert np.max(np.abs(sim.probs(psi * ph, L) - sim.probs(psi, L))) <= 1e-13


def check_worked_example_d4(L):
    """The artifact appendix prints the first value of the two fused D4
    diagonals of its worked example.  Those blocks hold RZZ with IDs 2, 3, 9
    (first D4) and 12, 8 (second; the text's "7" is the H gate).  Applying the
    same RZZ gates (theta = ID) to |0000> leaves amplitude 0 equal to the D4's
    entry 0, whose real part must match the printed digits."""
    vals = {}
    with open(os.path.join(GOLDEN, "worked_example_d4.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                key, v = line.split()
                vals[key] = float(v)
    for key, gates in (("d4_first", [((0, 2), 2.0), ((1, 3), 3.0), ((0, 3), 9.0)]),
                       ("d4_second", [((1, 3), 12.0), ((0, 2), 8.0)])):
        psi = np.zeros(16, dtype=np.complex128)
        psi[0] = 1
        for tg, th in gates:
            sim.apply_gate(psi, tg, I.g_rzz(th), L)
        assert abs(psi[0].real - vals[key]) <= 2e-16, (key, psi[0].real, vals[key])
        assert np.sum(np.abs(psi[1:])) == 0


def check_qaoa(L):
    """<C> = |E|/2 when gamma = 0 or beta = 0; equals brute force otherwise."""
    rng = np.random.default_rng(9)
    for n in (4, 6, 8):
        edges = I.random_3regular(rng, n)
        g = rng.uniform(0, math.pi, 2)
        b = rng.uniform(0, math.pi, 2)
        for gg, bb in ((np.zeros(2), b), (g, np.zeros(2))):
            v = sim.qaoa_expectation(I.QaoaInstance(n, edges, gg, bb), L)
            assert abs(v - len(edges) / 2) <= 1e-12, (n, v)
        v = sim.qaoa_expectation(I.QaoaInstance(n, edges, g, b), L)
        assert abs(v - bf.qaoa_bruteforce(n, edges, g, b)) <= 1e-12


def check_qaoa_complete_closed_form(L):
    """H^n then RZZ on every pair and RX on every qubit keep the state
    symmetric: the oracle equals the symmetric-subspace closed form."""
    for n, p, seed in ((6, 2, 3), (9, 3, 7)):
        psi = sim.run(I.qaoa_complete(n=n, p=p, seed=seed), L)
        f = bf.dicke_amplitudes(n, I.qaoa_complete_angles(p=p, seed=seed))
        w = np.array([bin(i).count("1") for i in range(1 << n)])
        assert np.max(np.abs(psi - f[w])) <= 1e-13, n


ALL_CHECKS = [check_kron_bruteforce, check_h_all, check_ghz, check_x_all, check_cnot_orientation,
              check_rotation_expectations, check_norm_and_inverse, check_qft_closed_form,
              check_swap_tensor, check_pauli_bruteforce, check_probs, check_worked_example_d4,
              check_qaoa, check_qaoa_complete_closed_form]


@pytest.mark.parametrize("check", ALL_CHECKS, ids=lambda f: f.__name__)
def test_oracle_pin(check, oracle_lib):
    check(oracle_lib)


def test_qft_gate_count_matches_table2():
    """Table II lists 496 gates for 31-qubit QFT = 31 H + 31*30/2 CP."""
    assert len(I.qft(31)) == 496


def test_gate_matrices_unitary():
    rng = np.random.default_rng(1)
    for m in (I.g_h(), I.g_x(), I.g_y(), I.g_z(), I.g_rx(0.4), I.g_ry(1.1), I.g_rz(2.2),
              I.g_u3(0.3, 1.2, 2.5), I.g_cx(), I.g_cz(), I.g_cp(0.7), I.g_swap(), I.g_rzz(1.3),
              I.g_cut_phase(0.9), I.g_haar(rng, 4), I.g_haar(rng, 8)):
        assert np.allclose(m.conj().T @ m, np.eye(m.shape[0]), atol=1e-14)
    h = I.g_haar(rng, 4)
    assert abs(np.linalg.det(h) - 1) <= 1e-13
