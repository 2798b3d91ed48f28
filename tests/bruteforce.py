"""Independent brute-force constructions used to pin the oracle.

None of these reuse the oracle's gather/scatter index loop:
  - full_unitary builds each gate's 2^n x 2^n matrix as a sum of Kronecker
    products of 2x2 matrix units (textbook tensor-product construction,
    qubit 0 = rightmost factor), then multiplies the matrices;
  - tensor_swap exchanges qubits by swapping axes of the (2,)*n tensor view;
  - pauli_matrix builds Pauli strings by numpy.kron.
"""
from __future__ import annotations

import itertools
import math

import math

import numpy as np

_I2 = np.eye(2, dtype=np.complex128)


def _unit(r, c):
    e = np.zeros((2, 2), dtype=np.complex128)
    e[r, c] = 1.0
    return e


def embed(n, targets, g):
    """Full 2^n x 2^n matrix of gate g on `targets` (targets[0] = MSB of the
    gate's local index): sum over (r, c) of g[r, c] * kron_{q=n-1..0} F_q with
    F_q = |r_j><c_j| if q = targets[j] else I."""
    k = len(targets)
    full = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    pos = {t: j for j, t in enumerate(targets)}
    for r in range(1 << k):
        for c in range(1 << k):
            if g[r, c] == 0:
                continue
            m = np.ones((1, 1), dtype=np.complex128)
            for q in range(n - 1, -1, -1):
                if q in pos:
                    j = pos[q]
                    f = _unit((r >> (k - 1 - j)) & 1, (c >> (k - 1 - j)) & 1)
                else:
                    f = _I2
                m = np.kron(m, f)
            full += g[r, c] * m
    return full


def full_unitary(circuit):
    U = np.eye(1 << circuit.n, dtype=np.complex128)
    for g in circuit.gates:
        U = embed(circuit.n, g.targets, g.matrix) @ U
    return U


def run(circuit):
    e0 = np.zeros(1 << circuit.n, dtype=np.complex128)
    e0[0] = 1
    return full_unitary(circuit) @ e0


def tensor_swap(psi, a, b):
    """Swap qubit pairs (a[j], b[j]) by swapping axes of the (2,)*n tensor,
    axis 0 = qubit n-1."""
    n = int(psi.size).bit_length() - 1
    t = psi.reshape((2,) * n)
    axes = list(range(n))
    for x, y in zip(a, b):
        ax, ay = n - 1 - x, n - 1 - y
        axes[ax], axes[ay] = axes[ay], axes[ax]
    return np.ascontiguousarray(np.transpose(t, axes)).reshape(-1)


_P = {"I": _I2, "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
      "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
      "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128)}


def pauli_letters(n, xmask, zmask):
    out = []
    for q in range(n):
        x, z = (xmask >> q) & 1, (zmask >> q) & 1
        out.append({(0, 0): "I", (1, 0): "X", (0, 1): "Z", (1, 1): "Y"}[(x, z)])
    return out


def pauli_matrix(n, xmask, zmask):
    letters = pauli_letters(n, xmask, zmask)
    m = np.ones((1, 1), dtype=np.complex128)
    for q in range(n - 1, -1, -1):
        m = np.kron(m, _P[letters[q]])
    return m


def maxcut_diag(n, edges):
    z = np.arange(1 << n)
    c = np.zeros(1 << n)
    for u, v in edges:
        c += ((z >> u) ^ (z >> v)) & 1
    return c


def qaoa_bruteforce(n, edges, gammas, betas):
    """|+>^n, e^{-i g C} as a dense diagonal, e^{-i b X} per qubit as a
    kron-embedded 2x2; <C> = psi^dag diag(C) psi."""
    cdiag = maxcut_diag(n, edges)
    psi = np.full(1 << n, 2 ** (-n / 2), dtype=np.complex128)
    for g, b in zip(gammas, betas):
        psi = np.exp(-1j * g * cdiag) * psi
        rx = np.array([[math.cos(b), -1j * math.sin(b)], [-1j * math.sin(b), math.cos(b)]])
        for q in range(n):
            psi = embed(n, (q,), rx) @ psi
    return float(np.real(np.vdot(psi, cdiag * psi)))


def all_pauli_masks(n):
    for x, z in itertools.product(range(1 << n), repeat=2):
        yield x, z


def dicke_amplitudes(n, angles):
    """Amplitude of a basis state of Hamming weight w, for w = 0..n, after H on
    every qubit and p layers of (RZZ(gamma) on every pair, RX(beta) on every
    qubit), computed in the (n+1)-dimensional symmetric (Dicke) subspace:
    H^n gives c_w = sqrt(C(n, w)) 2^{-n/2}; the RZZ layer multiplies c_w by
    exp(-i gamma/2 * ((n - 2w)^2 - n) / 2); the RX layer is exp(-i beta J_x)
    with <D_{w+1}|J_x|D_w> = sqrt((w + 1)(n - w)) / 2; the amplitude is
    c_w / sqrt(C(n, w))."""
    w = np.arange(n + 1)
    binom = np.array([math.comb(n, int(k)) for k in w], dtype=np.float64)
    c = np.sqrt(binom) * 2.0 ** (-n / 2) + 0j
    off = 0.5 * np.sqrt((w[:-1] + 1.0) * (n - w[:-1]))
    Jx = np.diag(off, 1) + np.diag(off, -1)
    lam, V = np.linalg.eigh(Jx)
    S = n - 2 * w
    for gamma, beta in angles:
        c = c * np.exp(-0.5j * gamma * (S * S - n) / 2.0)
        c = V @ (np.exp(-1j * beta * lam) * (V.T @ c))
    return c / np.sqrt(binom)
