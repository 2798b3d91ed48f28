"""ctypes wrapper around the plain C oracle (oracle.c) -- TEST INFRASTRUCTURE.

Complex128 state vectors are numpy arrays; the C code sees them as
interleaved (re, im) doubles.  See oracle.c for the conventions (Eq. 1-4).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib(path: str | None = None):
    """Load liboracle.so (built on first use if absent)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or _build.LIB
    if not os.path.exists(p):
        _build.build(force=True)
    L = C.CDLL(p)
    dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
    L.or_apply_gate.argtypes = [dp, C.c_int, C.c_int, ip, dp]
    L.or_apply_gate.restype = C.c_int
    L.or_apply_circuit.argtypes = [dp, C.c_int, C.c_int, ip, ip, dp]
    L.or_apply_circuit.restype = C.c_int
    L.or_init_zero.argtypes = [dp, C.c_int]
    L.or_swap_qubits.argtypes = [dp, C.c_int, C.c_int, ip, ip]
    L.or_swap_qubits.restype = C.c_int
    L.or_probs.argtypes = [dp, C.c_int, dp]
    L.or_expect_pauli.argtypes = [dp, C.c_int, C.c_ulonglong, C.c_ulonglong, dp, dp]
    L.or_norm2.argtypes = [dp, C.c_int]
    L.or_norm2.restype = C.c_double
    L.or_qaoa_cost_phase.argtypes = [dp, C.c_int, C.c_int, ip, C.c_double]
    L.or_maxcut_expect.argtypes = [dp, C.c_int, C.c_int, ip]
    L.or_maxcut_expect.restype = C.c_double
    L.or_num_threads.restype = C.c_int
    if path is None:
        _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def zero_state(n: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().or_init_zero(_dp(psi.view(np.float64)), n)
    return psi


def apply_gate(psi: np.ndarray, targets, matrix, L=None) -> None:
    """In place: one gate, Eq. 2 / Eq. 3 (first target = MSB of local index)."""
    L = L or lib()
    n = int(psi.size).bit_length() - 1
    t = np.ascontiguousarray(targets, dtype=np.int32)
    m = np.ascontiguousarray(matrix, dtype=np.complex128)
    rc = L.or_apply_gate(_dp(psi.view(np.float64)), n, len(t), _ip(t), _dp(m.view(np.float64)))
    if rc:
        raise ValueError("oracle rejected gate %r" % (tuple(targets),))


def apply_circuit(psi: np.ndarray, circuit, L=None) -> None:
    """In place: the circuit's gates one by one, in order."""
    L = L or lib()
    k, t, m = circuit.arrays()
    rc = L.or_apply_circuit(_dp(psi.view(np.float64)), circuit.n, len(k), _ip(k), _ip(t), _dp(m))
    if rc:
        raise ValueError("oracle rejected circuit")


def run(circuit, L=None) -> np.ndarray:
    """|0...0> then the circuit."""
    psi = zero_state(circuit.n) if L is None else None
    if psi is None:
        psi = np.empty(1 << circuit.n, dtype=np.complex128)
        L.or_init_zero(_dp(psi.view(np.float64)), circuit.n)
    apply_circuit(psi, circuit, L)
    return psi


def swap_qubits(psi: np.ndarray, a, b, L=None) -> None:
    """In place: Eq. 4 bit exchange a[j] <-> b[j]."""
    L = L or lib()
    n = int(psi.size).bit_length() - 1
    a = np.ascontiguousarray(a, dtype=np.int32)
    b = np.ascontiguousarray(b, dtype=np.int32)
    rc = L.or_swap_qubits(_dp(psi.view(np.float64)), n, len(a), _ip(a), _ip(b))
    if rc:
        raise ValueError("oracle rejected swap")


def probs(psi: np.ndarray, L=None) -> np.ndarray:
    L = L or lib()
    n = int(psi.size).bit_length() - 1
    p = np.empty(psi.size, dtype=np.float64)
    L.or_probs(_dp(np.ascontiguousarray(psi).view(np.float64)), n, _dp(p))
    return p


def expect_pauli(psi: np.ndarray, xmask: int, zmask: int, L=None) -> complex:
    """<P> for the Pauli string with letters (x_q, z_q): 00=I 10=X 01=Z 11=Y."""
    L = L or lib()
    n = int(psi.size).bit_length() - 1
    re, im = C.c_double(), C.c_double()
    L.or_expect_pauli(_dp(np.ascontiguousarray(psi).view(np.float64)), n, xmask, zmask,
                      C.byref(re), C.byref(im))
    return complex(re.value, im.value)


def expect(psi: np.ndarray, terms, L=None) -> float:
    """sum_t coeff_t * Re <P_t> over (xmask, zmask, coeff) terms."""
    return float(sum(c * expect_pauli(psi, x, z, L).real for x, z, c in terms))


def norm2(psi: np.ndarray, L=None) -> float:
    L = L or lib()
    n = int(psi.size).bit_length() - 1
    return float(L.or_norm2(_dp(np.ascontiguousarray(psi).view(np.float64)), n))


def qaoa_expectation(inst, L=None) -> float:
    """QAOA MaxCut <C> by its definition: |+>^n, then for each layer
    a_z <- e^{-i gamma C(z)} a_z followed by RX(2 beta) on every qubit;
    <C> = sum_z |a_z|^2 C(z).  RX(t) = [[cos t/2, -i sin t/2], [-i sin t/2, cos t/2]]
    is written out here on its own (not taken from the shared generator)."""
    L = L or lib()
    n = inst.n
    psi = np.full(1 << n, 2.0 ** (-n / 2), dtype=np.complex128)
    e = np.ascontiguousarray(np.array(inst.edges, dtype=np.int32).reshape(-1))
    for g, b in zip(inst.gammas, inst.betas):
        L.or_qaoa_cost_phase(_dp(psi.view(np.float64)), n, len(inst.edges), _ip(e), float(g))
        c, s = np.cos(b), np.sin(b)  # RX(2b): half angle b
        rx = np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)
        for q in range(n):
            apply_gate(psi, (q,), rx, L)
    return float(L.or_maxcut_expect(_dp(psi.view(np.float64)), n, len(inst.edges), _ip(e)))


def num_threads(L=None) -> int:
    return int((L or lib()).or_num_threads())
