"""complex64 path: FP32 state, matrices composed in FP64 and rounded once,
FP64 readouts.  Parity is stated per result as the measured ||delta psi||_2
(and max |delta amp|, 1 - fidelity where the reference state is at hand)
against two figures from tests/c64_bounds.py: a rigorous first-order bound
(asserted) and a typical estimate from the probabilistic rounding model
(asserted with a stated multiple, c64_bounds.TYPICAL_MULTIPLE).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import sim
from paper_2406_14084_amd import inputs as I
from paper_2406_14084_amd import qs
from tests import c64_bounds as B
from tests.c64_bounds import bound_for
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


@pytest.mark.parametrize("n,seed,kmax", [(12, 1, 3), (16, 2, 4), (18, 3, 5)])
def test_c64_random_vs_oracle(torch, n, seed, kmax):
    c = I.random_dense(n, 120, seed, kmax=3)
    say("c64 random", n, seed)
    st = qs.State(n, "c64")
    st.init_zero()
    p = qs.Plan(c, kmax=kmax, dtype="c64")
    st.apply_plan(p)
    got = st.numpy().astype(np.complex128)
    want = sim.run(c)
    d2 = float(np.linalg.norm(got - want))
    rig, typ = bound_for(p)
    say("||d||2 = %.3e  max|d| = %.3e  bound %.3e (typical %.3e)" % (d2, np.max(np.abs(got - want)), rig, typ))
    B.check(d2, rig, typ)


def test_c64_u3_cz_20q_half_buffer_vs_oracle(torch):
    """complex64 U3 + CZ: blocks of shear rotations and diagonals whose
    exchanges run in two rounds through half the LDS buffer (every block of
    this plan), within the rigorous bound of the oracle."""
    c = I.random_u3_2q(n=20, depth=20, seed=2020)
    say("c64 u3cz20 half-buffer")
    st = qs.State(20, "c64")
    st.init_zero()
    p = qs.Plan(c, kmax=5, dtype="c64")
    w, offs, R, C, mats = p.program()
    assert sum(1 for o in offs if int(w[o + 3]) & 4) == p.stats()["blocks"] > 0
    st.apply_plan(p)
    got = st.numpy().astype(np.complex128)
    d2 = float(np.linalg.norm(got - sim.run(c)))
    rig, typ = bound_for(p)
    say("||d||2 = %.3e  bound %.3e (typical %.3e)" % (d2, rig, typ))
    B.check(d2, rig, typ)


def test_c64_u3_cx_20q_vs_oracle(torch):
    """The 32-qubit U3 + CX recipe at 20 qubits, full depth 60."""
    c = I.random_u3_2q(n=20, depth=60, seed=20003, two="CX")
    say("c64 u3cx20")
    st = qs.State(20, "c64")
    st.init_zero()
    p = qs.Plan(c, kmax=5, dtype="c64")
    st.apply_plan(p)
    got = st.numpy().astype(np.complex128)
    want = sim.run(c)
    d2 = float(np.linalg.norm(got - want))
    rig, typ = bound_for(p)
    fid = abs(np.vdot(want, got)) ** 2 / np.vdot(got, got).real
    say("||d||2 = %.3e  max|d| = %.3e  1-F = %.3e  bound %.3e (typical %.3e)"
        % (d2, np.max(np.abs(got - want)), 1 - fid, rig, typ))
    B.check(d2, rig, typ)
    assert 1 - fid <= rig ** 2 + 1e-12


def test_c64_gbg_vs_oracle(torch):
    c = I.random_dense(14, 40, 9, kmax=5)
    st = qs.State(14, "c64")
    st.init_zero()
    st.apply_circuit_gbg(c)
    got = st.numpy().astype(np.complex128)
    want = sim.run(c)
    rig, typ = B.bound_gbg(c)
    d2 = float(np.linalg.norm(got - want))
    say("gbg c64: ||d||2 = %.3e bound %.3e (typical %.3e)" % (d2, rig, typ))
    B.check(d2, rig, typ)


def test_c64_swap_exact(torch):
    n = 16
    rng = np.random.default_rng(4)
    psi = (rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)).astype(np.complex64)
    st = qs.State(n, "c64")
    st.tensor.copy_(torch.from_numpy(psi))
    st.swap_qubits((0, 3, 5), (15, 9, 12))
    want = psi.astype(np.complex128)
    sim.swap_qubits(want, (0, 3, 5), (15, 9, 12))
    assert np.array_equal(st.numpy().astype(np.complex128), want)


def test_c64_vs_c128_32q(torch):
    """Full size: the 32-qubit depth-60 U3 + CX circuit in complex64 (32 GiB)
    against the same plan run in complex128 on the GPU (64 GiB); the
    difference must stay inside the complex64 bound (the complex128 run is
    itself within 1e-12 of exact by the complex128 parity tests)."""
    n = 32
    c = I.random_u3_2q(n=n, depth=60, seed=32003, two="CX")
    say("c64 vs c128 32q")
    s32 = qs.State(n, "c64")
    s32.init_zero()
    p32 = qs.Plan(c, kmax=5, dtype="c64")
    s32.apply_plan(p32)
    s64 = qs.State(n, "c128")
    s64.init_zero()
    s64.apply_plan(qs.Plan(c, kmax=5))
    # chunked comparison to bound memory
    d2 = 0.0
    dmax = 0.0
    ov = 0.0 + 0.0j
    nrm = 0.0
    step = 1 << 28
    for i in range(0, 1 << n, step):
        a = s32.tensor[i:i + step].to(torch.complex128)
        b = s64.tensor[i:i + step]
        diff = (a - b).abs()
        d2 += float((diff ** 2).sum().item())
        dmax = max(dmax, float(diff.max().item()))
        ov += complex(torch.vdot(b, a).item())
        nrm += float((a.abs() ** 2).sum().item())
    d2 = math.sqrt(d2)
    fid = abs(ov) ** 2 / nrm
    rig, typ = bound_for(p32)
    say("32q: ||d||2 = %.3e max|d| = %.3e 1-F = %.3e bound %.3e typical %.3e" % (d2, dmax, 1 - fid, rig, typ))
    B.check(d2, rig, typ)


@pytest.mark.parametrize("n,seed,chunk", [(14, 21, 0), (18, 22, 11), (20, 23, 12)])
def test_c64_matrix_core_ops_vs_oracle(torch, n, seed, chunk):
    """Dense ops of 4-5 qubits on the matrix cores (FP32 products, FP32
    accumulation): within the same rigorous bound as the vector path (the
    inner-product bound holds for any summation order), and close to the
    vector-FMA run of the same circuit."""
    rng = np.random.default_rng(seed)
    c = I.random_dense(n, 100, seed, kmax=3)
    for _ in range(12):
        tg = tuple(int(x) for x in rng.choice(n, 5, replace=False))
        c.add("U5", tg, I.g_haar(rng, 32))
    want = sim.run(c)
    out = {}
    for mf in (True, False):
        p = qs.Plan(c, kmax=5, dtype="c64", chunk_qubits=chunk, mfma=mf)
        assert (p.stats()["ops_mfma"] > 0) == mf
        st = qs.State(n, "c64")
        st.init_zero()
        st.apply_plan(p)
        got = st.numpy().astype(np.complex128)
        d2 = float(np.linalg.norm(got - want))
        rig, typ = bound_for(p)
        say("mfma=%s n=%d ||d||2 = %.3e bound %.3e (typical %.3e) mfma ops %d"
            % (mf, n, d2, rig, typ, p.stats()["ops_mfma"]))
        B.check(d2, rig, typ)
        out[mf] = (got, rig)
    assert float(np.linalg.norm(out[True][0] - out[False][0])) <= out[True][1] + out[False][1]


def test_c64_max_size_34q_inverse(torch):
    """Largest supported state (34 qubits, complex64: 128 GiB): a U3 + CX
    circuit and its inverse, fused and blocked, return |0...0> within the
    rigorous bound of both plans (indices above 2^32 exercise 64-bit
    offsets in every kernel on the path)."""
    n = 34
    c = I.random_u3_2q(n=n, depth=4, seed=34004, two="CX")
    say("c64 34q inverse")
    st = qs.State(n, "c64")
    st.init_zero()
    p1 = qs.Plan(c, kmax=5, dtype="c64")
    p2 = qs.Plan(c.inverse(), kmax=5, dtype="c64")
    st.apply_plan(p1)
    st.apply_plan(p2)
    (r1, t1), (r2, t2) = bound_for(p1), bound_for(p2)
    rig, typ = r1 + r2, math.hypot(t1, t2)
    a0 = complex(st.tensor[0].item())
    norm = st.expect([(0, 0, 1.0)])
    # ||psi - e0||^2 = norm - 2 Re a0 + 1, accumulated in FP64 on the GPU
    d2 = math.sqrt(max(0.0, norm - 2 * a0.real + 1.0))
    say("34q: |a0 - 1| = %.3e  ||psi - e0|| = %.3e  bound %.3e (typical %.3e)" % (abs(a0 - 1), d2, rig, typ))
    assert abs(a0 - 1) <= rig and d2 <= rig + 1e-6
    # the FP64 norm is accumulated from FP32 amplitudes: ||psi - e0|| computed as
    # sqrt(norm - 2 Re a0 + 1) carries an absolute error of about sqrt(2^34 u^2)
    B.check(abs(a0 - 1), rig, typ)
