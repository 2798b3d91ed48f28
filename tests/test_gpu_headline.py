"""The paper's headline circuits at 31 qubits on one GPU (Table II): the
textbook QFT (496 gates) and QAOA with p = 5 on the complete graph (2,511
gates), complex128, fused and blocked, checked at full size against
closed forms computed independently of the simulator:

- QFT without the final swaps maps |x> to 2^{-n/2} sum_y e^{2 pi i x y / 2^n}
  |bitrev(y)>: sampled amplitudes, and |a_i|^2 = 2^{-n} for every i;
- QAOA on the complete graph keeps the state symmetric under qubit
  permutations, so amplitude i depends only on w = popcount(i).  In the
  basis of symmetric (Dicke) states the circuit is an (n+1)-dimensional
  problem: H^n gives c_w = sqrt(C(n, w)) 2^{-n/2}; RZZ(gamma) on every pair
  multiplies c_w by exp(-i gamma/2 * ((n - 2w)^2 - n) / 2) (the sum of
  z_j z_k over pairs is (S^2 - n)/2 with S = n - 2w); RX(beta) on every
  qubit is exp(-i beta J_x) with <D_{w+1}|J_x|D_w> = sqrt((w + 1)(n - w)) / 2;
  amplitude i is c_w / sqrt(C(n, w)).

A 14-qubit instance of the QAOA recipe is also compared element by element
with the oracle.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import sim
from paper_2406_14084_amd import inputs as I
from paper_2406_14084_amd import qs
from tests.bruteforce import dicke_amplitudes
from tests.gpu_util import TOL_C128, max_abs_diff, need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


def bitrev(v, n):
    return int(format(v, "0%db" % n)[::-1], 2)


def sample_indices(n, count, seed):
    rng = np.random.default_rng(seed)
    idx = set(int(v) for v in rng.integers(0, 1 << n, size=count, dtype=np.int64))
    idx |= {0, 1, (1 << n) - 1, (1 << n) - 2, 1 << (n - 1), (1 << (n - 1)) - 1}
    return sorted(idx)


def test_qft31_closed_form(torch):
    n = 31
    N = 1 << n
    x = 1234567891 % N
    c = I.qft(n)
    p = qs.Plan(c, kmax=5)
    say("qft31: %d gates, %s" % (len(c), {k: p.stats()[k] for k in ("blocks", "swap_passes")}))
    st = qs.State(n, "c128")
    st.init_basis(x)
    st.apply_plan(p)
    pr = st.probs()
    pmin, pmax = float(pr.min().item()), float(pr.max().item())
    del pr
    say("qft31: |a|^2 in [%.17g, %.17g], 2^-n = %.17g" % (pmin, pmax, 1.0 / N))
    assert abs(pmin - 1.0 / N) <= 1e-12 / math.sqrt(N) and abs(pmax - 1.0 / N) <= 1e-12 / math.sqrt(N)
    worst = 0.0
    for i in sample_indices(n, 4096, 3):
        y = bitrev(i, n)
        ph = 2 * math.pi * ((x * y) % N) / N
        want = complex(math.cos(ph), math.sin(ph)) / math.sqrt(N)
        got = complex(st.tensor[i].item())
        worst = max(worst, abs(got - want))
    say("qft31: max |d amp| over the sample = %.3e" % worst)
    assert worst <= TOL_C128


def test_qaoa_complete_14q_vs_oracle(torch):
    c = I.qaoa_complete(n=14, p=5, seed=14005)
    say("qaoa complete 14q")
    st = qs.State(14, "c128")
    st.init_zero()
    st.apply_plan(qs.Plan(c, kmax=5))
    got = st.numpy()
    want = sim.run(c)
    assert max_abs_diff(got, want) <= TOL_C128
    # the symmetric-subspace closed form agrees with the oracle too
    f = dicke_amplitudes(14, I.qaoa_complete_angles(p=5, seed=14005))
    w = np.array([bin(i).count("1") for i in range(1 << 14)])
    assert np.max(np.abs(want - f[w])) <= 1e-12


def test_qaoa31_symmetric_closed_form(torch):
    n = 31
    c = I.qaoa_complete(n=n, p=5, seed=31005)
    assert len(c) == 2511
    p = qs.Plan(c, kmax=5)
    say("qaoa31: %d gates, %s" % (len(c), {k: p.stats()[k] for k in ("blocks", "swap_passes")}))
    st = qs.State(n, "c128")
    st.init_zero()
    st.apply_plan(p)
    f = dicke_amplitudes(n, I.qaoa_complete_angles(p=5, seed=31005))
    worst = 0.0
    for i in sample_indices(n, 4096, 4):
        got = complex(st.tensor[i].item())
        worst = max(worst, abs(got - f[bin(i).count("1")]))
    norm = st.expect([(0, 0, 1.0)])
    say("qaoa31: max |d amp| over the sample = %.3e, norm - 1 = %.3e" % (worst, norm - 1))
    assert worst <= TOL_C128 and abs(norm - 1.0) <= 1e-11
