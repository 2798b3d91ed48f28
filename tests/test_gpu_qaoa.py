"""Batched QAOA MaxCut: 512 instances (random 3-regular graphs, 10-20 qubits,
p = 4) in one persistent launch, checked instance by instance against the
CPU oracle.

Tolerance for <C> with a complex64 state: the state error is at most
eps = sum over ops (one diagonal cost layer + n RX gates per layer) of the
per-op bounds of test_gpu_c64 plus the rounding of the initial amplitude, and
|<C>' - <C>| <= (2 eps + eps^2) * max_z C(z) <= (2 eps + eps^2) * |E|.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import sim
from paper_2406_14084_amd import inputs as I
from paper_2406_14084_amd import qs
from tests.gpu_util import need_gpu, say
from tests.c64_bounds import EPS_DIAG, U32, eps_dense

pytestmark = pytest.mark.gpu


def tol(inst):
    eps = U32 + len(inst.gammas) * (EPS_DIAG + inst.n * eps_dense(1))
    return (2 * eps + eps * eps) * len(inst.edges)


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


@pytest.fixture(scope="module")
def batch512(torch):
    insts = I.qaoa_batch(count=512, p=4, seed=512004)
    say("qaoa batch create", len(insts))
    b = qs.QaoaBatch(insts, "c64")
    ref = np.array([sim.qaoa_expectation(q) for q in insts])
    return insts, b, ref


def test_batched_vs_oracle(torch, batch512):
    insts, b, ref = batch512
    say("qaoa batched run")
    got = b.run(graph=False).cpu().numpy().copy()
    assert b.error() == 0
    bad = [(i, got[i], ref[i]) for i, q in enumerate(insts) if abs(got[i] - ref[i]) > tol(q)]
    say("max |d<C>| = %.3e" % float(np.max(np.abs(got - ref))))
    assert not bad, bad[:5]


def test_sequential_matches_batched(torch, batch512):
    insts, b, ref = batch512
    say("qaoa sequential run")
    batched = b.run().cpu().numpy().copy()
    seq = b.run_sequential().cpu().numpy().copy()
    assert b.error() == 0
    assert np.max(np.abs(seq - batched)) <= 1e-9
    assert all(abs(seq[i] - ref[i]) <= tol(q) for i, q in enumerate(insts))


def test_graph_replays(torch, batch512):
    """Replay the captured graph several times with eager work in between;
    every replay must equal the eager result."""
    insts, b, ref = batch512
    eager = b.run(graph=False).cpu().numpy().copy()
    for rep in range(4):
        say("qaoa graph replay", rep)
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()           # unrelated eager work between replays
        got = b.run(graph=True).cpu().numpy().copy()
        assert b.error() == 0
        assert np.max(np.abs(got - eager)) <= 1e-9, rep


def test_autotune_keeps_results(torch, batch512):
    insts, b, ref = batch512
    say("qaoa autotune")
    choice, ms = b.autotune()
    assert 0 <= choice < 40 and ms > 0
    got = b.run(graph=True).cpu().numpy().copy()
    assert all(abs(got[i] - ref[i]) <= tol(q) for i, q in enumerate(insts))


def _between_batch(seed=77):
    """Instances on both sides of the two LDS chunk sizes (11-14 qubits; odd sizes
    on a ring with chords, even ones 3-regular)."""
    rng = np.random.default_rng(seed)
    out = []
    for n in (11, 12, 13, 14, 13, 12):
        if n % 2:
            edges = [(i, (i + 1) % n) for i in range(n)] + [(i, (i + n // 2) % n) for i in range(0, n, 3)]
            edges = sorted({(min(u, v), max(u, v)) for u, v in edges})
        else:
            edges = I.random_3regular(rng, n)
        out.append(I.QaoaInstance(n, edges, rng.uniform(0, math.pi, 3), rng.uniform(0, math.pi, 3)))
    return out


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("choice", [6, 26])
def test_each_lds_chunk_size(torch, dtype, choice):
    """Both LDS chunk sizes the autotuner may pick (choice 6: 13 qubits for
    complex64 / 12 for complex128; choice 26: one less; same launch shape and
    grouping): an instance between the two sizes runs whole in LDS under one and
    as chunk tasks in the workspace under the other; every <C> must match the
    oracle either way, and the sequential schedule the batched one."""
    insts = _between_batch()
    ref = np.array([sim.qaoa_expectation(q) for q in insts])
    say("qaoa set_choice", dtype, choice)
    b = qs.QaoaBatch(insts, dtype)
    b.set_choice(choice)
    got = b.run(graph=False).cpu().numpy().copy()
    seq = b.run_sequential().cpu().numpy().copy()
    assert b.error() == 0
    t = (lambda q: tol(q)) if dtype == "c64" else (lambda q: 1e-10)
    assert all(abs(got[i] - ref[i]) <= t(q) for i, q in enumerate(insts)), (got, ref)
    assert np.max(np.abs(seq - got)) <= 1e-9
    b.close()


def test_special_angles(torch):
    """gamma = 0 or beta = 0 leaves <C> = |E|/2 exactly in exact arithmetic."""
    rng = np.random.default_rng(2)
    insts = []
    for n in (10, 14, 18, 20):
        e = I.random_3regular(rng, n)
        insts.append(I.QaoaInstance(n, e, np.zeros(4), rng.uniform(0, math.pi, 4)))
        insts.append(I.QaoaInstance(n, e, rng.uniform(0, math.pi, 4), np.zeros(4)))
    b = qs.QaoaBatch(insts, "c64")
    got = b.run().cpu().numpy()
    for i, q in enumerate(insts):
        assert abs(got[i] - len(q.edges) / 2) <= tol(q), (i, got[i])


def test_complex128_batch(torch):
    insts = I.qaoa_batch(count=24, p=4, seed=7, sizes=(10, 12, 14, 16))
    b = qs.QaoaBatch(insts, "c128")
    got = b.run(graph=True).cpu().numpy()
    ref = np.array([sim.qaoa_expectation(q) for q in insts])
    assert np.max(np.abs(got - ref)) <= 1e-10
