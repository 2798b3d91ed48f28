"""The plan cost model on the GPU: the library's FP32 forward, backward and
Adam kernels against the FP64 oracle (oracle/mlp.py), training that lowers
the loss, and the learned planner (qs_fuse with planner=1) -- parity of its
plans with the oracle and its measured gain over the heuristic planner.
"""
from __future__ import annotations

import math
import os
import time

import numpy as np
import pytest

from oracle import mlp
from oracle import sim
from paper_2406_14084_amd import costmodel
from paper_2406_14084_amd import inputs as I
from paper_2406_14084_amd import qs
from tests.gpu_util import TOL_C128, max_abs_diff, need_gpu, say

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


def unflatten(flat):
    """Flat parameter vector (library order) -> oracle dict in FP64."""
    out, at = {}, 0
    for name in mlp.ORDER:
        size = int(np.prod(mlp.SHAPES[name]))
        out[name] = np.asarray(flat[at:at + size], dtype=np.float64).reshape(mlp.SHAPES[name])
        at += size
    assert at == qs.COST_PARAMS
    return out


def flatten(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name in mlp.ORDER])


def features_like(rng, B):
    """Inputs in the range the planner's features take (mostly in [0, 1], some zeros)."""
    X = rng.uniform(0, 1, size=(B, qs.COST_FEATURES))
    X[rng.uniform(size=X.shape) < 0.3] = 0.0
    return X.astype(np.float32)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_gradients_vs_oracle(torch):
    """GPU FP32 gradients of one minibatch (B = 256) against the FP64 chain
    rule: relative L2 error <= 1e-4 per tensor, loss within 1e-5."""
    rng = np.random.default_rng(11)
    m = qs.CostModel(seed=3)
    p0 = m.get_params()
    X = features_like(rng, 256)
    t = rng.normal(2.0, 1.0, size=256).astype(np.float32)
    loss = m.train_step(X, t, lr=1e-3)
    g = m.get_grads()
    ref_loss, ref_g = mlp.backward(unflatten(p0), X.astype(np.float64), t.astype(np.float64))
    say("loss gpu %.8f oracle %.8f" % (loss, ref_loss))
    assert abs(loss - ref_loss) <= 1e-5 * max(1.0, ref_loss)
    G = unflatten(g)
    for name in mlp.ORDER:
        e = rel_l2(G[name], ref_g[name])
        say("grad %s rel L2 %.2e" % (name, e))
        assert e <= 1e-4, name


def test_adam_vs_oracle(torch):
    """Three Adam steps: each GPU update equals the oracle's Adam applied to
    the GPU's own gradients (so the check isolates the optimiser), to FP32
    rounding of the parameters."""
    rng = np.random.default_rng(12)
    m = qs.CostModel(seed=4)
    p = unflatten(m.get_params())
    state = mlp.new_adam_state()
    lr = 3e-3
    for step in range(3):
        X = features_like(rng, 128)
        t = rng.normal(0.0, 1.0, size=128).astype(np.float32)
        m.train_step(X, t, lr=lr, want_loss=False)
        g = unflatten(m.get_grads())
        mlp.adam_step(p, g, state, lr=lr)
        got = m.get_params().astype(np.float64)
        want = flatten(p)
        err = np.abs(got - want)
        tol = 4 * U32 * np.maximum(np.abs(want), lr) + 1e-9
        say("adam step %d max |dp| %.2e" % (step + 1, float(err.max())))
        assert np.all(err <= tol), step
        p = unflatten(got)         # continue from the GPU's rounded parameters


def test_predict_vs_oracle(torch):
    """Forward on 1500 rows (two internal chunks) against the FP64 forward."""
    rng = np.random.default_rng(13)
    m = qs.CostModel(seed=5)
    p = unflatten(m.get_params())
    X = features_like(rng, 1500)
    got = m.predict(X).cpu().numpy().astype(np.float64)
    want, _ = mlp.forward(p, X.astype(np.float64))
    scale = np.maximum(np.abs(want), 1.0)
    say("predict max rel %.2e" % float(np.max(np.abs(got - want) / scale)))
    assert np.all(np.abs(got - want) <= 1e-5 * scale)


def test_training_lowers_loss(torch):
    """A teacher network's outputs are learnable: 600 GPU Adam steps on
    minibatches of 256 cut the held-out loss at least tenfold."""
    rng = np.random.default_rng(14)
    teacher = mlp.init_params(rng)
    X = features_like(rng, 4096)
    y, _ = mlp.forward(teacher, X.astype(np.float64))
    y = (0.3 * y).astype(np.float32)
    Xtr, ytr, Xva, yva = X[:3584], y[:3584], X[3584:], y[3584:]
    m = qs.CostModel(seed=6)
    before = mlp.loss(unflatten(m.get_params()), Xva.astype(np.float64), yva.astype(np.float64))
    Xd = torch.from_numpy(Xtr).cuda()
    yd = torch.from_numpy(ytr).cuda()
    for s in range(600):
        i = (s * 256) % 3584
        m.train_step(Xd[i:i + 256], yd[i:i + 256], lr=1e-3, want_loss=False)
    after = mlp.loss(unflatten(m.get_params()), Xva.astype(np.float64), yva.astype(np.float64))
    say("held-out loss %.4f -> %.4f" % (before, after))
    assert after <= 0.1 * before


def test_train_step_rejects_bad_batch(torch):
    m = qs.CostModel(seed=1)
    X = np.zeros((2000, qs.COST_FEATURES), np.float32)
    with pytest.raises(qs.QSError):
        m.train_step(X, np.zeros(2000, np.float32))


def trained_model():
    if not os.path.exists(costmodel.PARAMS_PATH):
        pytest.skip("no trained cost-model parameters committed")
    return costmodel.load_default()


@pytest.mark.parametrize("n,seed", [(14, 1), (20, 2)])
def test_learned_plans_vs_oracle(torch, n, seed):
    """Whatever plan the learned planner picks, the amplitudes equal the
    oracle's to the complex128 tolerance."""
    model = trained_model()
    c = I.random_su4(n=n, depth=12, seed=seed)
    p = qs.Plan(c, kmax=5, planner=1, cost_model=model)
    s = p.stats()
    say("learned plan", n, {k: s[k] for k in ("planner", "candidates", "chunk_qubits", "reg_qubits", "low_qubits",
                                              "predicted_ms", "predicted_heuristic_ms")})
    assert s["candidates"] > 1 and s["predicted_ms"] > 0 and s["planner"] in (0, 1)
    st = qs.State(n, "c128")
    st.init_zero()
    st.apply_plan(p)
    assert max_abs_diff(st.numpy(), sim.run(c)) <= TOL_C128


def _timed(st, plan, torch):
    st.init_zero()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    st.apply_plan(plan)
    b.record()
    b.synchronize()
    return a.elapsed_time(b)


def test_learned_vs_heuristic_33q(torch):
    """What the trained network gains, on a 33-qubit complex128 circuit
    (128 GiB) of depth 60 with Haar SU(4) gates on random pairs.  Three plans
    of the same circuit: the learned planner's, the heuristic's (fixed
    geometry, also the learned planner's fallback) and the paper's objective
    over the same candidates (fewest passes, Eq. 7).  The learned plan must
    not lose to the heuristic and must beat the pass-count choice; all three
    give the same amplitudes (4096 sampled indices and the norm), and the learned
    plans of the circuit and of its inverse return the state to |0...0>."""
    model = trained_model()
    n = 33
    c = I.random_su4(n=n, depth=60, seed=33005)
    plans = {"heuristic": qs.Plan(c, kmax=5), "learned": qs.Plan(c, kmax=5, planner=1, cost_model=model),
             "passes": qs.Plan(c, kmax=5, planner=3)}
    for k, p in plans.items():
        s = p.stats()
        say("33q %-9s C%d r%d L%d blocks %d swaps %d predicted %.0f ms"
            % (k, s["chunk_qubits"], s["reg_qubits"], s["low_qubits"], s["blocks"], s["swap_passes"], s["predicted_ms"]))
    st = qs.State(n, "c128")
    rng = np.random.default_rng(33)
    idx = torch.from_numpy(rng.integers(0, 1 << n, size=4096)).cuda()
    t, samp = {}, {}
    for k in ("heuristic", "learned", "passes"):
        t[k] = _timed(st, plans[k], torch)
        samp[k] = st.tensor[idx].cpu().numpy()
        norm = st.expect([(0, 0, 1.0)])          # sum of |a|^2 in FP64, no 2^n temporary
        say("33q %-9s %.1f ms  norm-1 %.2e" % (k, t[k], norm - 1))
        assert abs(norm - 1.0) <= 1e-10
    say("33q gain of the learned plan: %.1f %% vs heuristic, %.1f %% vs fewest passes"
        % (100 * (t["heuristic"] - t["learned"]) / t["heuristic"], 100 * (t["passes"] - t["learned"]) / t["passes"]))
    assert max_abs_diff(samp["learned"], samp["heuristic"]) <= TOL_C128
    assert max_abs_diff(samp["passes"], samp["heuristic"]) <= TOL_C128
    assert t["learned"] <= 1.02 * t["heuristic"]
    assert t["learned"] <= 0.95 * t["passes"]
    # every amplitude of the learned plans, in one buffer: the learned plan of the circuit,
    # then the learned plan of its inverse, must return |0...0> (a_0 = 1 with the norm 1
    # leaves at most |norm - |a_0|^2| for all other amplitudes together)
    pinv = qs.Plan(c.inverse(), kmax=5, planner=1, cost_model=model)
    st.init_zero()
    st.apply_plan(plans["learned"])
    st.apply_plan(pinv)
    a0 = complex(st.amplitudes(0, 1)[0])
    norm = st.expect([(0, 0, 1.0)])
    far = np.abs(st.tensor[idx[idx != 0]].cpu().numpy()).max()
    say("33q learned plan then learned inverse: |a0 - 1| %.2e  norm-1 %.2e  max sampled |a| %.2e"
        % (abs(a0 - 1), norm - 1, far))
    assert abs(a0 - 1.0) <= 1e-10 and abs(norm - 1.0) <= 1e-10 and far <= 1e-10


def test_learned_vs_heuristic_c64_30q(torch):
    """complex64 (where the learned search also toggles the matrix cores):
    30-qubit U3 + CX, depth 60.  The learned plan must not lose to the
    heuristic (best of two runs each) and both states agree within the sum of
    their rigorous complex64 bounds."""
    from tests import c64_bounds as B
    from tests.c64_bounds import bound_for
    model = trained_model()
    n = 30
    c = I.random_u3_2q(n=n, depth=60, seed=30064, two="CX")
    ph = qs.Plan(c, kmax=5, dtype="c64")
    pl = qs.Plan(c, kmax=5, dtype="c64", planner=1, cost_model=model)
    s = pl.stats()
    say("c64 30q learned choice C%d r%d L%d planner %d mfma ops %d predicted %.1f ms (heuristic %.1f ms)"
        % (s["chunk_qubits"], s["reg_qubits"], s["low_qubits"], s["planner"], s["ops_mfma"], s["predicted_ms"],
           s["predicted_heuristic_ms"]))
    st = qs.State(n, "c64")
    th = min(_timed(st, ph, torch) for _ in range(2))
    a = st.tensor.to(torch.complex128)
    tl = min(_timed(st, pl, torch) for _ in range(2))
    d = float(torch.linalg.vector_norm(st.tensor.to(torch.complex128) - a).item())
    del a
    say("c64 30q heuristic %.1f ms  learned %.1f ms  gain %.1f %%  ||d||2 %.2e"
        % (th, tl, 100 * (th - tl) / th, d))
    (rh, th_), (rl, tl_) = bound_for(ph), bound_for(pl)
    B.check(d, rh + rl, math.hypot(th_, tl_))
    assert tl <= 1.01 * th
