"""Pins for the FP64 cost-model reference: central finite differences on
every parameter tensor, and a descent property of the Adam step."""
import numpy as np

from oracle import mlp


def _setup(seed=0, B=16):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(rng)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.uniform(-0.1, 0.1, size=mlp.SHAPES[k])
    X = rng.standard_normal((B, 48))
    t = rng.standard_normal(B)
    return p, X, t


def test_backward_matches_central_differences():
    p, X, t = _setup()
    _, g = mlp.backward(p, X, t)
    rng = np.random.default_rng(1)
    h = 1e-6
    for name in mlp.ORDER:
        flat = p[name].reshape(-1)
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = mlp.loss(p, X, t)
            flat[i] = old - h
            lm = mlp.loss(p, X, t)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, i, fd, an)


def test_adam_reduces_loss():
    p, X, t = _setup(seed=2, B=64)
    st = mlp.new_adam_state()
    l0 = mlp.loss(p, X, t)
    for _ in range(200):
        _, g = mlp.backward(p, X, t)
        mlp.adam_step(p, g, st, lr=1e-3)
    assert mlp.loss(p, X, t) < 0.2 * l0


def test_adam_first_step_is_sign_times_lr():
    """With bias correction, the first Adam step moves each weight by
    lr * g / (|g| + eps'), i.e. about lr in the direction of -sign(g)."""
    p, X, t = _setup(seed=3)
    _, g = mlp.backward(p, X, t)
    before = {k: v.copy() for k, v in p.items()}
    mlp.adam_step(p, g, mlp.new_adam_state(), lr=1e-3)
    d = p["W2"] - before["W2"]
    big = np.abs(g["W2"]) > 1e-4
    assert np.allclose(d[big], -1e-3 * np.sign(g["W2"][big]), rtol=1e-3)
