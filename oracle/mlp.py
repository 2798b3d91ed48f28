"""FP64 numpy reference for the plan cost model -- TEST INFRASTRUCTURE.

The paper has no learned component; its planner minimises the number of gate
blocks (Sec. IV, Eq. 7).  The cost model replaces that count by a predicted
time.  This file is the plain definition of the network and its training
step, against which the GPU kernels are checked:

  h1 = relu(X W1^T + b1)      X: (B, 48)   W1: (128, 48)  b1: (128,)
  h2 = relu(h1 W2^T + b2)                  W2: (128, 128) b2: (128,)
  y  = h2 W3^T + b3                        W3: (1, 128)   b3: (1,)
  L  = (1/B) sum_b (y_b - t_b)^2

Backward is the chain rule written out; relu'(0) is taken as 0.  Adam
(Kingma & Ba, 2015) with bias correction:
  m <- b1 m + (1-b1) g ; v <- b2 v + (1-b2) g^2
  w <- w - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)

Parity unpinned against the paper (it has none); pinned by central finite
differences in the tests.
"""
from __future__ import annotations

import numpy as np

SHAPES = {"W1": (128, 48), "b1": (128,), "W2": (128, 128), "b2": (128,), "W3": (1, 128), "b3": (1,)}
ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def init_params(rng: np.random.Generator):
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases."""
    p = {}
    for name in ORDER:
        shp = SHAPES[name]
        if name.startswith("W"):
            bound = np.sqrt(6.0 / shp[1])
            p[name] = rng.uniform(-bound, bound, size=shp)
        else:
            p[name] = np.zeros(shp)
    return p


def forward(p, X):
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["W3"].T + p["b3"]
    return y[:, 0], (X, z1, h1, z2, h2)


def loss(p, X, t):
    y, _ = forward(p, X)
    return float(np.mean((y - t) ** 2))


def backward(p, X, t):
    """Returns (loss, grads dict)."""
    y, (X, z1, h1, z2, h2) = forward(p, X)
    B = X.shape[0]
    dy = (2.0 / B) * (y - t)                # (B,)
    g = {}
    g["W3"] = dy[None, :] @ h2              # (1,128)
    g["b3"] = np.array([dy.sum()])
    dh2 = dy[:, None] @ p["W3"]             # (B,128)
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return float(np.mean((y - t) ** 2)), g


def adam_step(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In place on p and state ({'t': int, 'm': {...}, 'v': {...}})."""
    state["t"] += 1
    t = state["t"]
    for name in ORDER:
        m = state["m"].setdefault(name, np.zeros(SHAPES[name]))
        v = state["v"].setdefault(name, np.zeros(SHAPES[name]))
        m[...] = b1 * m + (1 - b1) * g[name]
        v[...] = b2 * v + (1 - b2) * g[name] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[name] = p[name] - lr * mh / (np.sqrt(vh) + eps)


def new_adam_state():
    return {"t": 0, "m": {}, "v": {}}
