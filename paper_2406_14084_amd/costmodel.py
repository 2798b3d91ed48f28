"""Plan cost model: timing harvest, GPU training and the stored parameters.

The learned planner (qs_fuse with planner=1) ranks candidate plans by the
sum over their steps of a predicted time.  The model maps a step's 48
features (qs_plan_block_features) to y = ln(picoseconds per amplitude) of
that step; a step then costs 2^n * exp(y) ps.  Training data are the
simulator's own per-step timings (qs_apply_plan_timed) of random circuits at
26-32 qubits, planned over the same geometry grid the learned planner
searches.  Training runs on the GPU in the library's kernels (forward,
backward, Adam: qs_costmodel_train_step); nothing here computes gradients.

    python -m paper_2406_14084_amd.costmodel harvest --out data.npz
    python -m paper_2406_14084_amd.costmodel train --data data.npz --save

The committed parameters (data/costmodel_params.npy, float32, 22913 values,
with data/costmodel_meta.json describing how they were made) are what
load_default() returns.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import inputs as I
from . import qs

_HERE = os.path.dirname(os.path.abspath(__file__))
PARAMS_PATH = os.path.join(_HERE, "data", "costmodel_params.npy")
META_PATH = os.path.join(_HERE, "data", "costmodel_meta.json")

# The grid the learned planner searches (chunk C, register bits r, low bits L,
# fusion width k, matrix cores for complex64, single-qubit gates split or
# whole); the harvest samples plans from the same grid.
GRID_C = (11, 12, 13)
GRID_R = (3, 4, 5)
GRID_L = (3, 4, 5)
GRID_K = (2, 3, 4, 5)


def target_of(ms, n):
    """ln(picoseconds per amplitude) of a step that took ms milliseconds on 2^n amplitudes."""
    return np.log(np.maximum(ms, 1e-6) * 1e9 / float(1 << n))


def suite(n, rng):
    """Random circuit families of the harvest at n qubits (seeded)."""
    s = int(rng.integers(1 << 30))
    return [
        ("u3cz", I.random_u3_2q(n=n, depth=16, seed=s, two="CZ")),
        ("u3cx", I.random_u3_2q(n=n, depth=16, seed=s + 1, two="CX")),
        ("su4", I.random_su4(n=n, depth=16, seed=s + 2)),
        ("layered", I.layered_rotations(n=n, layers=12, seed=s + 3)),
        ("dense3", I.random_dense(n, 12 * n, s + 4, kmax=3)),
        ("dense2", I.random_dense(n, 10 * n, s + 5, kmax=2, kinds=("dense",))),
    ]


def grid(dtype):
    """(C, r, L, k, matrix cores, split) points the planner searches for this dtype."""
    mfs = (True, False) if dtype == "c64" else (True,)
    return [(C, r, L, k, mf, sp) for C in GRID_C for r in GRID_R for L in GRID_L for k in GRID_K for mf in mfs
            for sp in (True, False)]


def grid_options(rng, count, dtype="c128"):
    """count distinct grid points, plus the heuristic default."""
    pts = grid(dtype)
    idx = rng.choice(len(pts), size=min(count, len(pts)), replace=False)
    return [None] + [pts[i] for i in idx]


def opt_name(opt):
    return "heur" if opt is None else "C%dr%dL%dk%d%s%s" % (opt[:4] + ("" if opt[4] else "v", "" if opt[5] else "w"))


def _plan(circ, opt, dtype):
    if opt is None:
        return qs.Plan(circ, kmax=5, dtype=dtype)
    C, r, L, k, mf, sp = opt
    return qs.Plan(circ, kmax=k, dtype=dtype, chunk_qubits=C, reg_qubits=r, low_qubits=L, mfma=mf, split=sp)


def harvest(sizes=(26, 27, 28, 29, 30, 32), opts_per=(8, 8, 8, 6, 5, 2), dtypes=("c128",), seed=2406,
            families=None, log=print):
    """Time every step of sampled plans; returns dict of arrays
    X (rows, 48) float32, y (rows,) float32 and per-row metadata."""
    rng = np.random.default_rng(seed)
    X, y, meta = [], [], []
    for n, cnt in zip(sizes, opts_per):
        for dtype in dtypes:
            st = qs.State(n, dtype)
            st.init_zero()
            for fam, circ in suite(n, rng):
                if families and fam not in families:
                    continue
                for opt in grid_options(rng, cnt, dtype):
                    try:
                        p = _plan(circ, opt, dtype)
                    except qs.QSError:
                        continue
                    f = p.features()
                    st.apply_plan_timed(p)                 # first run: code loading, table upload
                    ms, _ = st.apply_plan_timed(p)
                    ms2, _ = st.apply_plan_timed(p)
                    ms = np.minimum(ms, ms2)
                    X.append(f)
                    y.append(target_of(ms, n).astype(np.float32))
                    tag = "%s/%d/%s/%s" % (fam, n, dtype, opt_name(opt))
                    meta += [tag] * len(ms)
                    log("harvest %-28s steps %3d  total %.2f ms" % (tag, len(ms), float(ms.sum())))
                    p.close()
            st.close()
            del st
    return {"X": np.concatenate(X).astype(np.float32), "y": np.concatenate(y).astype(np.float32),
            "tag": np.array(meta)}


def train(X, y, steps=6000, batch=256, lr=1e-3, seed=0, val_frac=0.15, log=print):
    """Train a fresh model on the GPU; returns (model, report dict)."""
    import torch
    rng = np.random.default_rng(seed)
    N = X.shape[0]
    perm = rng.permutation(N)
    nval = int(N * val_frac)
    va, tr = perm[:nval], perm[nval:]
    Xt = torch.from_numpy(X[tr]).cuda()
    yt = torch.from_numpy(y[tr]).cuda()
    model = qs.CostModel(seed=seed)
    losses = []
    ntr = len(tr)
    t0 = time.time()
    order = torch.randperm(ntr, generator=torch.Generator().manual_seed(seed)).cuda()
    pos = 0
    for s in range(steps):
        if pos + batch > ntr:
            order = torch.randperm(ntr, generator=torch.Generator().manual_seed(seed + s)).cuda()
            pos = 0
        idx = order[pos:pos + batch]
        pos += batch
        cur_lr = lr * (0.1 ** (s / steps))      # exponential decay to lr/10
        want = (s % 200 == 0) or s == steps - 1
        l = model.train_step(Xt[idx].contiguous(), yt[idx].contiguous(), lr=cur_lr, want_loss=want)
        if want:
            losses.append((s, l))
            log("train step %5d  minibatch loss %.5f" % (s, l))
    torch.cuda.synchronize()
    train_s = time.time() - t0
    rep = {"rows": int(N), "train_rows": int(ntr), "val_rows": int(nval), "steps": steps, "batch": batch,
           "lr": lr, "train_seconds": train_s, "losses": losses}
    if nval:
        pv = model.predict(X[va]).cpu().numpy()
        rep["val_mse"] = float(np.mean((pv - y[va]) ** 2))
        rep["val_mean_abs_rel_time_err"] = float(np.mean(np.abs(np.exp(pv - y[va]) - 1)))
    pt = model.predict(X[tr]).cpu().numpy()
    rep["train_mse"] = float(np.mean((pt - y[tr]) ** 2))
    rep["target_var"] = float(np.var(y))
    return model, rep


def save(model, report, out_dir=None):
    pp, mp = PARAMS_PATH, META_PATH
    if out_dir:
        pp, mp = os.path.join(out_dir, os.path.basename(pp)), os.path.join(out_dir, os.path.basename(mp))
    os.makedirs(os.path.dirname(pp), exist_ok=True)
    np.save(pp, model.get_params().astype(np.float32), allow_pickle=False)
    with open(mp, "w") as f:
        json.dump(report, f, indent=1)
    return pp


def load_default(stream=None):
    """A CostModel holding the committed parameters (raises if absent)."""
    if not os.path.exists(PARAMS_PATH):
        raise RuntimeError("no trained cost-model parameters at %s" % PARAMS_PATH)
    p = np.load(PARAMS_PATH, allow_pickle=False)
    m = qs.CostModel(seed=0, stream=stream)
    m.set_params(p)
    return m


def rank_check(model, circ, dtype="c128", log=print):
    """Predicted vs measured time of every grid plan of one circuit
    (a held-out ranking check); returns rows (opt, predicted ms, measured ms)."""
    import torch
    st = qs.State(circ.n, dtype)
    st.init_zero()
    rows = []
    for opt in [None] + grid(dtype):
        try:
            p = _plan(circ, opt, dtype)
        except qs.QSError:
            continue
        f = p.features()
        pred = float(np.sum(np.exp(model.predict(f).cpu().numpy().astype(np.float64))) * (1 << circ.n) * 1e-9)
        st.apply_plan_timed(p)
        ms, _ = st.apply_plan_timed(p)
        rows.append((opt, pred, float(ms.sum())))
        log("rank %-16s predicted %8.2f ms  measured %8.2f ms" % (opt_name(opt), pred, float(ms.sum())))
        p.close()
    torch.cuda.synchronize()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    h = sub.add_parser("harvest")
    h.add_argument("--out", required=True)
    h.add_argument("--quick", action="store_true", help="26-28 qubits only")
    h.add_argument("--c64", action="store_true", help="also time complex64 plans")
    t = sub.add_parser("train")
    t.add_argument("--data", required=True, nargs="+")
    t.add_argument("--steps", type=int, default=6000)
    t.add_argument("--save", action="store_true")
    t.add_argument("--out-dir", default=None, help="write the parameters here instead of the package data folder")
    t.add_argument("--rank-n", type=int, default=0, help="after training, rank all grid plans of a held-out SU(4) circuit")
    t.add_argument("--rank-c64", type=int, default=0,
                   help="after training, rank all complex64 grid plans of a held-out U3+CX circuit of this size")
    a = ap.parse_args(argv)
    say = lambda *x: (print(*x), sys.stdout.flush())
    if a.cmd == "harvest":
        kw = {}
        if a.quick:
            kw = dict(sizes=(26, 27, 28), opts_per=(6, 6, 6))
        if a.c64:
            kw["dtypes"] = ("c128", "c64")
        d = harvest(log=say, **kw)
        np.savez(a.out, **d)
        say("rows", d["X"].shape[0])
    else:
        parts = [np.load(p, allow_pickle=False) for p in a.data]
        X = np.concatenate([p["X"] for p in parts])
        y = np.concatenate([p["y"] for p in parts])
        model, rep = train(X, y, steps=a.steps, log=say)
        rep["data"] = "per-step timings of seeded random circuits at 26-32 qubits (u3cz, u3cx, su4, layered, " \
                      "dense3, dense2), complex128 and complex64, over the planner's candidate grid; " \
                      "target ln(ps per amplitude)"
        say(json.dumps({k: v for k, v in rep.items() if k != "losses"}))
        if a.rank_n:
            rows = rank_check(model, I.random_su4(n=a.rank_n, depth=24, seed=777), log=say)
            best_meas = min(rows, key=lambda r: r[2])
            best_pred = min(rows, key=lambda r: r[1])
            rep["rank_check"] = {"n": a.rank_n, "heuristic_ms": rows[0][2], "best_measured_ms": best_meas[2],
                                 "pick_measured_ms": best_pred[2], "pick": str(best_pred[0])}
            say(json.dumps(rep["rank_check"]))
        if a.rank_c64:
            rows = rank_check(model, I.random_u3_2q(n=a.rank_c64, depth=30, seed=778, two="CX"), dtype="c64", log=say)
            best_meas = min(rows, key=lambda r: r[2])
            best_pred = min(rows, key=lambda r: r[1])
            rep["rank_check_c64"] = {"n": a.rank_c64, "heuristic_ms": rows[0][2], "best_measured_ms": best_meas[2],
                                     "pick_measured_ms": best_pred[2], "pick": str(best_pred[0])}
            say(json.dumps(rep["rank_check_c64"]))
        if a.save:
            say("saved", save(model, rep, a.out_dir))


if __name__ == "__main__":
    main()
