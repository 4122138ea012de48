"""Driver of the learned per-axis closure: training data from fine-grid runs
of the solver, training and evaluation of the network.  Every computation
runs in the library (``chfpe_closure_*``, ``chfpe_set_closure``); this module
only sequences the calls and stacks their host arrays.
"""
from __future__ import annotations

import copy

import numpy as np

from . import (ClosureTrainer, Solver, closure_eval, closure_features, params_from_workload)


def fine_of(w: dict) -> dict:
    """The 2:1 fine grid of a workload (twice the points per axis, same box)."""
    f = copy.deepcopy(w)
    f["Nq"] = [2 * n for n in w["Nq"]]
    f["Np"] = [2 * n for n in w["Np"]]
    return f


def fine_moments(w: dict, n_eq: int, n_prop: int, every: int, dt: float, progress=None):
    """Moments of fine-grid snapshots along the states a 2D response visits:
    W_eq after n_eq steps, then A^x W_eq and B^x of it, each propagated
    n_prop steps with a snapshot every `every` steps.  Returns per axis
    (G_a, b_a) and the (c_a, t_a) array, summed over the snapshots.
    `progress(n)`, if given, is called after each snapshot n."""
    wf = fine_of(w)
    acc = None
    n_snap = 0
    with Solver(params_from_workload(wf, precision=0, batch=1)) as s:
        s.equilibrate(n_eq, dt)

        def add():
            nonlocal acc, n_snap
            G, b, ct = s.closure_moments()
            if acc is None:
                acc = [G, b, ct]
            else:
                acc = [[x + y for x, y in zip(acc[0], G)], [x + y for x, y in zip(acc[1], b)], acc[2] + ct]
            n_snap += 1
            if progress is not None:
                progress(n_snap)

        add()
        for op in ("A", "B"):
            s.perturb(w[op])
            add()
            for _ in range(n_prop // every):
                s.propagate(every, dt)
                add()
    return acc


def save_moments(path: str, mom) -> None:
    """Write one draw's moments (per axis G_a, b_a; the (c, t) array) to .npz."""
    G, b, ct = mom
    arrs = {f"G{a}": np.asarray(G[a]) for a in range(len(G))}
    arrs.update({f"b{a}": np.asarray(b[a]) for a in range(len(b))})
    np.savez(path, ct=np.asarray(ct), **arrs)


def load_moments(path: str):
    """Read moments written by save_moments."""
    z = np.load(path)
    n = len(z["ct"])
    return [z[f"G{a}"] for a in range(n)], [z[f"b{a}"] for a in range(n)], z["ct"]


def training_set(draws):
    """Stack per-draw (workload, moments) into the trainer's arrays: features,
    group starts, G, b and (c, t) with one group per (draw, axis)."""
    feats, gstart, Gs, bs, cts = [], [0], [], [], []
    for w, (G, b, ct) in draws:
        f, _ = closure_features(params_from_workload(w))
        feats.append(f)
        for a in range(len(b)):
            gstart.append(gstart[-1] + len(b[a]))
            Gs.append(np.asarray(G[a]).ravel())
            bs.append(b[a])
            cts.append(ct[a])
    return (np.concatenate(feats), np.array(gstart, dtype=np.int32), np.concatenate(Gs),
            np.concatenate(bs), np.concatenate(cts))


def init_params(seed: int) -> np.ndarray:
    """Seeded initial weights (FP32, 577): W1 ~ N(0, 1/16), small W2, zero biases."""
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.normal(0.0, 0.25, 16 * 32), np.zeros(32), rng.normal(0.0, 0.01, 32),
                           [0.0]]).astype(np.float32)


def entries(prm, w: dict) -> np.ndarray:
    """Closure entries s (FP64, one per row) of the network for workload w."""
    f, _ = closure_features(params_from_workload(w))
    return closure_eval(prm, f).astype(np.float64)


def train(data, steps: int, lr: float, seed: int = 0, schedule=(1.0, 0.3, 0.1)):
    """Train from the stacked data; the step count is split evenly over the
    learning-rate factors of `schedule`.  Returns (trainer, loss history)."""
    tr = ClosureTrainer(init_params(seed))
    feat, gstart, G, b, ct = data
    hist = []
    per = max(1, steps // len(schedule))
    for fct in schedule:
        hist.append(tr.train(feat, gstart, G, b, ct, per, lr * fct))
    return tr, np.concatenate(hist)
