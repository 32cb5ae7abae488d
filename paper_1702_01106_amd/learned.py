"""Training set-up of the learned initial guess (argument marshalling and
bookkeeping only; every pair, gradient and update is computed by libgrim).

Pairs come from the plain FP64 solver on training seeds; the input and output
normalisation are the pairs' mean / standard deviation (computed by libgrim);
the weights start from a seeded He initialisation; training is Adam on the
GPU.
"""
from __future__ import annotations

import numpy as np

from . import grim
from . import workloads as W

N_USED = {8: 5, 10: 7}


def collect(wl: dict, seeds, steps: int, stride: int, cap: int):
    """(X, T) device tensors of training pairs from FP64 runs of wl on seeds."""
    import torch

    X = torch.empty((cap, grim.MLP_IN), dtype=torch.float32, device="cuda")
    T = torch.empty((cap, grim.MLP_OUT), dtype=torch.float32, device="cuda")
    n = 0
    for seed in seeds:
        ctx = grim.Context(dict(wl, guess="pn"))
        P0 = W.initial_state(wl, seed=seed)
        ctx.set_prims(P0)
        dt = ctx.cfl_dt(wl["cfl"])
        got = grim.grim_collect_pairs(ctx.ctx, dt, steps, stride, X[n:], T[n:], cap - n)
        ctx.close()
        n += got
        if n >= cap:
            break
    return X[:n], T[:n]


def normalisation(ctx, X, T, n_used: int):
    """Input mean and 1/std (0 for constant inputs); output std, 0 for an
    output that is constant over the pairs (for example the third velocity
    of a 2-D run) or unused, which holds that output at exactly zero.
    Computed by libgrim (grim_mlp_normalisation)."""
    return grim.grim_mlp_normalisation(ctx.ctx, X, T, X.shape[0], n_used)


def he_init(seed: int, x_mean, x_istd, y_scale):
    rng = np.random.default_rng(seed)
    parts = [
        rng.normal(0.0, np.sqrt(2.0 / grim.MLP_IN), (grim.MLP_IN, grim.MLP_HIDDEN)).ravel(),
        np.zeros(grim.MLP_HIDDEN),
        rng.normal(0.0, np.sqrt(2.0 / grim.MLP_HIDDEN), (grim.MLP_HIDDEN, grim.MLP_HIDDEN)).ravel(),
        np.zeros(grim.MLP_HIDDEN),
        rng.normal(0.0, np.sqrt(1.0 / grim.MLP_HIDDEN), (grim.MLP_HIDDEN, grim.MLP_OUT)).ravel(),
        np.zeros(grim.MLP_OUT),
        np.asarray(x_mean, dtype=np.float64), np.asarray(x_istd, dtype=np.float64),
        np.asarray(y_scale, dtype=np.float64),
    ]
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == grim.MLP_PARAMS
    return w


def train_guess(wl: dict, seeds=(1, 2, 3, 4), steps: int = None, pairs: int = 1_000_000, epochs: int = 8,
                batch: int = 4096, lr: float = 2e-3, init_seed: int = 0):
    """Collect ~`pairs` training pairs from FP64 runs on `seeds` and train the
    network on the GPU.  Returns (weights, info)."""
    steps = wl["steps"] if steps is None else steps
    zones = int(np.prod(wl["n"]))
    candidates = len(seeds) * steps * 2 * zones
    stride = max(1, candidates // pairs)
    X, T = collect(wl, seeds, steps, stride, pairs)
    n_used = N_USED[wl["nvar"]]
    ctx = grim.Context(dict(wl, guess="pn"))
    xm, xs, ys = normalisation(ctx, X, T, n_used)
    w0 = he_init(init_seed, xm, xs, ys)
    grim.grim_mlp_set_weights(ctx.ctx, w0)
    hist = grim.grim_mlp_train(ctx.ctx, X, T, X.shape[0], epochs, batch, n_used, lr=lr, seed=init_seed)
    w = grim.grim_mlp_get_weights(ctx.ctx)
    ctx.close()
    return w, {"pairs": int(X.shape[0]), "stride": stride, "loss": [float(v) for v in hist], "n_used": n_used}
