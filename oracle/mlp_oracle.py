"""Plain FP64 numpy oracle of the learned-guess network (test infrastructure only).

Network: x (32) -> normalise -> 128 -> GELU -> 128 -> GELU -> 16 -> scale.
    xh = (x - x_mean) * x_istd
    z1 = xh W1 + b1,  h1 = gelu(z1)
    z2 = h1 W2 + b2,  h2 = gelu(z2)
    y  = (h2 W3 + b3) * y_scale
GELU is the exact form 0.5 z (1 + erf(z / sqrt(2))).  Parameters are one flat
float vector in the order W1 [32][128], b1, W2 [128][128], b2, W3 [128][16],
b3, x_mean [32], x_istd [32], y_scale [16] (22880 values).  Training changes
only W and b.

`forward(..., bf16=True)` rounds the normalised input, the weights and both
hidden activations to bfloat16 (round to nearest even), as the GPU inference
does, and keeps everything else in FP64.
"""
from __future__ import annotations

import math

import numpy as np

D_IN, HID, D_OUT = 32, 128, 16
SHAPES = [("W1", (D_IN, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (HID, D_OUT)),
          ("b3", (D_OUT,)), ("x_mean", (D_IN,)), ("x_istd", (D_IN,)), ("y_scale", (D_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
TRAINABLE = ("W1", "b1", "W2", "b2", "W3", "b3")


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == N_PARAMS
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(a):
    """Round to bfloat16 (nearest even) and return as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


_erf = np.vectorize(math.erf)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(theta, X, bf16_inference: bool = False, keep: bool = False):
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    r = bf16 if bf16_inference else (lambda a: a)
    xh = r((X - p["x_mean"]) * p["x_istd"])
    z1 = xh @ r(p["W1"]) + p["b1"]
    h1 = r(gelu(z1))
    z2 = h1 @ r(p["W2"]) + p["b2"]
    h2 = r(gelu(z2))
    o = h2 @ r(p["W3"]) + p["b3"]
    y = o * p["y_scale"]
    if keep:
        return y, dict(xh=xh, z1=z1, h1=h1, z2=z2, h2=h2)
    return y


def backward(theta, X, dY):
    """Gradient of sum(dY * y) with respect to every parameter (flat vector;
    zero for the fixed normalisation entries)."""
    p = unpack(theta)
    y, c = forward(theta, X, keep=True)
    do = np.asarray(dY, dtype=np.float64) * p["y_scale"]
    g = {name: np.zeros(shape) for name, shape in SHAPES}
    g["W3"] = c["h2"].T @ do
    g["b3"] = do.sum(axis=0)
    dz2 = (do @ p["W3"].T) * gelu_grad(c["z2"])
    g["W2"] = c["h1"].T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"].T) * gelu_grad(c["z1"])
    g["W1"] = c["xh"].T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


def _inv(ys):
    """1 / y_scale, with 0 for outputs whose scale is 0 (held at zero, no loss)."""
    ys = np.asarray(ys, dtype=np.float64)
    return np.where(ys != 0.0, 1.0 / np.where(ys != 0.0, ys, 1.0), 0.0)


def mse_loss(theta, X, T, n_used: int):
    """Mean over rows and the first n_used outputs of ((y - t) / y_scale)^2;
    outputs with y_scale 0 contribute 0 (they still count in the mean)."""
    iys = _inv(unpack(theta)["y_scale"])
    y = forward(theta, X)
    d = ((y - T) * iys)[:, :n_used]
    return float(np.mean(d * d))


def mse_grad(theta, X, T, n_used: int):
    iys = _inv(unpack(theta)["y_scale"])
    y = forward(theta, X)
    dY = np.zeros_like(y)
    dY[:, :n_used] = 2.0 * ((y - T) * iys * iys)[:, :n_used] / (y.shape[0] * n_used)
    return backward(theta, X, dY)


def init_params(seed: int = 0, x_mean=None, x_istd=None, y_scale=None):
    """He-style initialisation (seeded) with the given normalisation."""
    rng = np.random.default_rng(seed)
    p = {}
    p["W1"] = rng.normal(0.0, math.sqrt(2.0 / D_IN), (D_IN, HID))
    p["b1"] = np.zeros(HID)
    p["W2"] = rng.normal(0.0, math.sqrt(2.0 / HID), (HID, HID))
    p["b2"] = np.zeros(HID)
    p["W3"] = rng.normal(0.0, math.sqrt(1.0 / HID), (HID, D_OUT))
    p["b3"] = np.zeros(D_OUT)
    p["x_mean"] = np.zeros(D_IN) if x_mean is None else np.asarray(x_mean, dtype=np.float64)
    p["x_istd"] = np.ones(D_IN) if x_istd is None else np.asarray(x_istd, dtype=np.float64)
    p["y_scale"] = np.ones(D_OUT) if y_scale is None else np.asarray(y_scale, dtype=np.float64)
    return pack(p)
