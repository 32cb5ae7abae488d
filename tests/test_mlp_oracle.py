"""Pins of the FP64 MLP oracle: GELU special values, the forward map on
hand-built weights, gradients against central differences of the loss, and
the bfloat16 rounding against its definition."""
import math

import numpy as np

from oracle import mlp_oracle as M


def test_gelu_values():
    z = np.array([0.0, 1.0, -1.0, 6.0, -6.0])
    g = M.gelu(z)
    # 0.5 z (1 + erf(z/sqrt 2)): Phi(1) = 0.841344746...
    assert g[0] == 0.0
    assert abs(g[1] - 0.8413447460685429) < 1e-15
    assert abs(g[2] + 0.15865525393145707) < 1e-15
    assert abs(g[3] - 6.0) < 1e-8 and abs(g[4]) < 1e-8
    h = 1e-6
    for x in (-2.0, -0.3, 0.0, 0.7, 3.0):
        fd = (M.gelu(np.array(x + h)) - M.gelu(np.array(x - h))) / (2 * h)
        assert abs(fd - M.gelu_grad(np.array(x))) < 1e-9


def test_forward_on_hand_built_weights():
    """One path x0 -> hidden 0 -> hidden 0 -> output 0 with unit weights:
    y0 = s * gelu(gelu(a x0 + b1) + b2) + b3 * s."""
    p = M.unpack(M.init_params(0))
    for k in ("W1", "W2", "W3", "b1", "b2", "b3"):
        p[k] = np.zeros_like(p[k])
    p["W1"][0, 0] = 0.5
    p["W2"][0, 0] = 1.0
    p["W3"][0, 0] = 1.0
    p["b1"][0] = 0.1
    p["b2"][0] = -0.2
    p["b3"][0] = 0.3
    p["x_mean"][:] = 1.0
    p["x_istd"][:] = 2.0
    p["y_scale"][:] = 3.0
    th = M.pack(p)
    x = np.zeros((1, M.D_IN))
    x[0, 0] = 2.0
    xh = (2.0 - 1.0) * 2.0
    g1 = 0.5 * (0.5 * xh + 0.1) * (1 + math.erf((0.5 * xh + 0.1) / math.sqrt(2)))
    g2 = 0.5 * (g1 - 0.2) * (1 + math.erf((g1 - 0.2) / math.sqrt(2)))
    y = M.forward(th, x)
    assert abs(y[0, 0] - 3.0 * (g2 + 0.3)) < 1e-14
    assert np.all(y[0, 1:] == 0.0)


def test_gradients_against_central_differences():
    rng = np.random.default_rng(1)
    th = M.init_params(3, x_mean=rng.normal(size=M.D_IN), x_istd=rng.uniform(0.5, 2, M.D_IN),
                       y_scale=rng.uniform(0.5, 2, M.D_OUT))
    X = rng.normal(size=(6, M.D_IN))
    T = rng.normal(size=(6, M.D_OUT))
    g = M.mse_grad(th, X, T, 7)
    idx = rng.choice(M.N_PARAMS - 80, size=40, replace=False)  # trainable part only
    for i in idx:
        h = 1e-6 * max(1.0, abs(th[i]))
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (M.mse_loss(tp, X, T, 7) - M.mse_loss(tm, X, T, 7)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])
    assert np.all(g[M.N_PARAMS - 80:] == 0.0)


def test_bf16_rounding():
    # exact bfloat16 values are unchanged; halfway cases round to even
    assert M.bf16(np.array([1.0, -2.5, 3.140625]))[2] == 3.140625
    one_ulp = 2.0 ** -7
    assert M.bf16(np.array(1.0 + one_ulp / 2))[()] == 1.0               # tie -> even (1.0)
    assert M.bf16(np.array(1.0 + 1.5 * one_ulp))[()] == 1.0 + 2 * one_ulp  # tie -> even
    assert M.bf16(np.array(1.0 + 0.6 * one_ulp))[()] == 1.0 + one_ulp


def test_zero_scale_output_is_held_at_zero():
    """An output with y_scale 0 is exactly zero, carries no loss and gets no
    gradient; the other outputs are unaffected."""
    rng = np.random.default_rng(7)
    ys = rng.uniform(0.5, 2, M.D_OUT)
    th = M.init_params(4, y_scale=ys)
    ys0 = ys.copy()
    ys0[2] = 0.0
    th0 = M.init_params(4, y_scale=ys0)
    X = rng.normal(size=(5, M.D_IN))
    T = rng.normal(size=(5, M.D_OUT))
    T0 = T.copy()
    T0[:, 2] = 0.0
    y, y0 = M.forward(th, X), M.forward(th0, X)
    assert np.all(y0[:, 2] == 0.0)
    assert np.array_equal(np.delete(y0, 2, axis=1), np.delete(y, 2, axis=1))
    # loss without output 2: the same sum, the same 7-output denominator
    d = ((y - T) / ys)[:, :7]
    d[:, 2] = 0.0
    assert abs(M.mse_loss(th0, X, T0, 7) - np.mean(d * d)) < 1e-15
    g = M.mse_grad(th0, X, T0, 7)
    W3 = M.unpack(g)["W3"]
    assert np.all(W3[:, 2] == 0.0) and np.any(W3[:, 1] != 0.0)
