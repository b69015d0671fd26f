"""Pins of the oracle's learned-cost-model pieces (MLP, bfloat16 rounding,
Adam) and of the per-box features."""
import numpy as np
import pytest

import oracle
import picsynth


def _init(seed):
    rng = np.random.default_rng(seed)
    P = np.zeros(oracle.NPARAM_MLP)
    o = 0
    for fan_in, fan_out in ((16, 64), (64, 64), (64, 1)):
        lim = np.sqrt(6.0 / fan_in)
        P[o:o + fan_in * fan_out] = rng.uniform(-lim, lim, fan_in * fan_out); o += fan_in * fan_out
        P[o:o + fan_out] = rng.uniform(-0.1, 0.1, fan_out); o += fan_out
    return P


def test_mlp_gradient_finite_differences():
    rng = np.random.default_rng(1)
    P = _init(2)
    X = rng.normal(size=(9, 16))
    y = rng.normal(size=9)
    loss, g, _ = oracle.mlp_loss_grad(P, X, y)
    h = 1e-6
    idx = np.r_[0, 5, 1023, 1024, 1100, 1088 + 4095, 5248, 5300, 5312]
    for i in idx:
        Pp = P.copy(); Pp[i] += h
        Pm = P.copy(); Pm[i] -= h
        fd = (oracle.mlp_loss_grad(Pp, X, y, want_grad=False)[0] -
              oracle.mlp_loss_grad(Pm, X, y, want_grad=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9


def test_mlp_forward_by_hand():
    # one hidden unit path: W1[0,0] = 2, b1 = 0; W2[0,0] = 3; W3[0] = 0.5, b3 = 1
    P = np.zeros(oracle.NPARAM_MLP)
    P[0] = 2.0
    P[16 * 64 + 64] = 3.0
    P[16 * 64 + 64 + 64 * 64 + 64] = 0.5
    P[-1] = 1.0
    X = np.zeros((2, 16)); X[0, 0] = 1.5; X[1, 0] = -1.0
    loss, _, yhat = oracle.mlp_loss_grad(P, X, np.array([0.0, 0.0]), want_grad=False)
    np.testing.assert_array_equal(yhat, [1.0 + 0.5 * 3 * 2 * 1.5, 1.0])   # ReLU cuts the negative one
    assert loss == (5.5 ** 2 + 1.0) / 2


def test_bf16_rounding():
    assert oracle.bf16(1.0 + 2 ** -8) == 1.0                 # tie -> even
    assert oracle.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6   # tie -> even (up)
    assert oracle.bf16(1.0 + 2 ** -7) == 1.0 + 2 ** -7       # representable
    assert oracle.bf16(-3.0) == -3.0


def test_mlp_mirror_mode_exact_on_representable_values():
    # With bfloat16-exact inputs, weights and activations, rounding changes nothing.
    P = np.zeros(oracle.NPARAM_MLP)
    rng = np.random.default_rng(4)
    P[:16 * 64] = rng.integers(-2, 3, 16 * 64) * 0.25
    o = 16 * 64 + 64
    P[o:o + 64 * 64] = rng.integers(-2, 3, 64 * 64) * 0.125
    o += 64 * 64 + 64
    P[o:o + 64] = rng.integers(-2, 3, 64) * 0.5
    X = rng.integers(-2, 3, (5, 16)).astype(float)
    y = rng.normal(size=5)
    a = oracle.mlp_loss_grad(P, X, y, mirror=False)
    b = oracle.mlp_loss_grad(P, X, y, mirror=True)
    assert a[0] == b[0]
    # and on generic values mirror mode stays within bfloat16 precision
    P = _init(5)
    X = rng.normal(size=(64, 16))
    la = oracle.mlp_loss_grad(P, X, y=np.zeros(64), mirror=False)[2]
    lb = oracle.mlp_loss_grad(P, X, y=np.zeros(64), mirror=True)[2]
    assert np.abs(la - lb).max() < 0.05 * np.abs(la).max()


def test_adam_first_step_and_training_reduces_loss():
    P = np.array([1.0, -2.0]); m = np.zeros(2); v = np.zeros(2)
    oracle.adam(P, np.array([0.3, -4.0]), m, v, 1, lr=0.1)
    # first bias-corrected step is lr * g / (|g| + eps)
    np.testing.assert_allclose(P, [1.0 - 0.1 * 0.3 / (0.3 + 1e-8), -2.0 + 0.1 * 4.0 / (4.0 + 1e-8)], rtol=1e-15)
    rng = np.random.default_rng(7)
    X = rng.normal(size=(256, 16))
    y = np.log1p(np.abs(X[:, 0]) * 3 + X[:, 1] ** 2)
    P = _init(8); m = np.zeros_like(P); v = np.zeros_like(P)
    l0 = oracle.mlp_loss_grad(P, X, y, want_grad=False)[0]
    for t in range(1, 201):
        _, g, _ = oracle.mlp_loss_grad(P, X, y)
        oracle.adam(P, g, m, v, t)
    l1 = oracle.mlp_loss_grad(P, X, y, want_grad=False)[0]
    assert l1 < 0.2 * l0


def test_box_features_by_hand():
    n = (16, 16, 16)
    boxes = picsynth.uniform_boxes(n, 8)
    # box 0 = [0,8)^3 (touches domain faces); 3 particles in cell (1,1,1), one in (0,5,5)
    x = np.array([[1.2, 1.5, 1.7], [1.9, 1.1, 1.3], [1.5, 1.5, 1.5], [0.5, 5.5, 5.5],
                  [12.0, 12.0, 12.0]])
    u = np.array([[3.0, 4.0, 0.0], [0.0, 0.0, 1.0], [0.0, 0.0, 0.0], [0.0, 0.0, 2.0], [1, 1, 1]])
    sp = np.array([0, 0, 1, 0, 1], np.int32)
    f = oracle.box_features(n, boxes, x, u, sp, 2, 2)
    f0 = f[0]
    assert f0[0] == np.log(4.0) and f0[1] == np.log(2.0)
    # 512 cells: 510 empty, one with 1, one with 3
    assert f0[2] == np.log(511.0) and f0[3] == np.log(2.0) and f0[4] == np.log(2.0)
    assert f0[10] == np.log(512.0) and f0[11] == 2.0 and f0[12] == 1.0
    assert f0[13] == np.log(2.0)            # only the particle at x=0.5 is in the outer layer
    assert f0[14] == np.log(4.0)
    assert abs(f0[15] - (5.0 + 1.0 + 0.0 + 2.0) / 4.0) < 1e-15
    # box 7 = [8,16)^3 touches the upper faces; its particle is in an inner cell
    f7 = f[7]
    assert f7[12] == 1.0 and f7[13] == 0.0 and f7[1] == np.log(2.0)
