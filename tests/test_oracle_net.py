"""Pins of the classifier oracle (oracle/net.py) against facts that do not come from itself:
a brute-force loop convolution, shift and identity kernels, the adjoint identity of the
convolution's backward pass, central finite differences of the loss, closed forms of the
binary cross-entropy and of a network whose convolutions are zero, Adam's first step, and
hand-indexed stamps."""
import itertools

import numpy as np
import pytest

from oracle import net


def test_parameter_count():
    # 33*32*9 + 32 + 32*64*9 + 64 + 64*32*9 + 32 + 32 + 1
    assert net.N_PARAM == 9536 + 18496 + 18464 + 33 == 46529


def _conv_loops(X, W, b):
    B, I, H, Wd = X.shape
    O = W.shape[0]
    Z = np.zeros((B, O, H, Wd))
    for bb, o, y, x in itertools.product(range(B), range(O), range(H), range(Wd)):
        s = b[o]
        for i, dy, dx in itertools.product(range(I), range(3), range(3)):
            yy, xx = y + dy - 1, x + dx - 1
            if 0 <= yy < H and 0 <= xx < Wd:
                s += W[o, i, dy, dx] * X[bb, i, yy, xx]
        Z[bb, o, y, x] = s
    return Z


def test_conv_matches_brute_force_loops():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((2, 3, 4, 5))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    np.testing.assert_allclose(net.conv3x3(X, W, b), _conv_loops(X, W, b), rtol=0, atol=1e-12)


def test_conv_identity_and_shift_kernels():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((1, 2, 5, 5))
    W = np.zeros((2, 2, 3, 3))
    W[0, 0, 1, 1] = W[1, 1, 1, 1] = 1.0
    np.testing.assert_array_equal(net.conv3x3(X, W, np.zeros(2)), X)
    # tap (0, 0) reads X[y - 1][x - 1]: the image moves down and right, zero filled
    W = np.zeros((1, 2, 3, 3))
    W[0, 1, 0, 0] = 1.0
    Z = net.conv3x3(X, W, np.array([0.5]))[0, 0]
    assert np.all(Z[0, :] == 0.5) and np.all(Z[:, 0] == 0.5)
    np.testing.assert_array_equal(Z[1:, 1:], X[0, 1, :-1, :-1] + 0.5)


def test_conv_backward_is_the_adjoint():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((2, 3, 9, 9))
    W = rng.standard_normal((5, 3, 3, 3))
    dZ = rng.standard_normal((2, 5, 9, 9))
    dX, dW, db = net.conv3x3_backward(X, W, dZ)
    lin = net.conv3x3(X, W, np.zeros(5))
    # <conv(X), dZ> = <X, conv^T(dZ)> = <W, dW>
    assert np.isclose(np.sum(lin * dZ), np.sum(X * dX), rtol=1e-12)
    assert np.isclose(np.sum(lin * dZ), np.sum(W * dW), rtol=1e-12)
    np.testing.assert_allclose(db, dZ.sum(axis=(0, 2, 3)), rtol=1e-14)


def _init(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for name, shp in net.SHAPES:
        fan_in = int(np.prod(shp[1:])) if len(shp) > 1 else 32
        parts.append(rng.uniform(-1, 1, size=shp).reshape(-1) * scale * np.sqrt(6.0 / fan_in))
    return np.concatenate(parts)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    theta = _init(5)
    X = rng.standard_normal((3, 33, 9, 9))
    y = np.array([1.0, 0.0, 1.0])
    loss, g = net.loss_and_grad(theta, X, y)
    assert np.isclose(loss, net.bce(net.forward(theta, X)[0], y))
    h = 1e-6
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in net.SHAPES])
    idx = []
    for k in range(len(net.SHAPES)):  # a few entries of every tensor
        idx += list(rng.integers(offs[k], offs[k + 1], size=min(6, offs[k + 1] - offs[k])))
    for j in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        fd = (net.bce(net.forward(tp, X)[0], y) - net.bce(net.forward(tm, X)[0], y)) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1e-3, np.abs(g).max()), (j, fd, g[j])


def test_bce_closed_forms():
    assert np.isclose(net.bce(np.zeros(4), np.array([0, 1, 0, 1.0])), np.log(2.0))
    assert net.bce(np.array([800.0]), np.array([1.0])) < 1e-300 + 1e-12
    assert np.isclose(net.bce(np.array([-800.0]), np.array([1.0])), 800.0)
    assert np.isclose(net.sigmoid(np.log(3.0)), 0.75)


def test_zero_convolutions_closed_form():
    """W1 = W2 = W3 = 0, b1 = b2 = 0: the features are relu(b3) for every stamp, so
    z = w4 . relu(b3) + b4, dL/db4 = sum_b dz_b, dL/dw4 = relu(b3) sum_b dz_b,
    dL/db3 = w4 [b3 > 0] sum_b dz_b, and every other gradient is zero."""
    rng = np.random.default_rng(6)
    p = {name: np.zeros(shp) for name, shp in net.SHAPES}
    p["b3"] = rng.standard_normal(32)
    p["w4"] = rng.standard_normal(32)
    p["b4"] = np.array([0.3])
    theta = net.pack(p)
    X = rng.standard_normal((4, 33, 9, 9))
    y = np.array([1.0, 0.0, 0.0, 1.0])
    r = np.maximum(p["b3"], 0)
    z0 = p["w4"] @ r + 0.3
    z, _ = net.forward(theta, X)
    np.testing.assert_allclose(z, z0, rtol=1e-13)
    loss, g = net.loss_and_grad(theta, X, y)
    s = np.sum((1 / (1 + np.exp(-z0)) - y) / 4)
    G = net.unpack(g)
    assert np.isclose(G["b4"][0], s)
    np.testing.assert_allclose(G["w4"], r * s, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(G["b3"], p["w4"] * (p["b3"] > 0) * s, rtol=1e-12, atol=1e-15)
    for name in ("W1", "b1", "W2", "b2", "W3"):
        assert np.all(G[name] == 0)


def test_adam_first_step_is_sign_step():
    g = np.array([0.5, -2.0, 1e-3])
    theta, m, v = net.adam(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(theta, -0.01 * np.sign(g), rtol=1e-14)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_stamps_by_hand():
    C, N = 40, 12
    c, y, x = np.meshgrid(np.arange(C), np.arange(N), np.arange(N), indexing="ij")
    cube = (c * 10000 + y * 100 + x).astype(np.float64)
    s = net.stamps(cube, [(20, 6, 5), (2, 0, 11)])
    assert s.shape == (2, 33, 9, 9)
    assert s[0, 16, 4, 4] == 20 * 10000 + 6 * 100 + 5
    assert s[0, 0, 0, 0] == 4 * 10000 + 2 * 100 + 1
    assert s[0, 32, 8, 8] == 36 * 10000 + 10 * 100 + 9
    # near the cube's corner: channels below 0, rows above 0 and columns past 11 are zero
    assert s[1, 16, 4, 4] == 2 * 10000 + 0 + 11
    assert np.all(s[1, :14] == 0) and np.all(s[1, :, :4] == 0) and np.all(s[1, :, :, 5:] == 0)
    assert s[1, 14, 4, 4] == 0 * 10000 + 0 + 11
