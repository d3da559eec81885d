"""Pins of the FP64 network reference: central finite differences of the loss
(gradients), a linear network against its closed form, and Adam's first
steps written out."""
import numpy as np
import pytest

from oracle import mlp_oracle as M


def test_gradients_match_central_differences():
    dims = [7, 6, 5, 4]
    rng = np.random.default_rng(0)
    p = M.init_params(dims, 1) + rng.normal(0, 0.05, M.param_count(dims))
    x = rng.normal(0, 1, (5, dims[0]))
    t = rng.normal(0, 1, (5, dims[-1]))

    def loss(pp):
        y, _ = M.forward(pp, dims, x)
        return M.mse(y, t)[0]
    y, hs = M.forward(p, dims, x)
    _, dy = M.mse(y, t)
    g, gx = M.backward(p, dims, hs, dy)
    h = 1e-6
    num = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        num[i] = (loss(p + e) - loss(p - e)) / (2 * h)
    assert np.max(np.abs(num - g)) <= 1e-6 * max(1.0, np.max(np.abs(g)))
    # input gradient too
    numx = np.zeros_like(x)
    for idx in np.ndindex(*x.shape):
        e = np.zeros_like(x)
        e[idx] = h
        ya, _ = M.forward(p, dims, x + e)
        yb, _ = M.forward(p, dims, x - e)
        numx[idx] = (M.mse(ya, t)[0] - M.mse(yb, t)[0]) / (2 * h)
    assert np.max(np.abs(numx - gx)) <= 1e-6 * max(1.0, np.max(np.abs(gx)))


def test_single_linear_layer_closed_form():
    """One layer, no activation: y = x W + b; dL/dW = x^T dy, dL/db = sum dy."""
    dims = [3, 2]
    rng = np.random.default_rng(4)
    W = rng.normal(size=(3, 2))
    b = rng.normal(size=2)
    p = np.concatenate([W.ravel(), b])
    x = rng.normal(size=(4, 3))
    y, hs = M.forward(p, dims, x)
    np.testing.assert_allclose(y, x @ W + b, rtol=0, atol=1e-14)
    dy = rng.normal(size=(4, 2))
    g, gx = M.backward(p, dims, hs, dy)
    np.testing.assert_allclose(g[:6].reshape(3, 2), x.T @ dy, atol=1e-14)
    np.testing.assert_allclose(g[6:], dy.sum(0), atol=1e-14)
    np.testing.assert_allclose(gx, dy @ W.T, atol=1e-14)


def test_relu_blocks_gradient():
    dims = [2, 3, 1]
    W1 = np.array([[1.0, -1.0, 0.5], [0.0, 2.0, -1.0]])
    p = np.concatenate([W1.ravel(), np.zeros(3), np.ones(3), [0.0]])
    x = np.array([[1.0, -1.0]])             # z1 = [1, -3, 1.5] -> relu [1, 0, 1.5]
    y, hs = M.forward(p, dims, x)
    assert y[0, 0] == 2.5
    g, _ = M.backward(p, dims, hs, np.ones((1, 1)))
    gW1 = g[:6].reshape(2, 3)
    assert np.all(gW1[:, 1] == 0.0)        # the dead unit gets no gradient
    np.testing.assert_allclose(gW1[:, 0], x[0])


def test_adam_first_steps():
    p = np.array([1.0, -2.0])
    g = np.array([0.5, -0.25])
    m = np.zeros(2)
    v = np.zeros(2)
    p1, m1, v1 = M.adam_step(p, g, m, v, 1, lr=0.1)
    # first bias-corrected step moves each coordinate by lr * sign(g)
    np.testing.assert_allclose(p1, p - 0.1 * np.sign(g), rtol=0, atol=1e-7)
    np.testing.assert_allclose(m1, 0.1 * g)
    np.testing.assert_allclose(v1, 0.001 * g * g)


def test_mse_mean_normalisation_by_hand():
    """mse = mean over every element of (y - t)^2, gradient 2 (y - t) / (number of elements)."""
    y = np.array([[1.0, 2.0], [3.0, 4.0]])
    t = np.array([[0.0, 2.0], [1.0, 1.0]])
    loss, g = M.mse(y, t)
    assert loss == 3.5                                      # (1 + 0 + 4 + 9) / 4
    np.testing.assert_array_equal(g, np.array([[0.5, 0.0], [1.0, 1.5]]))
    loss1, g1 = M.mse(np.array([[2.0, -1.0, 0.0]]), np.zeros((1, 3)))
    assert loss1 == pytest.approx(5.0 / 3.0, rel=1e-15)
    np.testing.assert_allclose(g1, np.array([[4.0 / 3.0, -2.0 / 3.0, 0.0]]), rtol=1e-15)
