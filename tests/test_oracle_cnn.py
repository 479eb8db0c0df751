"""Pins of the FP64 warm-start network oracle: library correlation, finite differences and the
closed form of one Adam step."""
import numpy as np
from scipy.signal import correlate2d

from oracle import cnn as C


def test_conv_forward_matches_library_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 7, 5))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = C.conv3x3(x, w, b)
    for co in range(4):
        ref = b[co] + sum(correlate2d(x[ci], w[co, ci], mode="same", boundary="fill")
                          for ci in range(3))
        assert np.allclose(y[co], ref, atol=1e-12)


def test_conv_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 5, 4))
    w = rng.standard_normal((3, 2, 3, 3))
    b = rng.standard_normal(3)
    dy = rng.standard_normal((3, 5, 4))
    dx, dw, db = C.conv3x3_backward(x, w, dy)
    obj = lambda x_, w_, b_: float(np.sum(dy * C.conv3x3(x_, w_, b_)))
    h = 1e-6
    for idx in [(0, 0, 0), (1, 4, 3), (0, 2, 1), (1, 0, 3)]:
        e = np.zeros_like(x)
        e[idx] = h
        fd = (obj(x + e, w, b) - obj(x - e, w, b)) / (2 * h)
        assert abs(fd - dx[idx]) < 1e-6 * (1 + abs(fd))
    for idx in [(0, 0, 0, 0), (2, 1, 2, 1), (1, 0, 1, 2)]:
        e = np.zeros_like(w)
        e[idx] = h
        fd = (obj(x, w + e, b) - obj(x, w - e, b)) / (2 * h)
        assert abs(fd - dw[idx]) < 1e-6 * (1 + abs(fd))
    assert np.allclose(db, dy.sum(axis=(1, 2)))


def test_network_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    cin = 3
    theta = 0.2 * rng.standard_normal(C.param_count(cin))
    batch = []
    for k in range(2):
        f = rng.uniform(0, 1, (6, 5))
        batch.append((f, [0.3 * (k + 1), -2.0], f + 0.1 * rng.standard_normal((6, 5))))
    loss, grad = C.loss_and_grad(theta, batch)
    assert loss > 0
    h = 1e-6
    for i in rng.choice(theta.size, 25, replace=False):
        e = np.zeros_like(theta)
        e[i] = h
        fd = (C.loss_and_grad(theta + e, batch)[0] - C.loss_and_grad(theta - e, batch)[0]) / (2 * h)
        assert abs(fd - grad[i]) < 1e-5 * (1 + abs(fd)), i


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3])
    theta, m, v = C.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.1, eps=0.0)
    # bias-corrected moments equal g and g^2 after one step: the update is -lr sign(g)
    assert np.allclose(theta, -0.1 * np.sign(g))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_param_count_and_layer_shapes():
    assert C.layer_shapes(11) == [(32, 11), (32, 32), (32, 32), (32, 32), (1, 32)]
    assert C.param_count(11) == 32 * 11 * 9 + 32 + 3 * (32 * 32 * 9 + 32) + 32 * 9 + 1
