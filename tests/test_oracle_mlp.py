"""Pins of the FP64 controller oracle (oracle/mlp.py) against facts that do
not come from its own code: finite differences, closed forms of special
weights, the linear regime of tanh, and the exact form of Adam's
bias-corrected steps."""
import math

import numpy as np
import pytest

from oracle import mlp as M


def rand_w(seed, scale=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-scale, scale, M.N_PARAMS)


def test_parameter_count_and_layout():
    assert M.N_PARAMS == 3 * 32 + 32 + 32 * 32 + 32 + 32 + 1 == 1217
    w = np.arange(M.N_PARAMS, dtype=np.float64)
    P = M.unpack(w)
    assert P["W1"][1, 0] == 3 and P["b1"][0] == 96 and P["W2"][0, 1] == 129
    assert P["b3"][0] == 1216
    assert np.array_equal(M.pack(P), w)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_parameter_gradient_matches_central_differences(seed):
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    w = rand_w(seed)
    X = rng.normal(size=(7, 3))
    dY = rng.normal(size=7)
    _, cache = M.forward(w, X)
    g, _ = M.backward(w, X, cache, dY)
    h = 1e-6
    for i in range(M.N_PARAMS):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (M.forward(wp, X)[0] @ dY - M.forward(wm, X)[0] @ dY) / (2 * h)
        assert abs(g[i] - fd) <= 1e-7 * (1.0 + abs(fd)), (i, g[i], fd)


def test_input_gradient_matches_central_differences():
    rng = np.random.Generator(np.random.PCG64(7))
    w = rand_w(3)
    X = rng.normal(size=(5, 3))
    dY = rng.normal(size=5)
    _, cache = M.forward(w, X)
    _, dX = M.backward(w, X, cache, dY)
    h = 1e-6
    for k in range(5):
        for j in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[k, j] += h
            Xm[k, j] -= h
            fd = (M.forward(w, Xp)[0] @ dY - M.forward(w, Xm)[0] @ dY) / (2 * h)
            assert abs(dX[k, j] - fd) <= 1e-7 * (1.0 + abs(fd))


def test_constant_second_layer_gives_constant_output():
    """W2 = 0: the second hidden layer is tanh(b2) for every input, so
    Y = W3 . tanh(b2) + b3 whatever X is, and dX = 0."""
    P = M.unpack(rand_w(5))
    P["W2"][:] = 0.0
    w = M.pack(P)
    X = np.random.default_rng(1).normal(size=(9, 3))
    Y, cache = M.forward(w, X)
    expect = float(sum(P["W3"][0, i] * math.tanh(P["b2"][i]) for i in range(32)) + P["b3"][0])
    assert np.allclose(Y, expect, rtol=0, atol=1e-14)
    _, dX = M.backward(w, X, cache, np.ones(9))
    assert np.all(dX == 0.0)


def test_small_weights_are_the_linear_map():
    """With weights of size s and zero biases tanh(z) = z + O(z^3), so the
    network is the product W3 W2 W1 up to a relative O(s^2) term."""
    s = 1e-4
    P = M.unpack(rand_w(9, s))
    for b in ("b1", "b2", "b3"):
        P[b][:] = 0.0
    w = M.pack(P)
    X = np.random.default_rng(2).normal(size=(6, 3))
    Y, _ = M.forward(w, X)
    lin = np.array([sum(P["W3"][0, i] * sum(P["W2"][i, j] * sum(P["W1"][j, k] * x[k]
                                                                 for k in range(3))
                                            for j in range(32))
                        for i in range(32)) for x in X])
    assert np.all(np.abs(Y - lin) <= 1e-6 * np.abs(lin) + 1e-30)


def test_mse_gradient():
    Y = np.array([1.0, 2.0, 4.0])
    T = np.array([0.0, 2.0, 1.0])
    loss, g = M.mse_grad(Y, T)
    assert loss == pytest.approx((1 + 0 + 9) / 6, abs=1e-15)
    assert np.allclose(g, [1 / 3, 0.0, 1.0], atol=1e-16)


def test_adam_first_and_constant_gradient_steps():
    """Bias correction makes m_hat = g and v_hat = g^2 exactly for a constant
    gradient, so every step moves each parameter by lr g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    w = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 0.01, 1e-8
    for step in range(1, 6):
        w_new, m, v = M.adam_step(w, m, v, g, step, lr=lr, eps=eps)
        assert np.allclose(w_new - w, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-18), step
        w = w_new


def test_adam_minimises_a_quadratic():
    """Adam on f(w) = 1/2 |w - c|^2 ends near c."""
    c = np.array([0.3, -1.2, 2.0])
    w, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for step in range(1, 3001):
        w, m, v = M.adam_step(w, m, v, w - c, step, lr=0.01)
    assert np.allclose(w, c, atol=1e-3)


def test_training_fits_a_smooth_target():
    """Full-batch Adam on a smooth target of the three inputs lowers the loss
    by two orders of magnitude (the pieces work together)."""
    rng = np.random.Generator(np.random.PCG64(11))
    X = rng.uniform(-1, 1, size=(256, 3))
    T = 0.5 * np.sin(1.5 * X[:, 0]) + 0.3 * X[:, 1] * X[:, 2] - 0.2
    w = M.init_params(0).astype(np.float64)
    m, v = np.zeros_like(w), np.zeros_like(w)
    loss0 = M.mse_grad(M.forward(w, X)[0], T)[0]
    for step in range(1, 1501):
        Y, cache = M.forward(w, X)
        loss, dY = M.mse_grad(Y, T)
        g, _ = M.backward(w, X, cache, dY)
        w, m, v = M.adam_step(w, m, v, g, step, lr=3e-3)
    assert loss < loss0 / 100, (loss0, loss)


def test_controller_features_and_delta_map():
    x = M.features(0.7, 1.5, 0.3)
    assert np.array_equal(x, np.zeros(3))
    assert M.delta_from_output(0.0, 1.4, 1.41) == pytest.approx(0.1, rel=1e-15)
    assert M.delta_from_output(math.log(2.0), 1.4, 1.41) == pytest.approx(0.2, rel=1e-15)
    assert M.delta_from_output(50.0, 1.4, 1.41) == 0.7          # min(w)/2
    assert M.delta_from_output(-50.0, 1.4, 1.41) == 1e-3
