"""Pins of the FP64 MLP oracle (policy network for the sketch size):
closed forms of special cases, finite differences, and the Adam update under
a constant gradient.  None of them re-types the oracle's own formulas."""
import numpy as np
import pytest

from oracle import mlp

F, H, O = 8, 64, 2


def rand_theta(seed, scale=0.2):
    g = np.random.default_rng(seed)
    return g.standard_normal(mlp.param_count(F, H, O)) * scale


def test_param_count_and_layout():
    assert mlp.param_count(F, H, O) == F * H + H + 2 * (H * H + H) + H * O + O == 9026
    th = np.arange(mlp.param_count(F, H, O), dtype=np.float64)
    layers = mlp.unpack(th, F, H, O)
    assert [W.shape for W, _ in layers] == [(H, F), (H, H), (H, H), (O, H)]
    # W_1 row-major then b_1
    assert layers[0][0][1, 0] == F and layers[0][1][0] == F * H


def test_linear_regime_collapses_to_one_affine_map():
    """Positive inputs, weights and biases keep every ReLU in its identity
    branch, so the network is the single affine map x -> A x + c with
    A = W4 W3 W2 W1 and c built by folding the biases."""
    g = np.random.default_rng(1)
    th = np.abs(g.standard_normal(mlp.param_count(F, H, O))) * 0.1
    X = np.abs(g.standard_normal((7, F)))
    (W1, b1), (W2, b2), (W3, b3), (W4, b4) = mlp.unpack(th, F, H, O)
    A = W4 @ W3 @ W2 @ W1
    c = W4 @ (W3 @ (W2 @ b1 + b2) + b3) + b4
    Y, _ = mlp.forward(th, X, F, H, O)
    np.testing.assert_allclose(Y, X @ A.T + c, rtol=1e-12)


def test_dead_hidden_layer_outputs_last_bias():
    """A last hidden layer whose pre-activations are all negative outputs
    exactly b_4, and its gradient reaches only b_4."""
    th = rand_theta(2)
    layers = mlp.unpack(th, F, H, O)
    W3, b3 = layers[2]
    W3[:] = 0.0
    b3[:] = -1.0
    X = np.random.default_rng(3).standard_normal((5, F))
    T = np.random.default_rng(4).standard_normal((5, O))
    Y, _ = mlp.forward(th, X, F, H, O)
    np.testing.assert_array_equal(Y, np.broadcast_to(layers[3][1], Y.shape))
    L, g = mlp.loss_grad(th, X, T, F, H, O)
    nb4 = O
    assert np.all(g[:-nb4] == 0.0)
    # closed form for the output bias: dL/db = 2 / (B O) * sum_b (y - t)
    np.testing.assert_allclose(g[-nb4:], 2.0 * (Y - T).sum(axis=0) / (5 * O), rtol=1e-13)


@pytest.mark.parametrize("seed", [5, 6])
def test_gradient_matches_central_differences(seed):
    th = rand_theta(seed)
    g = np.random.default_rng(seed + 100)
    X = g.standard_normal((16, F))
    T = g.standard_normal((16, O))
    L, grad = mlp.loss_grad(th, X, T, F, H, O)
    assert L == pytest.approx(mlp.loss(th, X, T, F, H, O), rel=1e-14)
    idx = np.concatenate([np.arange(0, 40), g.choice(th.size, 120, replace=False), np.arange(th.size - 10, th.size)])
    fd = mlp.finite_difference_grad(th, X, T, F, H, O, h=1e-6, idx=idx)
    np.testing.assert_allclose(grad[idx], fd, rtol=2e-5, atol=1e-9)


def test_gradient_mutations_are_caught():
    """Dropping the ReLU mask or the 1/(B O) factor in backpropagation
    disagrees with finite differences."""
    th = rand_theta(7)
    g = np.random.default_rng(8)
    X = g.standard_normal((12, F))
    T = g.standard_normal((12, O))
    _, grad = mlp.loss_grad(th, X, T, F, H, O)
    idx = np.arange(0, mlp.param_count(F, H, O), 37)
    fd = mlp.finite_difference_grad(th, X, T, F, H, O, idx=idx)
    assert np.allclose(grad[idx], fd, rtol=1e-4, atol=1e-9)
    assert not np.allclose(grad[idx] * 12, fd, rtol=1e-4, atol=1e-9)

    def no_mask(theta, X, T):
        layers = mlp.unpack(theta, F, H, O)
        Y, zs = mlp.forward(theta, X, F, H, O)
        ins = [X] + [np.maximum(z, 0.0) for z in zs[:-1]]
        delta = 2.0 * (Y - T) / (X.shape[0] * O)
        out = [None] * 4
        for li in range(3, -1, -1):
            out[li] = np.concatenate([(delta.T @ ins[li]).reshape(-1), delta.sum(0)])
            if li:
                delta = delta @ layers[li][0]
        return np.concatenate(out)

    assert not np.allclose(no_mask(th, X, T)[idx], fd, rtol=1e-4, atol=1e-9)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments are exactly g and
    g^2, so each step moves theta by lr * g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th = np.array([1.0, 2.0, 3.0, 4.0])
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 1e-2, 1e-8
    t = th.copy()
    for step in range(1, 6):
        t, m, v = mlp.adam_step(t, m, v, g, step, lr, eps=eps)
    np.testing.assert_allclose(t, th - 5 * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_training_fits_a_linear_target():
    """Adam on the oracle network drives the loss on an affine target far
    below its starting value (sanity of the whole training step)."""
    g = np.random.default_rng(9)
    X = g.standard_normal((64, F))
    A = g.standard_normal((O, F))
    T = X @ A.T + 0.3
    th = rand_theta(10, scale=0.15)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    L0 = mlp.loss(th, X, T, F, H, O)
    for step in range(1, 301):
        _, gr = mlp.loss_grad(th, X, T, F, H, O)
        th, m, v = mlp.adam_step(th, m, v, gr, step, 3e-3)
    assert mlp.loss(th, X, T, F, H, O) < 0.02 * L0
