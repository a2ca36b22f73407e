"""Pins of the FP64 surrogate-network reference: gradients against central
finite differences, and AdamW against its closed-form first step."""
import numpy as np

from oracle import mlp


def test_gradient_matches_central_differences():
    shapes = mlp.layer_shapes(5, 12, 3)
    p = mlp.init_params(shapes, seed=3)
    rng = np.random.default_rng(0)
    X = rng.normal(size=(7, 5))
    y = rng.normal(size=7)
    L, g = mlp.loss_and_grad(p, X, y, shapes)
    assert g.shape == p.shape
    h = 1e-6
    idx = rng.choice(p.size, 60, replace=False)
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (mlp.loss_and_grad(p + e, X, y, shapes)[0] - mlp.loss_and_grad(p - e, X, y, shapes)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_parameter_count_of_the_surrogate():
    assert mlp.num_params(mlp.layer_shapes(5, 128, 3)) == 33921


def test_adamw_first_step_is_sign_step():
    """With m0 = v0 = 0 the bias-corrected first step is lr * g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = mlp.adamw_step(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-2, eps=0.0)
    np.testing.assert_allclose(p - p1, 1e-2 * np.sign(g), rtol=1e-12)
    # decoupled weight decay alone shrinks the weights geometrically
    p2, _, _ = mlp.adamw_step(p, np.zeros(50), np.zeros(50), np.zeros(50) + 1.0, 1, lr=1e-2, wd=0.1)
    np.testing.assert_allclose(p2, p * (1 - 1e-3), rtol=1e-12)


def test_training_reduces_loss_on_a_smooth_target():
    shapes = mlp.layer_shapes(2, 16, 2)
    p = mlp.init_params(shapes, seed=0)
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, size=(64, 2))
    y = np.sin(2 * X[:, 0]) + X[:, 1] ** 2
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    L0 = mlp.loss_and_grad(p, X, y, shapes)[0]
    for t in range(1, 301):
        L, g = mlp.loss_and_grad(p, X, y, shapes)
        p, m, v = mlp.adamw_step(p, g, m, v, t, lr=1e-2)
    assert L < 0.1 * L0
