"""Pins of the FP64 MLP oracle: finite-difference gradients, Adam algebra."""
import numpy as np

from oracle import mlp


def test_mlp_gradient_matches_finite_differences():
    d_in, H, d_out = 5, 7, 3
    p = mlp.init(d_in, H, d_out, seed=3)
    rng = np.random.default_rng(0)
    X = rng.standard_normal((11, d_in))
    T = rng.standard_normal((11, d_out))
    _, g = mlp.loss_and_grad(p, X, T, d_in, H, d_out)
    h = 1e-6
    idx = rng.choice(p.size, 40, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = mlp.loss_and_grad(p + e, X, T, d_in, H, d_out)
        lm, _ = mlp.loss_and_grad(p - e, X, T, d_in, H, d_out)
        assert abs((lp - lm) / (2 * h) - g[i]) < 1e-7 * max(1.0, abs(g[i]))


def test_mlp_layout_and_silu():
    assert mlp.n_params(32, 256, 6) == 32 * 256 + 256 + 256 * 256 + 256 + 256 * 6 + 6
    z = np.linspace(-5, 5, 11)
    assert np.allclose(mlp.silu(z), z / (1 + np.exp(-z)))
    h = 1e-6
    assert np.allclose((mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h), mlp.dsilu(z), atol=1e-8)


def test_adam_first_step_is_sign_step():
    """With zero moments the first bias-corrected Adam step is lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    assert np.allclose(p, -0.1 * g / (np.abs(g) + 1e-8))
