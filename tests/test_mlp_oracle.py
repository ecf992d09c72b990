"""Pins of the surrogate MLP oracle (CPU): backward pass against central finite
differences in FP64, and the GELU derivative against its finite difference."""
import numpy as np

from oracle import mlp


def test_gelu_derivative_matches_finite_difference():
    z = np.linspace(-6, 6, 1001)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, rtol=1e-7, atol=1e-9)
    # GELU reduces to the identity far right and to zero far left
    assert abs(mlp.gelu(10.0) - 10.0) < 1e-12 and abs(mlp.gelu(-10.0)) < 1e-12


def test_backward_matches_central_differences():
    dims = (5, 7, 3)
    g = np.random.default_rng(0)
    theta = mlp.init_params(1, dims) + 0.1 * g.normal(size=mlp.n_params(*dims))
    X = g.normal(size=(11, 5))
    T = g.normal(size=(11, 3))
    L, grad = mlp.loss_and_grad(theta, X, T, dims)
    assert L == mlp.loss(theta, X, T, dims)
    fd = np.zeros_like(theta)
    h = 1e-6
    for k in range(theta.size):
        e = np.zeros_like(theta)
        e[k] = h
        fd[k] = (mlp.loss(theta + e, X, T, dims) - mlp.loss(theta - e, X, T, dims)) / (2 * h)
    assert np.linalg.norm(grad - fd) / np.linalg.norm(fd) < 1e-6


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9, -3.14159, 0.0])
    r = mlp.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0          # tie to even
    assert r[2] == 1.0 + 2 ** -6 or r[2] == 1.0 + 2 ** -7
    assert abs(r[3] + 3.14159) < 3.14159 * 2 ** -8
    assert np.all(mlp.bf16_round(r) == r)
