"""Pins of the surrogate MLP oracle (CPU): the forward pass on a network whose output
is known by hand, the GELU against the exact (erf) GELU it approximates, the
backward pass against central finite differences in FP64, and the bfloat16
rounding against hand-worked cases."""
import math

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
    """bfloat16 keeps 8 significant bits (7 stored): the spacing above 1 is 2^-7;
    ties go to the even neighbour."""
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7 + 2 ** -8 + 2 ** -12,
                  -3.14159, 0.0, 2.0 ** -130])
    r = mlp.bf16_round(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                          # tie between 1 and 1 + 2^-7: even is 1
    assert r[2] == 1.0 + 2 ** -7                # below the half-way point
    assert r[3] == 1.0 + 2 ** -6                # tie between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6
    assert r[4] == 1.0 + 2 ** -6                # above the half-way point
    assert r[5] == -3.140625                    # -0b11.00100100... -> 8 significant bits
    assert r[6] == 0.0
    assert r[7] == 2.0 ** -130                  # subnormal in float32, exact in bfloat16
    assert np.all(mlp.bf16_round(r) == r)


def test_gelu_close_to_exact_gelu():
    """The tanh form approximates the exact GELU z Phi(z) = z (1 + erf(z / sqrt 2)) / 2
    to within 5e-4 everywhere (the published accuracy of the approximation); a wrong
    constant in either term of the tanh argument breaks that bound."""
    z = np.linspace(-8, 8, 16001)
    exact = np.array([0.5 * t * (1.0 + math.erf(t / math.sqrt(2.0))) for t in z])
    assert np.abs(mlp.gelu(z) - exact).max() < 5e-4


def test_forward_on_a_hand_worked_network():
    """Forward pass of a 3 -> 4 -> 4 -> 2 network whose pre-activations are all far
    from zero, where GELU is exactly the identity (z >= 20) or zero (z <= -20) in
    FP64: the output follows by integer arithmetic, which fixes the layer order, the
    row-major layout of each weight matrix (inputs along rows) and the position of
    every bias in the flat parameter vector."""
    dims = (3, 4, 2)
    W1 = np.array([[10, 0, -10, 1], [0, 20, 0, 2], [5, 0, 0, 3]], dtype=float)
    b1 = np.array([5, -20, -40, 20], dtype=float)
    W2 = np.array([[1, 0, 0, -1], [0, 1, 0, 0], [0, 0, 1, 0], [0, 1, 2, 1]], dtype=float)
    b2 = np.array([0, 0, -100, 1], dtype=float)
    W3 = np.array([[1, 2], [3, 0], [5, 5], [0, -1]], dtype=float)
    b3 = np.array([7, -7], dtype=float)
    theta = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
    assert theta.size == mlp.n_params(*dims)
    X = np.array([[2, 3, 4]], dtype=float)
    # layer 1: z = (20+0+20+5, 0+60+0-20, -20+0+0-40, 2+6+12+20) = (45, 40, -60, 40),
    # h1 = (45, 40, 0, 40); layer 2: z = (45, 40+40, 0+80-100, -45+40+1) = (45, 80, -20, -4)
    Y, (Z1, H1, Z2, H2) = mlp.forward(theta, X, dims)
    assert np.all(Z1[0] == [45, 40, -60, 40])
    assert np.all(H1[0] == [45, 40, 0, 40])
    assert np.all(Z2[0] == [45, 80, -20, -4])
    assert H2[0, 0] == 45 and H2[0, 1] == 80 and H2[0, 2] == 0.0
    # the one unsaturated unit: GELU(-4) = -4 Phi(-4) ~ -1.3e-4 (tanh form: within 5e-4)
    assert abs(H2[0, 3]) < 1e-3
    # output: (45*1 + 80*3 + 0*5 + h*0 + 7, 45*2 + 0 + 0 - h - 7)
    h = H2[0, 3]
    assert Y[0, 0] == 45 + 240 + 7
    assert Y[0, 1] == 90 - h - 7


def test_bf16_passes_are_the_fp64_passes_with_roundings(monkeypatch):
    """The bfloat16-precision passes are the FP64 passes (pinned above by finite
    differences) with roundings inserted: with the rounding made the identity they
    reproduce loss, gradient and output exactly; with it, every stored activation
    and error is a bfloat16 number."""
    dims = (5, 7, 3)
    g = np.random.default_rng(4)
    theta = mlp.init_params(2, dims) + 0.1 * g.normal(size=mlp.n_params(*dims))
    X = mlp.bf16_round(g.normal(size=(9, 5)))
    T = g.normal(size=(9, 3))
    L, grad, a = mlp.loss_and_grad_bf16(theta, X, T, dims)
    for k in ("H1", "H2", "dY", "dZ2", "dZ1"):
        assert np.all(mlp.bf16_round(a[k]) == a[k]), k
    assert L != mlp.loss(theta, X, T, dims)
    monkeypatch.setattr(mlp, "bf16_round", lambda x: np.asarray(x, dtype=np.float64))
    L1, g1, a1 = mlp.loss_and_grad_bf16(theta, X, T, dims)
    L0, g0 = mlp.loss_and_grad(theta, X, T, dims)
    assert L1 == L0 and np.array_equal(g1, g0)
    assert np.array_equal(a1["Y"], mlp.forward(theta, X, dims)[0])
