"""FP64 oracle of the learned phase-change source surrogate -- TEST INFRASTRUCTURE.

A multilayer perceptron 17 -> 256 -> 256 -> 15 with GELU activations (tanh form,
0.5 z (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3)))) and a mean-squared-error loss
over the batch and the outputs.  Parameters are stored flat in the order
W1 (n_in x n_h, row-major), b1, W2 (n_h x n_h), b2, W3 (n_h x n_out), b3 -- the
layout the HIP library uses.  Written as plain matrix products so a reader can
check forward and backward by eye; the backward pass is pinned by central finite
differences in the tests.

``forward_bf16`` / ``loss_and_grad_bf16`` are the same passes at the network's
stated precision (bfloat16 weights and activations, wider accumulation): every
value the network stores in bfloat16 -- the hidden activations after the GELU, and
in the backward pass the output error and the two hidden-layer errors -- is rounded
to bfloat16 at that point, all other arithmetic stays FP64.
"""
import numpy as np

C_GELU = np.sqrt(2.0 / np.pi)


def shapes(n_in=17, n_h=256, n_out=15):
    return [(n_in, n_h), (n_h,), (n_h, n_h), (n_h,), (n_h, n_out), (n_out,)]


def n_params(n_in=17, n_h=256, n_out=15):
    return sum(int(np.prod(s)) for s in shapes(n_in, n_h, n_out))


def unpack(theta, n_in=17, n_h=256, n_out=15):
    out, k = [], 0
    for s in shapes(n_in, n_h, n_out):
        n = int(np.prod(s))
        out.append(theta[k:k + n].reshape(s))
        k += n
    return out


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(C_GELU * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    u = C_GELU * (z + 0.044715 * z ** 3)
    t = np.tanh(u)
    du = C_GELU * (1.0 + 3.0 * 0.044715 * z ** 2)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * du


def forward(theta, X, dims=(17, 256, 15)):
    W1, b1, W2, b2, W3, b3 = unpack(theta, *dims)
    Z1 = X @ W1 + b1
    H1 = gelu(Z1)
    Z2 = H1 @ W2 + b2
    H2 = gelu(Z2)
    Y = H2 @ W3 + b3
    return Y, (Z1, H1, Z2, H2)


def forward_bf16(theta, X, dims=(17, 256, 15)):
    """Forward pass with the hidden activations rounded to bfloat16 after the GELU.
    Returns Y and the pre-rounding activations G1, G2 beside Z1, H1, Z2, H2."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, *dims)
    Z1 = X @ W1 + b1
    G1 = gelu(Z1)
    H1 = bf16_round(G1)
    Z2 = H1 @ W2 + b2
    G2 = gelu(Z2)
    H2 = bf16_round(G2)
    Y = H2 @ W3 + b3
    return Y, dict(Z1=Z1, G1=G1, H1=H1, Z2=Z2, G2=G2, H2=H2)


def loss_and_grad_bf16(theta, X, T, dims=(17, 256, 15)):
    """Loss and gradient of the bfloat16 forward pass, with the output error
    dY = 2 (Y - T) / n and the hidden-layer errors dZ = (dH W^T) GELU'(Z) rounded to
    bfloat16 as they are formed.  Returns the loss, the flat gradient and every
    intermediate (pre-rounding values as P*)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, *dims)
    Y, a = forward_bf16(theta, X, dims)
    n = X.shape[0] * Y.shape[1]
    L = np.sum((Y - T) ** 2) / n
    PdY = 2.0 * (Y - T) / n
    dY = bf16_round(PdY)
    dW3 = a["H2"].T @ dY
    db3 = dY.sum(axis=0)
    A2 = dY @ W3.T
    PdZ2 = A2 * gelu_grad(a["Z2"])
    dZ2 = bf16_round(PdZ2)
    dW2 = a["H1"].T @ dZ2
    db2 = dZ2.sum(axis=0)
    A1 = dZ2 @ W2.T
    PdZ1 = A1 * gelu_grad(a["Z1"])
    dZ1 = bf16_round(PdZ1)
    dW1 = X.T @ dZ1
    db1 = dZ1.sum(axis=0)
    g = np.concatenate([v.ravel() for v in (dW1, db1, dW2, db2, dW3, db3)])
    a.update(Y=Y, PdY=PdY, dY=dY, A2=A2, PdZ2=PdZ2, dZ2=dZ2, A1=A1, PdZ1=PdZ1, dZ1=dZ1)
    return L, g, a


def loss(theta, X, T, dims=(17, 256, 15)):
    Y, _ = forward(theta, X, dims)
    return np.mean((Y - T) ** 2)


def loss_and_grad(theta, X, T, dims=(17, 256, 15)):
    """Loss and its gradient with respect to the flat parameter vector."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, *dims)
    Y, (Z1, H1, Z2, H2) = forward(theta, X, dims)
    n = X.shape[0] * Y.shape[1]
    L = np.sum((Y - T) ** 2) / n
    dY = 2.0 * (Y - T) / n
    dW3 = H2.T @ dY
    db3 = dY.sum(axis=0)
    dZ2 = (dY @ W3.T) * gelu_grad(Z2)
    dW2 = H1.T @ dZ2
    db2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2.T) * gelu_grad(Z1)
    dW1 = X.T @ dZ1
    db1 = dZ1.sum(axis=0)
    g = np.concatenate([a.ravel() for a in (dW1, db1, dW2, db2, dW3, db3)])
    return L, g


def init_params(seed=0, dims=(17, 256, 15)):
    """He-style initialisation (weights ~ N(0, 2/fan_in), biases 0)."""
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for s in shapes(*dims):
        if len(s) == 2:
            parts.append(g.normal(0.0, np.sqrt(2.0 / s[0]), size=s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)


def bf16_round(x):
    """Round float64 values to bfloat16 (round to nearest even) and back."""
    x32 = np.asarray(x, dtype=np.float32)
    b = x32.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)
