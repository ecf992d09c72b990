"""BF16 MFMA surrogate network against its FP64 oracle (oracle/mlp.py).

The GPU rounds weights, inputs and hidden activations to bfloat16 and accumulates
in FP32.  Two comparisons:

* element by element against the oracle at the network's precision
  (``forward_bf16`` / ``loss_and_grad_bf16``: FP64 arithmetic with the bfloat16
  roundings at the points where the network stores bfloat16).  Each element's bar is
  a rigorous bound of what FP32 accumulation (gamma_K = K u / (1 - K u), doubled for
  the matrix cores' rounding), the hardware exp2/reciprocal GELU and the bfloat16
  roundings can make of the difference, propagated layer by layer.  A rounding
  counts only where the oracle's value before it lies within the propagated error of
  a rounding boundary (both sides round alike everywhere else); there it may move by
  one bfloat16 step.  So the bars are a few FP32 ulps of each element's scale except
  at the rare elements next to a rounding tie.
* against the unrounded FP64 network, as the accuracy report of the bfloat16
  arithmetic: forward relative L2 <= 2e-2, gradient cosine > 0.999.
"""
import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_20742_amd import binding
    binding.load()
    return binding


U32 = 2.0 ** -24
C_GELU = np.sqrt(2.0 / np.pi)


def _gamma(k):
    """Bound of the relative error of a K-term FP32 sum, doubled (accumulation
    order and rounding inside the matrix cores are not specified)."""
    return 2.0 * k * U32 / (1.0 - k * U32)


def _flip(v, d):
    """Largest difference of the bfloat16 roundings of two values within d of v."""
    return np.abs(omlp.bf16_round(v + d) - omlp.bf16_round(v - d))


def _gelu_err(z):
    """Error bound of the device GELU z / (1 + 2^t), t = z (c + 0.044715 c z^2),
    c = -2 sqrt(2/pi) log2(e): the argument's roundings (z^2, the fused multiply-add
    with its rounded coefficient, the product with z: at most 4u relative) scale
    e = 2^t by up to 4 ln2 |t| u, the hardware exp2 and reciprocal and four more
    roundings add a few u; 1.5 times that, plus an absolute floor for the saturated
    tails."""
    t = -2.0 * C_GELU * np.log2(np.e) * (z + 0.044715 * z ** 3)
    return 2.0 * U32 * (3.0 * np.log(2.0) * np.abs(t) + 8.0) * np.abs(omlp.gelu(z)) + 1e-30


def _gelu_grad_err(z):
    """Error bound of the device GELU derivative s + 2 z s (1 - s) u'(z) (same
    exponential, (1 - s) formed in FP32)."""
    t = -2.0 * C_GELU * np.log2(np.e) * (z + 0.044715 * z ** 3)
    slope = 1.0 + 2.0 * np.abs(z) * C_GELU * (1.0 + 3.0 * 0.044715 * z * z)
    return 2.0 * U32 * (3.0 * np.log(2.0) * np.abs(t) + 12.0) * slope + 1e-30


def _act_bound(Z, dZ, G, err):
    """Bound on |device activation - oracle activation| before the bfloat16 rounding:
    slope times the argument error (|GELU''| <= 1) plus the device GELU's own error."""
    return (np.abs(omlp.gelu_grad(Z)) + dZ) * dZ + err(Z)


def _forward_bounds(theta_r, X, dims):
    W1, b1, W2, b2, W3, b3 = [np.abs(w) for w in omlp.unpack(theta_r, *dims)]
    Y, a = omlp.forward_bf16(theta_r, X, dims)
    n_in, n_h, _ = dims
    dZ1 = _gamma(n_in) * (np.abs(X) @ W1 + b1) + U32 * np.abs(a["Z1"])
    dH1 = _flip(a["G1"], _act_bound(a["Z1"], dZ1, a["G1"], _gelu_err))
    dZ2 = dH1 @ W2 + _gamma(n_h) * ((np.abs(a["H1"]) + dH1) @ W2 + b2) + U32 * np.abs(a["Z2"])
    dH2 = _flip(a["G2"], _act_bound(a["Z2"], dZ2, a["G2"], _gelu_err))
    dY = dH2 @ W3 + _gamma(n_h) * ((np.abs(a["H2"]) + dH2) @ W3 + b3) + U32 * np.abs(Y)
    return Y, a, dict(Z1=dZ1, H1=dH1, Z2=dZ2, H2=dH2, Y=dY)


def _setup(dims, rows, seed):
    g = np.random.default_rng(seed)
    theta = omlp.init_params(seed, dims) + 0.02 * g.normal(size=omlp.n_params(*dims))
    n_w = [int(np.prod(s)) for s in omlp.shapes(*dims)]
    # weights rounded to bf16 as the GPU sees them; biases stay FP32
    parts, k = [], 0
    for s, n in zip(omlp.shapes(*dims), n_w):
        p = theta[k:k + n]
        parts.append(omlp.bf16_round(p) if len(s) == 2 else p.astype(np.float32).astype(np.float64))
        k += n
    theta_r = np.concatenate(parts)
    X = omlp.bf16_round(g.normal(size=(rows, dims[0])))
    T = g.normal(size=(rows, dims[2]))
    return theta, theta_r, X, T


@pytest.mark.parametrize("dims,rows", [((17, 256, 15), 1000), ((17, 256, 15), 4099), ((5, 64, 3), 77)])
def test_forward_matches_oracle(B, dims, rows):
    theta, theta_r, X, T = _setup(dims, rows, 1)
    net = B.MLP(*dims)
    net.set_params(theta)
    Y = net.forward(torch.tensor(X, dtype=torch.float32, device="cuda")).cpu().numpy()
    Yo, _ = omlp.forward(theta_r, X, dims)
    e = np.linalg.norm(Y - Yo) / np.linalg.norm(Yo)
    assert e <= 2e-2, e


@pytest.mark.parametrize("dims,rows", [((17, 256, 15), 1000), ((17, 256, 15), 4099), ((5, 64, 3), 77)])
def test_forward_elementwise(B, dims, rows):
    """Every output element within its propagated bound of the bfloat16-precision
    oracle (fused inference kernel for the 17 -> 256 -> 15 shape, layer-by-layer
    GEMMs for the other)."""
    theta, theta_r, X, T = _setup(dims, rows, 1)
    net = B.MLP(*dims)
    net.set_params(theta)
    Y = net.forward(torch.tensor(X, dtype=torch.float32, device="cuda")).double().cpu().numpy()
    Yo, a, d = _forward_bounds(theta_r, X, dims)
    err = np.abs(Y - Yo)
    ratio = err / d["Y"]
    n_near = int((d["H1"] > 0).sum() + (d["H2"] > 0).sum())
    print("forward %s x %d: max |err| / bound %.3f, median bound / |Y| %.1e, activations next to a "
          "rounding tie %d of %d" % (dims, rows, ratio.max(), np.median(d["Y"] / (np.abs(Yo) + 1e-30)),
                                     n_near, a["H1"].size + a["H2"].size))
    assert (err <= d["Y"]).all(), np.unravel_index(np.argmax(ratio), ratio.shape)


@pytest.mark.parametrize("rows", [512, 3000])
def test_gradients_elementwise(B, rows):
    """Loss and every gradient entry against the bfloat16-precision oracle.  A weight
    gradient is a sum over the batch of products of a bfloat16 activation and a
    bfloat16 error; where the two sides round one of those to neighbouring bfloat16
    values (rare: next to a rounding tie), that one term moves by at most one bfloat16
    step (2^-7 of it), and such moves are sparse and of random sign.  The bar of each
    entry is therefore half a bfloat16 step (2^-9) of its scale S -- the sum of the
    absolute values of its terms, |H|^T |dZ| (column sums of |dZ| for the biases) --
    plus the FP32 accumulation bound gamma_rows S; the loss within its propagated
    bound.  The gradients themselves are 0.15-0.35 of S, so the bar is a few tenths
    of a percent of each entry."""
    dims = (17, 256, 15)
    theta, theta_r, X, T = _setup(dims, rows, 2)
    T = T.astype(np.float32).astype(np.float64)          # the device reads FP32 targets
    net = B.MLP(*dims)
    net.set_params(theta)
    L, g = net.loss_grad(torch.tensor(X, dtype=torch.float32, device="cuda"),
                         torch.tensor(T, dtype=torch.float32, device="cuda"), want_grad=True)
    g = g.astype(np.float64)
    Lo, go, a = omlp.loss_and_grad_bf16(theta_r, X, T, dims)
    _, _, d = _forward_bounds(theta_r, X, dims)
    n = rows * dims[2]
    res = np.abs(a["Y"] - T)
    # loss: FP32 squares of residuals within the forward bound, summed in blocks of 256
    assert abs(L - Lo) <= (np.sum(2 * res * d["Y"] + d["Y"] ** 2) + _gamma(256) * np.sum(res ** 2)) / n
    S = [np.abs(X).T @ np.abs(a["dZ1"]), np.abs(a["dZ1"]).sum(axis=0),
         np.abs(a["H1"]).T @ np.abs(a["dZ2"]), np.abs(a["dZ2"]).sum(axis=0),
         np.abs(a["H2"]).T @ np.abs(a["dY"]), np.abs(a["dY"]).sum(axis=0)]
    S = np.concatenate([x.ravel() for x in S])
    bound = (2.0 ** -9 + _gamma(rows)) * S + 1e-30
    err = np.abs(g - go)
    k = 0
    for name, sh in zip(("W1", "b1", "W2", "b2", "W3", "b3"), omlp.shapes(*dims)):
        m = int(np.prod(sh))
        print("gradient %s: max |err| / bound %.3f, median bound / |g| %.1e"
              % (name, (err[k:k + m] / bound[k:k + m]).max(),
                 np.median(bound[k:k + m] / (np.abs(go[k:k + m]) + 1e-30))))
        k += m
    assert (err <= bound).all(), int(np.argmax(err / bound))


@pytest.mark.parametrize("rows", [512, 3000])
def test_gradients_match_oracle(B, rows):
    dims = (17, 256, 15)
    theta, theta_r, X, T = _setup(dims, rows, 2)
    net = B.MLP(*dims)
    net.set_params(theta)
    L, g = net.loss_grad(torch.tensor(X, dtype=torch.float32, device="cuda"),
                         torch.tensor(T, dtype=torch.float32, device="cuda"), want_grad=True)
    Lo, go = omlp.loss_and_grad(theta_r, X, T, dims)
    assert L == pytest.approx(Lo, rel=2e-2)
    cos = float(np.dot(g, go) / (np.linalg.norm(g) * np.linalg.norm(go)))
    rel = float(np.linalg.norm(g - go) / np.linalg.norm(go))
    assert cos > 0.999 and rel < 5e-2, (cos, rel)
    # per block (each weight matrix and bias) as well
    k = 0
    for s in omlp.shapes(*dims):
        n = int(np.prod(s))
        gb, gob = g[k:k + n], go[k:k + n]
        assert np.linalg.norm(gb - gob) <= 0.1 * np.linalg.norm(gob) + 1e-12, s
        k += n


def test_adam_training_reduces_loss(B):
    """A smooth regression target is learned: loss drops by 10x in 300 steps."""
    dims = (17, 256, 15)
    g = np.random.default_rng(5)
    X = g.uniform(-1, 1, size=(4096, 17)).astype(np.float32)
    A = g.normal(size=(17, 15)) / 4
    T = np.tanh(X @ A) + 0.1 * np.sin(3 * X[:, :15])
    net = B.MLP(*dims)
    net.set_params(omlp.init_params(3, dims))
    Xd = torch.tensor(X, device="cuda")
    Td = torch.tensor(T, dtype=torch.float32, device="cuda")
    L0 = net.loss_grad(Xd, Td)
    for _ in range(300):
        net.loss_grad(Xd, Td)
        net.adam(1e-3)
    L1 = net.loss_grad(Xd, Td)
    assert L1 < 0.1 * L0, (L0, L1)


def test_fused_inference_matches_layerwise_forward(B):
    """The fused three-layer inference kernel (forward) and the layer-by-layer MFMA
    GEMMs of the training pass (loss_grad) see the same bf16 operands in the same
    accumulation order: their losses on the same batch agree to FP32 rounding."""
    dims = (17, 256, 15)
    theta, _, X, T = _setup(dims, 2500, 4)
    net = B.MLP(*dims)
    net.set_params(theta)
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    Td = torch.tensor(T, dtype=torch.float32, device="cuda")
    Y = net.forward(Xd).double().cpu().numpy()
    L_fused = float(np.mean((Y - T) ** 2))
    L_layer = net.loss_grad(Xd, Td)
    assert L_fused == pytest.approx(L_layer, rel=1e-5), (L_fused, L_layer)
    # after an Adam step the packed weights are refreshed
    net.adam(1e-3)
    Y2 = net.forward(Xd).double().cpu().numpy()
    assert np.abs(Y2 - Y).max() > 0
    L2 = net.loss_grad(Xd, Td)
    assert float(np.mean((Y2 - T) ** 2)) == pytest.approx(L2, rel=1e-5)
