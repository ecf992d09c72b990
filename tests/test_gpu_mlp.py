"""BF16 MFMA surrogate network against its FP64 oracle (oracle/mlp.py).

The GPU rounds weights, inputs and hidden activations to bfloat16 and accumulates
in FP32; the oracle runs in FP64 on the same bf16-rounded weights and inputs.
Bars: forward relative L2 <= 2e-2; loss within 2e-2; gradient relative L2
<= 5e-2 with cosine similarity > 0.999 (bf16 activations bound the agreement)."""
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
