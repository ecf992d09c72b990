"""Host-side logic of the surrogate trainer: the normalisation block layout that
cp_sur_set reads, the envelope, the target standardisation and the initialiser."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2504_20742_amd import surrogate as S


def _data(n=500, seed=0):
    g = np.random.default_rng(seed)
    X = torch.tensor(g.normal(size=(n, 17)) * np.arange(1, 18) + np.arange(17), dtype=torch.float32)
    X[:, 16] = 3.0                     # a constant feature
    D = torch.zeros((n, 15), dtype=torch.float32)
    for v in S.NET_VARS:
        D[:, v] = torch.tensor(g.normal(size=n) * (v + 1) + 0.5, dtype=torch.float32)
    lnS = torch.tensor(g.uniform(-3, 2, size=n), dtype=torch.float32)
    dt = torch.full((n,), 1e-6, dtype=torch.float64)
    return S.Dataset(X, D, lnS, dt)


def test_norm_block_layout():
    d = _data()
    nm = S.Norm(d, lnS_gate=0.05)
    p = nm.pack()
    assert p.dtype == np.float32 and p.size == S.N_NORM == 118
    o = 0
    for name, k in (("s_in", 15), ("mu_in", 17), ("sd_in", 17), ("lo", 17), ("hi", 17), ("mu_out", 15),
                    ("sd_out", 15)):
        assert np.allclose(p[o:o + k], getattr(nm, name)), name
        o += k
    assert np.allclose(p[o:], [0.05, float(d.lnS.min()), float(d.lnS.max()), 0.2, 0.01])


def test_norm_statistics_and_envelope():
    d = _data()
    nm = S.Norm(d)
    Z = nm.inputs(d.X).double().numpy()
    # standardised features: zero mean, unit spread, inside [lo, hi]; constant feature kept at 0
    assert np.allclose(Z[:, :16].mean(0), 0, atol=1e-5)
    assert np.allclose(Z[:, :16].std(0, ddof=1), 1, atol=1e-4)
    assert nm.sd_in[16] == 1.0 and np.all(Z[:, 16] == 0)
    assert np.all(Z >= nm.lo - 1e-6) and np.all(Z <= nm.hi + 1e-6)
    assert np.allclose(nm.lo, Z.min(0), atol=1e-5) and np.allclose(nm.hi, Z.max(0), atol=1e-5)
    T = nm.targets(d.D)
    back = nm.decode(T)
    assert torch.allclose(back, d.D, atol=1e-5)
    for v in range(15):
        if v not in S.NET_VARS:
            assert nm.mu_out[v] == 0 and nm.sd_out[v] == 1


def test_split_is_a_partition():
    d = _data(1000)
    a, b = d.split(0.1, seed=3)
    assert len(a) + len(b) == 1000 and len(b) == 100
    rows = {tuple(r) for r in torch.cat([a.X, b.X]).numpy().round(6)}
    assert len(rows) == len({tuple(r) for r in d.X.numpy().round(6)})


def test_init_params_shapes_and_scale():
    p = S.init_params(0)
    n = 17 * 256 + 256 + 256 * 256 + 256 + 256 * 15 + 15
    assert p.size == n and p.dtype == np.float32
    W2 = p[17 * 256 + 256:17 * 256 + 256 + 256 * 256]
    assert abs(W2.std() - np.sqrt(2.0 / 256)) < 0.01 * np.sqrt(2.0 / 256) * 10
    b1 = p[17 * 256:17 * 256 + 256]
    assert np.all(b1 == 0)
    assert np.array_equal(p, S.init_params(0)) and not np.array_equal(p, S.init_params(1))


def test_feature_scales_positive():
    assert S.S_IN.shape == (15,) and np.all(S.S_IN > 0)
