"""The allocation-free network inference entry point (cp_mlp_forward_static) against
cp_mlp_forward, through the C ABI: the same kernels on the same inputs, so the
outputs must be equal bit for bit.  Two calls in a row with different networks,
the second on fewer rows, show that each call repacks its own weights into the
shared static scratch and that no state of the first call leaks into the second."""
import ctypes

import numpy as np
import pytest

from paper_2504_20742_amd import binding

pytestmark = pytest.mark.gpu

MAX_ROWS = 65536


def _net(seed):
    from oracle import mlp as omlp
    net = binding.MLP(17, 256, 15)
    theta = omlp.init_params(seed)
    g = np.random.default_rng(seed)
    theta = theta + 0.05 * g.normal(size=theta.size)   # non-zero biases too
    net.set_params(theta.astype(np.float32))
    return net


def test_static_forward_equals_forward():
    import torch
    torch.cuda.set_device(0)
    print("no-alloc: two networks, 5000 then 1234 rows", flush=True)
    A, B = _net(3), _net(4)
    g = torch.Generator(device="cpu").manual_seed(7)
    X1 = torch.randn((5000, 17), generator=g).cuda()
    X2 = torch.randn((1234, 17), generator=g).cuda()
    Y1 = A.forward_static(X1)
    torch.cuda.synchronize()
    Y1r = A.forward(X1)
    Y2 = B.forward_static(X2)
    torch.cuda.synchronize()
    Y2r = B.forward(X2)
    torch.cuda.synchronize()
    assert torch.isfinite(Y1).all() and torch.isfinite(Y2).all()
    assert torch.equal(Y1, Y1r)
    assert torch.equal(Y2, Y2r)
    # the first network again on the smaller input: its weights are packed anew
    Y3 = A.forward_static(X2)
    torch.cuda.synchronize()
    assert torch.equal(Y3, A.forward(X2))
    assert not torch.equal(Y3, Y2)
    # the largest allowed batch
    X4 = torch.randn((MAX_ROWS, 17), generator=g).cuda()
    Y4 = B.forward_static(X4)
    torch.cuda.synchronize()
    assert torch.equal(Y4, B.forward(X4))


def test_static_forward_refuses_sizes_beyond_the_scratch():
    import torch
    torch.cuda.set_device(0)
    net = _net(5)
    X = torch.zeros((4, 17), device="cuda")
    L = net.L
    Y = torch.empty((4, 15), device="cuda")
    assert L.cp_mlp_forward_static(net.h, X.data_ptr(), MAX_ROWS + 1, Y.data_ptr()) == binding.CP_EINVAL
    assert b"65536" in L.cp_mlp_error_string(net.h)
    assert L.cp_mlp_forward_static(net.h, X.data_ptr(), 0, Y.data_ptr()) == binding.CP_EINVAL
    assert L.cp_mlp_forward_static(net.h, None, 4, Y.data_ptr()) == binding.CP_EINVAL
    other = binding.MLP(17, 64, 15)      # not the fused inference shape
    assert L.cp_mlp_forward_static(other.h, X.data_ptr(), 4, Y.data_ptr()) == binding.CP_EUNSUPPORTED
