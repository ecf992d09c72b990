"""Drift of droplets and crystals (cp_set_drift) on the GPU against the FP64
oracle's drift flux.

* the drift part of the residual (drift on minus off) on a source-active state
  with droplets and crystals, within 1e-10 of its own size;
* 200 FP64 steps of the source-active jet with drift: per-variable relative
  L2 <= 1e-9; the mixed path within the mixed gates;
* the duct refuses drift.
"""
import numpy as np
import pytest

from paper_2504_20742_amd import inputs
from tests.test_gpu_parity import dev, host, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_20742_amd import binding
    binding.load()
    return binding


@pytest.fixture(scope="module")
def state(orc):
    """The source-active jet after 150 oracle steps: droplets and crystals exist."""
    m, c = inputs.sa1(2)
    o = orc.Oracle(m, c)
    U = o.init()
    o.run(U, 150)
    assert (U[5] > 1.0).sum() > 50 and (U[9] > 1.0).sum() > 10
    return m, c, U


def test_drift_residual(B, orc, state):
    m, c, U = state
    o = orc.Oracle(m, c)
    s = B.Solver(m, c)
    R0g, R0o = host(s.residual(dev(U))), o.residual(U)
    o.set_drift(True)
    s.set_drift(True)
    Dg = host(s.residual(dev(U))) - R0g
    Do = o.residual(U) - R0o
    assert np.all(Do[:5] == 0.0) and np.all(Do[13:] == 0.0)
    for v in range(5, 13):
        scale = np.abs(Do[v]).max()
        assert scale > 0.0, v
        err = np.abs(Dg[v] - Do[v]).max() / scale
        print("drift residual, variable %d: max %.3e, rel err %.2e" % (v, scale, err))
        assert err <= 1e-10, v
    s.close()


def test_drift_200_steps_fp64(B, orc):
    m, c = inputs.sa1(1)
    o = orc.Oracle(m, c)
    o.set_drift(True)
    Uo = o.init()
    to = o.run(Uo, 200)
    s = B.Solver(m, c)
    s.set_drift(True)
    U = s.init()
    t = s.step_n(U, 200)
    assert t == pytest.approx(to, rel=1e-12)
    e = rel_l2(host(U), Uo)
    print("drift, 200 FP64 steps: max per-variable rel L2 %.2e" % e.max())
    assert (e <= 1e-9).all(), e
    s.close()


def test_drift_mixed(B, orc):
    steps = 300
    m, c = inputs.sa1(1)
    o = orc.Oracle(m, c)
    o.set_drift(True)
    Uo = o.init()
    o.run(Uo, steps)
    s = B.Solver(m, c, B.CP_MIXED)
    s.set_drift(True)
    U = s.init()
    s.step_n(U, steps)
    Ug = host(U)
    gas = max(rel_l2(Ug[[0, 3, 4]], Uo[[0, 3, 4]]).max(),
              np.sqrt(np.sum((Ug[1:3] - Uo[1:3]) ** 2) / np.sum(Uo[1:3] ** 2)))
    ice = rel_l2(Ug[9:10], Uo[9:10])[0]
    print("mixed with drift vs FP64 oracle after %d steps: gas %.2e, ice mu0 %.2e" % (steps, gas, ice))
    assert gas <= 1e-4 and ice <= 2e-2
    s.close()


def test_duct_refuses_drift(B):
    m = inputs.mesh(16, 1, geom=inputs.GEOM_QUASI1D,
                    bc=(inputs.BC_INFLOW, inputs.BC_COPY, inputs.BC_WALL, inputs.BC_WALL))
    m["area_x"] = np.ones(17)
    s = B.Solver(m, inputs.case(phase_change=0))
    with pytest.raises(B.ContrailError) as e:
        s.set_drift(True)
    assert e.value.code == B.CP_EUNSUPPORTED
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_particle_times_match_oracle(B, orc, prec):
    """Drag-law diagnostics (response time and Stokes number of droplets and
    crystals) on a source-active jet with particles, against the oracle."""
    m, c = inputs.sa1(2)
    o = orc.Oracle(m, c)
    U0 = o.init()
    o.run(U0, 150)
    s = B.Solver(m, c, B.CP_FP64 if prec == "fp64" else B.CP_MIXED)
    U = dev(U0, s.dtype)
    tau, St = s.particle_times(U)
    Uh = U.double().cpu().numpy()          # the state the library saw (FP32 in the mixed path)
    to, So = o.particle_times(np.ascontiguousarray(Uh))
    tau, St = tau.cpu().numpy(), St.cpu().numpy()
    assert (to > 0).sum() > 100
    assert np.allclose(tau, to, rtol=1e-12, atol=0.0)
    assert np.allclose(St, So, rtol=1e-12, atol=0.0)
    s.close()
