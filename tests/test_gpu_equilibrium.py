"""The equilibrium comparison model (CP_Q_EQUILIBRIUM) on the GPU against the FP64
oracle's equilibrium model.

* the jump on 20000 random realisable cells, compared on the end state U + dt Q
  (relative to |U| + |dt Q|, as the kinetic source parity);
* 200 SSP-RK3 steps of the source-active jet in FP64: per-variable relative L2
  <= 1e-9 (the FP64 gate);
* the mixed path on the same jet: the mixed gates (gas state 1e-4, ice mu0 2e-2);
* on the GPU as in the oracle, the equilibrium model holds more condensed water
  than the kinetic model.
"""
import math

import numpy as np
import pytest

from paper_2504_20742_amd import inputs
from tests.test_gpu_parity import _cells, dev, host, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_20742_amd import binding
    binding.load()
    return binding


def _solver(B, m, c, prec=None):
    s = B.Solver(m, c, B.CP_FP64 if prec is None else prec)
    s.set_qmode(B.CP_Q_EQUILIBRIUM)
    return s


def test_equilibrium_jump_random_states(B, orc):
    nx, nr = 200, 100
    U = _cells(orc, nx * nr, seed=12).reshape(15, nr, nx)
    m, c = inputs.mesh(nx, nr), inputs.case()
    o = orc.Oracle(m, c)
    o.set_equilibrium(True)
    s = _solver(B, m, c)
    dt = 1e-7
    Qo = o.source(U, dt)
    Q = host(s.source(dev(U), dt))
    active = np.any(Qo != 0, axis=0)
    assert active.sum() > 5000
    assert np.array_equal(active, np.any(Q != 0, axis=0))
    err = np.abs(dt * (Q - Qo)) / (np.abs(U) + np.abs(dt * Qo) + 1e-300)
    print("equilibrium jump: %d active cells, max rel error %.2e, median %.2e"
          % (active.sum(), err.max(), np.median(err[:, active])))
    assert err.max() <= 1e-9
    s.close()


def test_equilibrium_200_steps_fp64(B, orc):
    m, c = inputs.sa1(1)
    o = orc.Oracle(m, c)
    o.set_equilibrium(True)
    Uo = o.init()
    to = o.run(Uo, 200)
    s = _solver(B, m, c)
    U = s.init()
    t = s.step_n(U, 200)
    assert t == pytest.approx(to, rel=1e-12)
    e = rel_l2(host(U), Uo)
    print("equilibrium, 200 FP64 steps: max per-variable rel L2 %.2e" % e.max())
    assert (e <= 1e-9).all(), e
    s.close()


def _condensed(U, faces):
    xf, rf = faces
    V = np.outer(np.diff(rf) * 0.5 * (rf[1:] + rf[:-1]), np.diff(xf))
    return float((V * 4.0 / 3.0 * math.pi * (1000.0 * U[8] + 917.0 * U[12])).sum())


def test_equilibrium_mixed_and_against_kinetics(B, orc):
    """Mixed path in equilibrium mode vs the FP64 oracle after 300 steps, and the
    condensed water of the equilibrium model above the kinetic model's."""
    steps = 300
    m, c = inputs.sa1(1)
    o = orc.Oracle(m, c)
    o.set_equilibrium(True)
    Uo = o.init()
    o.run(Uo, steps)
    s = _solver(B, m, c, B.CP_MIXED)
    U = s.init()
    s.step_n(U, steps)
    Ug = host(U)
    gas = max(rel_l2(Ug[[0, 3, 4]], Uo[[0, 3, 4]]).max(),
              np.sqrt(np.sum((Ug[1:3] - Uo[1:3]) ** 2) / np.sum(Uo[1:3] ** 2)))
    ice = rel_l2(Ug[9:10], Uo[9:10])[0]
    faces = s.faces()
    w_eq = _condensed(Ug, faces)
    s.close()
    k = B.Solver(m, c, B.CP_MIXED)
    Uk = k.init()
    k.step_n(Uk, steps)
    w_kin = _condensed(host(Uk), faces)
    k.close()
    print("mixed equilibrium vs FP64 oracle after %d steps: gas %.2e, ice mu0 %.2e; condensed water "
          "equilibrium %.4e vs kinetic %.4e" % (steps, gas, ice, w_eq, w_kin))
    assert gas <= 1e-4
    assert ice <= 2e-2
    assert w_eq > w_kin > 0
