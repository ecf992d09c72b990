"""Tabulated water properties (cp_set_property_table) on the GPU against the FP64
oracle reading its own table of the same spacing.

* the kinetic source on 20000 random realisable cells, end states within 1e-9 of
  |U| + |dt Q| (the bound of the closed-form source parity);
* 200 FP64 steps of the source-active jet with a 0.25 K table: per-variable
  relative L2 <= 1e-9; the equilibrium model on the same table likewise;
* the table changes the run only at its interpolation error (against the
  closed-form run), and spacing 0 returns to the closed forms bit for bit.
"""
import numpy as np
import pytest

from paper_2504_20742_amd import inputs
from tests.test_gpu_parity import _cells, dev, host, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

H = 0.25


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_20742_amd import binding
    binding.load()
    return binding


def test_table_source_random_states(B, orc):
    nx, nr = 200, 100
    U = _cells(orc, nx * nr, seed=13).reshape(15, nr, nx)
    m, c = inputs.mesh(nx, nr), inputs.case()
    o = orc.Oracle(m, c)
    o.set_property_table(H)
    s = B.Solver(m, c)
    s.set_property_table(H)
    dt = 1e-7
    Qo = o.source(U, dt)
    Q = host(s.source(dev(U), dt))
    err = np.abs(dt * (Q - Qo)) / (np.abs(U) + np.abs(dt * Qo) + 1e-300)
    print("table source: max rel error %.2e" % err.max())
    assert err.max() <= 1e-9
    with pytest.raises(B.ContrailError) as e:
        s.set_property_table(-1.0)
    assert e.value.code == B.CP_EINVAL
    s.close()


@pytest.mark.parametrize("equilibrium", [False, True])
def test_table_200_steps_fp64(B, orc, equilibrium):
    m, c = inputs.sa1(2)
    o = orc.Oracle(m, c)
    o.set_property_table(H)
    o.set_equilibrium(equilibrium)
    Uo = o.init()
    to = o.run(Uo, 200)
    s = B.Solver(m, c)
    s.set_property_table(H)
    if equilibrium:
        s.set_qmode(B.CP_Q_EQUILIBRIUM)
    U = s.init()
    t = s.step_n(U, 200)
    assert t == pytest.approx(to, rel=1e-12)
    e = rel_l2(host(U), Uo)
    print("table, equilibrium=%s, 200 FP64 steps: max per-variable rel L2 %.2e" % (equilibrium, e.max()))
    assert (e <= 1e-9).all(), e
    s.close()


def test_table_against_closed_forms(B):
    m, c = inputs.sa1(2)
    res = {}
    for h in (0.0, H, 0.0):
        s = B.Solver(m, c)
        s.set_property_table(H)
        s.set_property_table(h)          # setting 0 after a table restores the closed forms
        U = s.init()
        s.step_n(U, 100)
        res.setdefault(h, []).append(host(U))
        s.close()
    assert np.array_equal(res[0.0][0], res[0.0][1])
    e = rel_l2(res[H][0], res[0.0][0])
    print("0.25 K table vs closed forms after 100 steps: max per-variable rel L2 %.2e" % e.max())
    assert e.max() < 1e-4
