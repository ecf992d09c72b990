"""The measured workloads run at their stated lengths and sizes, against the oracle.

* The source-active jet on the production mesh (2048 x 512, stretched and clustered,
  hydrogen-like core water, cold bypass): 200 FP64 steps through cp_step_n -- the
  captured graph, the autotuned tile, the compacted list of source-active cells at
  full size -- against 200 oracle steps, per-variable relative L2 <= 1e-9.
* The mixed path on the source-active 96 x 48 jet for 5000 steps: the mixed gates
  (gas state 1e-4, ice number 2e-2, total water 1e-4) against the oracle.
* 64 plumes of uneven size (256 x 64 to 1024 x 256, emission index up to 9) for 2000
  mixed steps in one batch: every plume finite and realisable, within the mixed gates
  of the same batch run in FP64 (the FP64 path is the one matched to the oracle), and
  two plumes equal bit for bit to the same plumes run alone.  With the 250 K bypass of
  this workload the wettest plumes become supersaturated (ln S_l up to about 0.5, so
  their source is active and nucleation starts) but within 2000 steps the nucleated
  number stays far below one droplet per m^3; the number gates apply to populations
  above 1 m^-3, of which this workload has none.
"""
import threading

import numpy as np
import pytest

from paper_2504_20742_amd import inputs
from tests.test_gpu_parity import host, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_20742_amd import binding
    binding.load()
    return binding


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.abs(a).max()


def _gas(a, b):
    mom = np.sqrt(np.sum((a[1:3] - b[1:3]) ** 2) / np.sum(b[1:3] ** 2))
    return max(_rel(a[0], b[0]), _rel(a[3], b[3]), _rel(a[4], b[4]), mom)


def _water(U, dx, rdr):
    w = U[4] + 4.0 / 3.0 * np.pi * (1000.0 * U[8] + 917.0 * U[12])
    return float((w * rdr[:, None] * dx[None, :]).sum())


def test_source_active_production_mesh_200_fp64_steps(B, orc):
    m, c = inputs.sa2(0)
    print("configs: source-active jet 2048x512, 200 FP64 steps (oracle on the host meanwhile)", flush=True)
    o = orc.Oracle(m, c)
    Uo = o.init()
    res = {}
    th = threading.Thread(target=lambda: res.update(t=o.run(Uo, 200)))
    th.start()
    s = B.Solver(m, c, B.CP_FP64)
    U = s.init()
    t = s.step_n(U, 200)
    d = s.diag(U)
    Ug = host(U)
    s.close()
    th.join()
    print("active cells %d, max ln S_l %.2f" % (d["active_cells"], d["max_lnS_l"]), flush=True)
    assert d["active_cells"] > 1000                   # the compacted source list is live
    assert t == pytest.approx(res["t"], rel=1e-12)
    e = rel_l2(Ug, Uo)
    print("per-variable rel L2: %s" % " ".join("%.1e" % x for x in e))
    assert Uo[9].max() > 0 and Uo[5].max() > 0        # droplets and crystals present
    assert (e <= 1e-9).all(), e


def test_mixed_source_active_5000_steps(B, orc):
    m, c = inputs.sa1(1)
    print("configs: source-active jet 96x48, 5000 mixed steps", flush=True)
    o = orc.Oracle(m, c)
    Uo = o.init()
    to = o.run(Uo, 5000)
    s = B.Solver(m, c, B.CP_MIXED)
    U = s.init()
    t = s.step_n(U, 5000)
    Ug = host(U)
    s.close()
    gas, ice = _gas(Ug, Uo), _rel(Ug[9], Uo[9])
    wo, wg = o.diag(Uo)["water"], o.diag(Ug)["water"]
    print("after 5000 steps: gas %.2e  ice mu0 %.2e  water %.2e  t %.4e / %.4e"
          % (gas, ice, abs(wg - wo) / wo, t, to))
    assert Uo[9].max() > 0
    assert abs(t - to) / to < 1e-4
    assert gas <= 1e-4
    assert ice <= 2e-2
    assert abs(wg - wo) / wo <= 1e-4


def test_config4_batch_2000_mixed_steps(B):
    cases = inputs.config4(seed=0)
    ms, cs = [m for m, _ in cases], [c for _, c in cases]
    print("configs: 64 plumes, 2000 steps mixed and FP64", flush=True)
    bm = B.Batch(ms, cs, B.CP_MIXED)
    Um = bm.init()
    tm = bm.step_n(Um, 2000)
    bd = B.Batch(ms, cs, B.CP_FP64)
    Ud = bd.init()
    td = bd.step_n(Ud, 2000)
    worst = {"gas": 0.0, "liquid_mu0": 0.0, "ice_mu0": 0.0, "water": 0.0}
    nucleating, populated = 0, 0
    for p, (m, c) in enumerate(cases):
        a, b = host(Um[p]), host(Ud[p])
        assert np.isfinite(a).all(), p
        for base in (5, 9):     # realisable particle sets: non-negative moments
            M = a[base:base + 4]
            assert (M >= -1e-6 * np.abs(M).max(axis=(1, 2), keepdims=True) - 1e-300).all(), (p, base)
        assert (a[4] >= -1e-9 * a[4].max()).all(), p
        assert abs(tm[p] - td[p]) / td[p] < 1e-4, p
        # water per plume (vapour + condensate, per radian of the axisymmetric mesh)
        s = B.Solver(m, c, B.CP_FP64)
        xf, rf = s.faces()
        s.close()
        dx, rdr = xf[1:] - xf[:-1], (rf[1:] - rf[:-1]) * 0.5 * (rf[1:] + rf[:-1])
        wa, wb = _water(a, dx, rdr), _water(b, dx, rdr)
        worst["gas"] = max(worst["gas"], _gas(a, b))
        worst["water"] = max(worst["water"], abs(wa - wb) / wb)
        nucleating += int(b[5].max() > 0)
        for v, key in ((5, "liquid_mu0"), (9, "ice_mu0")):
            if b[v].max() > 1.0:
                populated += 1
                worst[key] = max(worst[key], _rel(a[v], b[v]))
    print("2000 steps, mixed vs FP64 over the plumes: %s; %d plumes nucleating, %d populations above 1/m^3"
          % (worst, nucleating, populated))
    assert nucleating > 0                                  # the source is live in the batch
    assert worst["gas"] <= 1e-4 and worst["water"] <= 1e-4
    assert worst["liquid_mu0"] <= 2e-2 and worst["ice_mu0"] <= 2e-2
    # two plumes (the smallest mesh, the lowest and the highest emission index) alone
    small = [p for p, (m, _) in enumerate(cases) if m["nx"] == 256]
    ei = [cases[p][1]["Y_core"] for p in small]
    for p in (small[int(np.argmin(ei))], small[int(np.argmax(ei))]):
        s = B.Solver(cases[p][0], cases[p][1], B.CP_MIXED)
        s.set_tile(32, 8)
        U = s.init()
        t = s.step_n(U, 2000)
        assert t == tm[p]
        assert torch.equal(U, Um[p]), p
        s.close()
    bm.close()
    bd.close()
