"""Pins of the oracle's two liquid populations (Sec. 2.2: soot-activated and
homogeneously nucleated droplets carried as two moment sets, each with its own
nucleation source, growth closure and freezing; variables 5..8 and 15..18).

What fixes the two-population model without comparing it with itself:
* without soot every droplet is homogeneous, so a run equals the one-population
  model's run with the liquid moved to 15..18, bit for bit;
* two populations of the same shape (one a multiple of the other) grow, evaporate
  and freeze like the single population of their sum (the r20 closure and the
  lognormal freezing closure depend only on moment ratios), instantaneously and
  sub-cycled;
* every activated soot particle is one new droplet of the soot-activated population,
  and both populations nucleate at the critical radius, summing to the
  one-population nucleation source;
* immersion freezing needs a soot core: homogeneous droplets freeze like a
  one-population liquid whose immersion freezing is switched off;
* total water is conserved; the extra moments are transported exactly like the
  first liquid set;
* only the soot-activated droplets' complete evaporation releases activated soot.
"""
import math

import numpy as np
import pytest

from paper_2504_20742_amd import inputs
from tests.test_oracle_pins import _cell, _lognormal

FPI = 4.0 / 3.0 * math.pi


def _bi(orc, m, c):
    o = orc.Oracle(m, c)
    o.set_bimodal(True)
    assert o.nv == 19
    return o


def _split(U15, frac_het, hom=None):
    """19-variable state: the liquid of U15 split into frac_het (soot-activated, 5..8)
    and the rest (homogeneous, 15..18), or given homogeneous moments."""
    U = np.concatenate([U15, np.zeros(4)])
    if hom is None:
        U[5:9] = frac_het * U15[5:9]
        U[15:19] = U15[5:9] - U[5:9]
    else:
        U[15:19] = hom
    return U


def _close(a, b, rel, floor=0.0):
    return abs(a - b) <= rel * max(abs(a), abs(b)) + floor


def test_no_soot_run_equals_one_population(orc):
    """Without soot (the hydrogen case of Sec. 4.3) all droplets nucleate
    homogeneously: the two-population run holds them in 15..18 and is otherwise the
    one-population run, bit for bit."""
    m, c = inputs.sa1(1, n_soot=0.0)
    o1 = orc.Oracle(m, c)
    U1 = o1.init()
    t1 = o1.run(U1, 150)
    o2 = _bi(orc, m, c)
    U2 = o2.init()
    t2 = o2.run(U2, 150)
    assert U1[5].max() > 0.0
    assert t1 == t2
    assert np.all(U2[5:9] == 0.0)
    assert np.array_equal(U2[15:19], U1[5:9])
    keep = [0, 1, 2, 3, 4, 9, 10, 11, 12, 13, 14]
    assert np.array_equal(U2[keep], U1[keep])


@pytest.mark.parametrize("T,S_l", [(230.0, 1.05), (230.0, 0.8), (262.0, 1.1), (262.0, 0.5)])
def test_proportional_populations_act_as_one(orc, T, S_l):
    """Eq. 16-21 and the freezing closure depend on moment ratios only: a liquid split
    30/70 into the two populations has the rates of the unsplit liquid (summed over
    the populations), and so has the sub-cycled integral.  A supersaturation of 5-10 %
    grows droplets larger than the critical radius with no nucleation (the barrier
    underflows exp), below one they evaporate (completely within dt at S_l = 0.5);
    230 K freezes, 262 K not."""
    m, c = inputs.sa0()
    o1 = orc.Oracle(m, c)
    o2 = _bi(orc, m, c)
    p = 23800.0
    L = orc.lib()
    pv = S_l * math.exp(L.or_ln_psat_liq(T))
    Y = pv / 461.52 / (pv / 461.52 + (p - pv) / 287.0)
    liq = _lognormal(3e9, 2e-7 if S_l > 0.6 else 2e-8, 1.4)
    U1 = _cell(orc, T=T, p=p, Y=Y, liq=liq, ice=_lognormal(1e8, 4e-7, 1.3))
    U2 = _split(U1, 0.3)
    S1, d1 = o1.rates_cell(U1)
    S2, d2 = o2.rates_cell(U2)
    assert d1["Jhom"] == 0.0 and d1["Jhet"] == 0.0
    assert (d1["Gl"] > 0) == (S_l > 1)
    assert (d1["mdot_f"] > 0) == (T < 273.15)
    for k in range(4):
        assert _close(S2[5 + k] + S2[15 + k], S1[5 + k], 1e-12), k
        assert _close(S2[5 + k], 0.3 * S1[5 + k], 1e-12), k
    for v in list(range(5)) + list(range(9, 15)):
        assert _close(S2[v], S1[v], 1e-12, 1e-300), v
    for dt in (1e-7, 1e-5, 1e-3):
        Q1, n1 = o1.source_cell(U1, dt)
        Q2, n2 = o2.source_cell(U2, dt)
        assert n1 == n2
        # end states rebuilt as U + dt Q carry a rounding of |U| (a population that
        # evaporates completely ends at that level, not at zero)
        E1, E2 = U1 + dt * Q1, U2 + dt * Q2
        for k in range(4):
            assert _close(E2[5 + k] + E2[15 + k], E1[5 + k], 1e-11, 1e-14 * abs(U1[5 + k])), (dt, k)
        for v in list(range(5)) + list(range(9, 15)):
            assert _close(E2[v], E1[v], 1e-11, 1e-14 * abs(U1[v])), (dt, v)
    if S_l < 0.6:   # evaporated completely
        assert abs(E1[8]) <= 1e-15 * U1[8] and abs(E2[8] + E2[18]) <= 1e-15 * U1[8]


def test_nucleation_routing(orc):
    """Eq. 4-10: new droplets appear at the critical radius in both populations; the
    soot-activated population gains exactly the activated soot number; the two
    nucleation sources sum to the one-population source."""
    m, c = inputs.sa0()
    o1 = orc.Oracle(m, c)
    o2 = _bi(orc, m, c)
    T, p = 225.0, 23800.0
    L = orc.lib()
    pv = 9.0 * math.exp(L.or_ln_psat_liq(T))
    Y = pv / 461.52 / (pv / 461.52 + (p - pv) / 287.0)
    U1 = _cell(orc, T=T, p=p, Y=Y, ns=1e13)
    U2 = _split(U1, 0.0)
    S1, d1 = o1.rates_cell(U1, h=1e-3)
    S2, d2 = o2.rates_cell(U2, h=1e-3)
    assert d1["Jhom"] > 0 and d1["Jhet"] > 0 and S2[14] > 0 and S2[15] > 0
    assert S2[5] == S2[14]
    assert _close(S2[5] + S2[15], S1[5], 1e-14)
    for k in range(1, 4):
        assert _close(S2[5 + k] / S2[5], S2[15 + k] / S2[15], 1e-14)
        assert _close(S2[5 + k] + S2[15 + k], S1[5 + k], 1e-14)
    for v in (0, 3, 4, 14):
        assert _close(S2[v], S1[v], 1e-13)


def test_immersion_freezing_needs_a_soot_core(orc):
    """Sec. 2.2 immersion freezing acts through the soot inside a droplet:
    homogeneously nucleated droplets freeze at the homogeneous (Koop) rate only, like a
    one-population liquid with immersion switched off (n_s = 0); the same droplets in
    the soot-activated population freeze like the one-population liquid."""
    m, c = inputs.sa0()
    c_noimm = dict(c, n_s=0.0)
    T, p = 238.0, 23800.0
    liq = _lognormal(2e9, 3e-7, 1.5)
    U1 = _cell(orc, T=T, p=p, Y=2e-4, liq=liq, ns=1e13, na=2e9)
    S_imm = orc.Oracle(m, c).rates_cell(U1)[0]
    S_no = orc.Oracle(m, c_noimm).rates_cell(U1)[0]
    o2 = _bi(orc, m, c)
    S_het = o2.rates_cell(_split(U1, 1.0))[0]
    S_hom = o2.rates_cell(_split(U1, 0.0))[0]
    assert S_imm[12] != S_no[12]                 # immersion freezing matters here
    for k in range(4):
        assert S_het[5 + k] == S_imm[5 + k]
        assert S_hom[15 + k] == S_no[5 + k]
        assert S_het[15 + k] == 0.0 and S_hom[5 + k] == 0.0
    for v in list(range(5)) + [9, 10, 11, 12]:
        assert S_het[v] == S_imm[v]
        assert S_hom[v] == S_no[v]


def test_water_conserved_two_populations(orc):
    """Eq. 25-26 with two liquid populations: the vapour sink balances the condensed
    water of both populations and the ice, instantaneous and sub-cycled."""
    m, c = inputs.sa0()
    o = _bi(orc, m, c)
    a = inputs.random_cells(150, seed=21)
    b = inputs.random_cells(150, seed=22)
    worst = 0.0
    for k in range(150):
        U1 = _cell(orc, T=a["T"][k], p=a["p"][k], Y=a["Y"][k], liq=a["liq"][:, k], ice=a["ice"][:, k],
                   ns=a["n_soot"][k], na=a["n_act"][k])
        U = _split(U1, None, hom=b["liq"][:, k])
        S = o.rates_cell(U)[0]
        cond = FPI * (1000.0 * (S[8] + S[18]) + 917.0 * S[12])
        worst = max(worst, abs(S[4] + cond) / (abs(S[4]) + abs(cond) + 1e-300))
        dt = 1e-5
        Q, _ = o.source_cell(U, dt)
        E = U + dt * Q
        w0 = U[4] + FPI * (1000.0 * (U[8] + U[18]) + 917.0 * U[12])
        w1 = E[4] + FPI * (1000.0 * (E[8] + E[18]) + 917.0 * E[12])
        worst = max(worst, abs(w1 - w0) / w0 * 1e-2)
        idx = [5, 6, 7, 8, 15, 16, 17, 18]
        assert np.all(E[idx] >= -1e-14 * np.abs(U[idx]))   # non-negative up to the U + dt Q rounding
    assert worst < 1e-12


def test_second_population_transported_like_the_first(orc):
    """The homogeneous moments are passive scalars of the same kind as the first
    liquid set: started equal to it, they have the same residual and stay equal,
    and the other variables are those of the one-population run."""
    m, c = inputs.sa1(2)
    o1 = orc.Oracle(m, c)
    U1 = o1.init()
    o1.run(U1, 120)
    assert (U1[5] > 1.0).sum() > 50
    c0 = dict(c, phase_change=0)
    p1 = orc.Oracle(m, c0)
    p2 = _bi(orc, m, c0)
    U2 = np.concatenate([U1, U1[5:9]])
    R1, R2 = p1.residual(U1), p2.residual(U2)
    assert np.array_equal(R2[15:19], R2[5:9])
    assert np.array_equal(R2[:15], R1)
    t1 = p1.run(U1, 25)
    t2 = p2.run(U2, 25)
    assert t1 == t2
    assert np.array_equal(U2[15:19], U2[5:9])
    assert np.array_equal(U2[:15], U1)


def test_bimodal_refuses_one_population_models(orc):
    """The equilibrium comparison model and the drift flux are defined for one
    liquid population: the switches refuse each other."""
    m, c = inputs.sa1(1)
    o = orc.Oracle(m, c)
    o.set_equilibrium(True)
    with pytest.raises(ValueError):
        o.set_bimodal(True)
    o.set_equilibrium(False)
    o.set_drift(True)
    with pytest.raises(ValueError):
        o.set_bimodal(True)
    o.set_drift(False)
    o.set_bimodal(True)
    with pytest.raises(ValueError):
        o.set_equilibrium(True)
    with pytest.raises(ValueError):
        o.set_drift(True)
    o.set_bimodal(False)
    assert o.nv == 15


def test_only_soot_activated_evaporation_releases_soot(orc):
    """Complete evaporation (R43): when the homogeneous droplets evaporate and the
    soot-activated ones survive, the activated soot stays activated; when the
    soot-activated droplets evaporate completely, their soot is released (N_act -> 0)
    even while homogeneous droplets survive."""
    m, c = inputs.sa0()
    o = _bi(orc, m, c)
    T, p = 262.0, 23800.0
    L = orc.lib()
    pv = 0.5 * math.exp(L.or_ln_psat_liq(T))
    Y = pv / 461.52 / (pv / 461.52 + (p - pv) / 287.0)
    small = _lognormal(1e9, 1e-8, 1.2)      # evaporates within dt
    large = _lognormal(1e8, 5e-6, 1.2)      # survives
    na = 1e8
    dt = 1e-3
    # homogeneous small, soot-activated large
    U = _split(_cell(orc, T=T, p=p, Y=Y, liq=large, ns=1e12, na=na), None, hom=small)
    Q, _ = o.source_cell(U, dt)
    E = U + dt * Q
    assert abs(E[18]) <= 1e-15 * U[18] and E[8] > 0.5 * U[8]
    assert E[14] == pytest.approx(U[14], rel=1e-12)
    # soot-activated small, homogeneous large
    U = _split(_cell(orc, T=T, p=p, Y=Y, liq=small, ns=1e12, na=na), None, hom=large)
    Q, _ = o.source_cell(U, dt)
    E = U + dt * Q
    assert abs(E[8]) <= 1e-15 * U[8] and E[18] > 0.5 * U[18]
    assert abs(E[14]) <= 1e-12 * U[14]
