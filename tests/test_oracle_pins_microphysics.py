"""Pins of the oracle's phase-change source against the paper's printed formulas.

Each test writes the printed relation of the passage it pins (Sec. 2.2, Eq. 14-16
and 19-21; Sec. 3.1, Eq. 22-26) with the constants the paper fixes, read from
tests/golden/paper_values.json, and compares the oracle's instantaneous source
(``or_source_rates_cell``) against it.  The readings where the paper is silent
(conductivity from the Prandtl number, Young's mean free path, the vapour's gamma
and c_p in nu, the rate scale of Eq. 14) are stated beside each use.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2504_20742_amd import inputs
from tests.test_oracle_pins import _cell, _lognormal

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))

# gas model of the solver (calorically perfect dry air and vapour, Sec. 4.1 air
# composition; vapour as an ideal triatomic gas) and the water constants at 0 C
R_A, CP_A = 287.0, 1004.5
R_V, CP_V, GAMMA_V = 461.52, 1846.08, 4.0 / 3.0
T0 = 273.15
L_VAP0, L_SUB0 = 2.5008e6, 2.8345e6
C_L, C_I = 4218.0, 2106.0
RHO_L, RHO_I = 1000.0, 917.0
PR_GAS, PR_V = 0.71, 1.0          # readings: gas conductivity c_p mu / Pr; Pr of Eq. 16
Q_C = 1.0                         # reading: condensation coefficient


def _sutherland(T):
    """Sutherland's law for air (mu_ref 1.716e-5 Pa s at 273.15 K, S = 110.4 K)."""
    return 1.716e-5 * (T / 273.15) ** 1.5 * (273.15 + 110.4) / (T + 110.4)


def _h_fg(T):
    return L_VAP0 + (CP_V - C_L) * (T - T0)


def _h_sg(T):
    return L_SUB0 + (CP_V - C_I) * (T - T0)


def _gas(orc, U):
    W = orc.cons_to_prim(U.copy())
    rho, p, Y, T = W[0], W[3], W[4], W[15]
    R = (1 - Y) * R_A + Y * R_V
    cp = (1 - Y) * CP_A + Y * CP_V
    return dict(rho=rho, p=p, Y=Y, T=T, R=R, cp=cp, rho_v=U[4])


def _young_G(r, T, p, R, cp, dT, h, rho_p, Tsat, r_crit, alpha, beta):
    """Eq. 16 as printed: G = lambda_g dT (1 - r_crit / r) /
    (rho_p h r (1 / (1 + 2 beta Kn) + 3.78 (1 - nu) Kn / Pr)), with
    nu = R_s T_sat / h (alpha - 1/2 - (2 - q_c)/(2 q_c) (gamma+1)/(2 gamma) c_p T_sat / h),
    Kn = lbar / (2 r).  r_crit = 0 drops the Kelvin factor (ice, no Kelvin term)."""
    mu = _sutherland(T)
    lam = cp * mu / PR_GAS
    lbar = 1.5 * mu * math.sqrt(R * T) / p
    Kn = lbar / (2.0 * r)
    nu = R_V * Tsat / h * (alpha - 0.5 - (2.0 - Q_C) / (2.0 * Q_C) * (GAMMA_V + 1.0) / (2.0 * GAMMA_V)
                           * CP_V * Tsat / h)
    return lam * dT * (1.0 - r_crit / r) / (rho_p * h * r * (1.0 / (1.0 + 2.0 * beta * Kn)
                                                             + 3.78 * (1.0 - nu) * Kn / PR_V))


def _y_at(orc, T, p, lnS, ice=False):
    L = orc.lib()
    lnps = L.or_ln_psat_ice(T) if ice else L.or_ln_psat_liq(T)
    pv = math.exp(lnps + lnS)
    rho_v, rho_a = pv / (R_V * T), (p - pv) / (R_A * T)
    return rho_v / (rho_a + rho_v)


def _lbar(T, p, Y):
    R = (1 - Y) * R_A + Y * R_V
    return 1.5 * _sutherland(T) * math.sqrt(R * T) / p


def _sigma_iapws(T):
    tau = 1.0 - T / 647.096
    return 0.2358 * tau ** 1.256 * (1.0 - 0.625 * tau)


@pytest.mark.parametrize("T", [238.0, 262.0])
@pytest.mark.parametrize("Kn", [1.0, 3.0, 10.0])
def test_droplet_growth_is_young_eq16(orc, T, Kn):
    """Eq. 16 on the full rate path: a monodisperse droplet population in
    supersaturated vapour (S_l = 1.4) grows at Young's rate with alpha and beta as
    printed (golden 11 and 0) at Knudsen numbers 1-10, where the (1 - nu) Kn term
    dominates the denominator; T_sat from the inverted Sonntag law, the Kelvin
    factor with r_crit of Eq. 3."""
    L = orc.lib()
    p = 23800.0
    Y = _y_at(orc, T, p, math.log(1.4))
    r = _lbar(T, p, Y) / (2.0 * Kn)
    N = 1e9
    m, c = inputs.sa0(n_soot=0.0)
    o = orc.Oracle(m, c)
    U = _cell(orc, T=T, p=p, Y=Y, liq=[N * r ** k for k in range(4)])
    S, d = o.rates_cell(U)
    g = _gas(orc, U)
    pv = g["rho_v"] * R_V * g["T"]
    Tsat = L.or_tsat_liq(pv, g["T"])
    lnS = math.log(pv) - L.or_ln_psat_liq(g["T"])
    rc = 2.0 * _sigma_iapws(g["T"]) / (RHO_L * R_V * g["T"] * lnS)
    G = _young_G(r, g["T"], g["p"], g["R"], g["cp"], Tsat - g["T"], _h_fg(g["T"]), RHO_L, Tsat, rc,
                 GOLD["young_alpha"]["value"], GOLD["young_beta"]["value"])
    assert G > 0
    assert d["Gl"] == pytest.approx(G, rel=1e-10)
    assert d["rcrit"] == pytest.approx(rc, rel=1e-12)


@pytest.mark.parametrize("T", [215.0, 245.0])
@pytest.mark.parametrize("Kn", [1.0, 10.0])
def test_crystal_growth_is_young_eq16_with_ice_properties(orc, T, Kn):
    """Eq. 16 for crystals (Sec. 2.2: growth "analogous" with the solid phase's
    properties): h_sg, rho_s, T_sat over ice, no Kelvin factor; the vapour is
    supersaturated over ice and subsaturated over liquid, so nothing nucleates."""
    L = orc.lib()
    p = 23800.0
    Y = _y_at(orc, T, p, math.log(1.15), ice=True)
    r = _lbar(T, p, Y) / (2.0 * Kn)
    m, c = inputs.sa0(n_soot=0.0)
    o = orc.Oracle(m, c)
    U = _cell(orc, T=T, p=p, Y=Y, ice=[2e8 * r ** k for k in range(4)])
    S, d = o.rates_cell(U)
    assert d["lnSl"] < 0 < d["lnSi"]
    g = _gas(orc, U)
    pv = g["rho_v"] * R_V * g["T"]
    Tsat = L.or_tsat_ice(pv, g["T"])
    G = _young_G(r, g["T"], g["p"], g["R"], g["cp"], Tsat - g["T"], _h_sg(g["T"]), RHO_I, Tsat, 0.0,
                 GOLD["young_alpha"]["value"], GOLD["young_beta"]["value"])
    assert G > 0
    assert d["Gs"] == pytest.approx(G, rel=1e-10)


def test_immersion_freezing_rate_eq14_15(orc):
    """Eq. 14-15 with n_s = 1e8 m^-2 (golden): the soot surface sum_i n_p,i 4 pi r_p,i^2
    of the lognormal soot (by quadrature) times n_s gives the immersion-freezing rate
    (with the rate scale k_imm = 1/s, the reading that makes Eq. 15 a rate); a
    droplet of radius r freezes the mass rho_l V (the reading that conserves water),
    so the frozen-mass rate of a monodisperse population is
    rho_l (4 pi/3)^2 J n r^6.  The soot's share is isolated as the difference of the
    same cell with and without soot, which removes the homogeneous (Koop) share."""
    ns = GOLD["surface_site_density_m2"]["value"]
    N_soot, rg, sg = 3e12, 15e-9, 1.6
    T, p = 262.0, 23800.0
    Y = _y_at(orc, T, p, math.log(0.9))       # subsaturated: no nucleation
    Nl, rl = 5e8, 2e-6
    liq = [Nl * rl ** k for k in range(4)]
    m, c = inputs.sa0(n_soot=N_soot)
    c.update(n_s=ns, k_imm=1.0, r_g_soot=rg, sigma_g_soot=sg)
    o = orc.Oracle(m, c)
    S1, d1 = o.rates_cell(_cell(orc, T=T, p=p, Y=Y, liq=liq, ns=N_soot))
    S0, d0 = o.rates_cell(_cell(orc, T=T, p=p, Y=Y, liq=liq, ns=0.0))
    # soot surface per unit volume: quadrature of the lognormal number density
    s = math.log(sg)
    x = np.linspace(math.log(rg) - 12 * s, math.log(rg) + 12 * s, 100001)
    f_dlnr = N_soot / (s * math.sqrt(2 * math.pi)) * np.exp(-(x - math.log(rg)) ** 2 / (2 * s * s))
    area = np.trapezoid(4 * math.pi * np.exp(2 * x) * f_dlnr, x)
    J_het = 1.0 * ns * area
    mdot = RHO_L * (4.0 / 3.0 * math.pi) ** 2 * J_het * Nl * rl ** 6
    assert d1["mdot_f"] - d0["mdot_f"] == pytest.approx(mdot, rel=1e-6)
    # the droplets that freeze leave the liquid and join the ice (number source J n V)
    assert (S0[5] - S1[5]) == pytest.approx(J_het * 4.0 / 3.0 * math.pi * Nl * rl ** 3, rel=1e-6)
    assert (S1[9] - S0[9]) == pytest.approx(J_het * 4.0 / 3.0 * math.pi * Nl * rl ** 3, rel=1e-6)
    # freezing moves water from liquid to ice and none from the vapour
    assert S1[4] == pytest.approx(S0[4], rel=1e-12, abs=1e-30)


def _dT_dt(orc, U, S, eps):
    """Temperature change of the gas over eps seconds of the instantaneous source, and
    the heat capacity rho c_v of the gas after it (fixed volume)."""
    U1 = U + eps * S
    g0, g1 = _gas(orc, U), _gas(orc, U1)
    rho_a = g1["rho"] - U1[4]
    rc_v = rho_a * (CP_A - R_A) + U1[4] * (CP_V - R_V)
    return g1["T"] - g0["T"], rc_v


def test_condensation_heats_gas_by_latent_heat(orc):
    """Eq. 22-26 energy exchange (the latent heat stays in the gas): at rest and at
    fixed volume, vapour that condenses on droplets warms the gas by
    rho c_v dT = (h_fg(T) - R_v T) dm -- the vapour leaves with the liquid's enthalpy
    and its internal energy e_v = h_v - R_v T stays behind.  Checked on the
    instantaneous source of a growing droplet population at 280 K (no freezing)."""
    T, p = 280.0, 23800.0
    Y = _y_at(orc, T, p, math.log(1.3))
    m, c = inputs.sa0(n_soot=0.0)
    o = orc.Oracle(m, c)
    U = _cell(orc, T=T, p=p, Y=Y, liq=[1e9 * 1e-6 ** k for k in range(4)])
    S, d = o.rates_cell(U)
    assert d["Gl"] > 0 and d["mdot_f"] == 0.0
    eps = 1e-4
    dT, rc_v = _dT_dt(orc, U, S, eps)
    dm = -eps * S[4]                       # vapour condensed
    assert dm > 0
    assert rc_v * dT == pytest.approx((_h_fg(T) - R_V * T) * dm, rel=1e-6)
    # the gas loses exactly the condensed mass, and keeps its momentum (at rest)
    assert S[0] == S[4] and S[1] == 0.0 and S[2] == 0.0


def test_deposition_heats_gas_by_sublimation_heat(orc):
    """As above for crystals growing from vapour (subsaturated over liquid): the gas
    warms by (h_sg(T) - R_v T) dm / (rho c_v)."""
    T, p = 235.0, 23800.0
    Y = _y_at(orc, T, p, math.log(1.2), ice=True)
    m, c = inputs.sa0(n_soot=0.0)
    o = orc.Oracle(m, c)
    U = _cell(orc, T=T, p=p, Y=Y, ice=[1e9 * 2e-6 ** k for k in range(4)])
    S, d = o.rates_cell(U)
    assert d["Gs"] > 0 and d["lnSl"] < 0
    eps = 1e-4
    dT, rc_v = _dT_dt(orc, U, S, eps)
    dm = -eps * S[4]
    assert dm > 0
    assert rc_v * dT == pytest.approx((_h_sg(T) - R_V * T) * dm, rel=1e-6)


def test_freezing_releases_fusion_heat(orc):
    """Freezing (Eq. 13, 15) moves mass from liquid to ice and releases
    h_sl = h_sg - h_fg per frozen kilogram to the gas: between the same cell with and
    without soot (immersion freezing on or off) the energy source differs by
    h_sl(T) d(mdot_f), the vapour source not at all."""
    T, p = 255.0, 23800.0
    Y = _y_at(orc, T, p, math.log(0.95))
    liq = [4e8 * 3e-6 ** k for k in range(4)]
    m, c = inputs.sa0(n_soot=1e13)
    o = orc.Oracle(m, c)
    S1, d1 = o.rates_cell(_cell(orc, T=T, p=p, Y=Y, liq=liq, ns=1e13))
    S0, d0 = o.rates_cell(_cell(orc, T=T, p=p, Y=Y, liq=liq, ns=0.0))
    dmf = d1["mdot_f"] - d0["mdot_f"]
    assert dmf > 0
    g = _gas(orc, _cell(orc, T=T, p=p, Y=Y, liq=liq, ns=1e13))
    h_sl = _h_sg(g["T"]) - _h_fg(g["T"])
    assert S1[3] - S0[3] == pytest.approx(h_sl * dmf, rel=1e-8)
    assert S1[4] == pytest.approx(S0[4], rel=1e-12)
    # the crystals gain the frozen mass: rho_s (4 pi/3) d(ice mu3) = d(mdot_f)
    assert RHO_I * 4.0 / 3.0 * math.pi * (S1[12] - S0[12]) == pytest.approx(dmf, rel=1e-10)


# ------------------------------------------------------ Eq. 19-21 (polydisperse)
def _growth_quadrature(T, p, R, cp, dT, h, Tsat, rc, f, r, k):
    """k * int r^(k-1) G(r) f(r) dr by the trapezoidal rule on the given nodes
    (Eq. 20, the growth term without the closure)."""
    G = _young_G(r, T, p, R, cp, dT, h, RHO_L, Tsat, rc, GOLD["young_alpha"]["value"],
                 GOLD["young_beta"]["value"])
    return k * np.trapezoid(r ** (k - 1) * G * f, r)


def _polydisperse_case(orc, moments):
    L = orc.lib()
    T, p = 283.0, 23800.0
    Y = _y_at(orc, T, p, math.log(0.8))     # subsaturated, warm: evaporation only
    m, c = inputs.sa0(n_soot=0.0)
    o = orc.Oracle(m, c)
    U = _cell(orc, T=T, p=p, Y=Y, liq=moments)
    S, d = o.rates_cell(U)
    g = _gas(orc, U)
    pv = g["rho_v"] * R_V * g["T"]
    Tsat = L.or_tsat_liq(pv, g["T"])
    lnS = math.log(pv) - L.or_ln_psat_liq(g["T"])
    rc = 2.0 * _sigma_iapws(g["T"]) / (RHO_L * R_V * g["T"] * lnS)
    args = (g["T"], g["p"], g["R"], g["cp"], Tsat - g["T"], _h_fg(g["T"]), Tsat, rc)
    return S, d, args


def _closure_error_lognormal(orc, sg, N=1e9, rg=0.4e-6):
    s = math.log(sg)
    mom = _lognormal(N, rg, sg)
    S, d, args = _polydisperse_case(orc, mom)
    assert d["Gl"] < 0 and S[5] == 0.0
    x = np.linspace(math.log(rg) - 10 * s, math.log(rg) + 10 * s, 100001)
    r = np.exp(x)
    f = N / (r * s * math.sqrt(2 * math.pi)) * np.exp(-(x - math.log(rg)) ** 2 / (2 * s * s))
    # Eq. 21 as printed: the closure evaluates G at r20 = sqrt(mu2 / mu0)
    r20 = math.sqrt(mom[2] / mom[0])
    G20 = _young_G(np.array([r20]), *args[:6], RHO_L, *args[6:], GOLD["young_alpha"]["value"],
                   GOLD["young_beta"]["value"])[0]
    errs = []
    for k in (1, 2, 3):
        assert S[5 + k] == pytest.approx(k * mom[k - 1] * G20, rel=1e-10)
        quad = _growth_quadrature(*args, f, r, k)
        errs.append(abs(S[5 + k] / quad - 1.0))
    return errs


def test_growth_moments_closure_against_quadrature_lognormal(orc):
    """Eq. 19-21: the r20 closure k mu_{k-1} G(r20) of the growth term against
    brute-force quadrature of k int r^(k-1) G(r) f(r) dr (10^5 nodes) over lognormal
    size distributions of growing width.  The closure error vanishes as the
    distribution narrows (sigma_g -> 1) and grows with sigma_g; it is not zero for
    a finite width (the closure is an approximation, Sec. 2.2)."""
    sgs = [1.001, 1.01, 1.1, 1.3, 1.6]
    errs = np.array([_closure_error_lognormal(orc, sg) for sg in sgs])
    # printed for the record: relative closure error of dmu_1, dmu_2, dmu_3
    for sg, e in zip(sgs, errs):
        print("lognormal sigma_g %.3f: closure error %.2e %.2e %.2e" % (sg, *e))
    assert errs[0].max() < 1e-5
    assert errs[1].max() < 1e-3
    assert np.all(np.diff(errs.max(axis=1)) > 0)
    assert errs[-1].max() < 0.5


def test_growth_moments_closure_against_quadrature_gamma(orc):
    """As above for gamma distributions f(r) = N r^(a-1) e^(-r/theta) / (Gamma(a) theta^a)
    of fixed mean radius: the closure error falls toward zero as the shape a grows
    (the distribution narrows), and the moments mu_k = N theta^k Gamma(a+k)/Gamma(a)
    match the quadrature's own moments."""
    N, rmean = 1e9, 0.5e-6
    errs = []
    for a in (4.0, 30.0, 300.0, 30000.0):
        th = rmean / a
        mom = [N * th ** k * math.exp(math.lgamma(a + k) - math.lgamma(a)) for k in range(4)]
        S, d, args = _polydisperse_case(orc, mom)
        sd = math.sqrt(a) * th
        r = np.linspace(max(rmean - 40 * sd, rmean * 1e-4), rmean + 60 * sd, 100001)
        f = N * np.exp((a - 1) * np.log(r / th) - r / th - math.lgamma(a)) / th
        assert np.trapezoid(r ** 3 * f, r) == pytest.approx(mom[3], rel=1e-6)
        e = []
        for k in (1, 2, 3):
            quad = _growth_quadrature(*args, f, r, k)
            e.append(abs(S[5 + k] / quad - 1.0))
        print("gamma shape %g: closure error %.2e %.2e %.2e" % (a, *e))
        errs.append(max(e))
    assert errs[-1] < 1e-4
    assert np.all(np.diff(errs) < 0)


@pytest.mark.parametrize("table_h", [0.0, 0.25])
def test_particle_free_subsaturated_cell_has_no_source(orc, table_h):
    """Eq. 4, 10 and 16-21 vanish together in a cell without droplets or crystals that
    is not supersaturated over liquid: no nucleation (the rates need ln S_l > 0; just
    above zero the barrier term makes them underflow to exactly zero), no growth and
    no freezing without particles.  The instantaneous rates of such cells, evaluated
    in full (with closed-form or tabulated properties, soot present), are exactly
    zero -- so skipping the source in them changes nothing."""
    g = np.random.default_rng(5)
    m, c = inputs.sa0(n_soot=1e13)
    o = orc.Oracle(m, c)
    if table_h:
        o.set_property_table(table_h)
    for lnS in np.concatenate([-np.logspace(-12, 0.5, 40), [0.0, 1e-9, 1e-6]]):
        T = g.uniform(180.0, 320.0)
        p = g.uniform(1e4, 1e5)
        U = _cell(orc, T=T, p=p, Y=_y_at(orc, T, p, lnS), ns=1e13, na=g.uniform(0, 1e13))
        S, d = o.rates_cell(U)
        assert np.all(S == 0.0), (T, p, lnS, S)
