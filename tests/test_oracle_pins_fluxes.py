"""Pins of the oracle's viscous, heat and diffusion fluxes (Sec. 3.1, Eq. 22-26;
Sec. 3.2 central viscous fluxes) against the continuum divergence they discretise.

A planar channel at uniform pressure, at rest or in a linear shear u = b r, with a
temperature or vapour profile quadratic in r: the convective (Roe) flux carries
nothing across the radial faces (no normal velocity, no pressure jump) and the axial
faces cancel, so each residual component is the discrete radial divergence of the
diffusive flux alone.  The test writes that flux as the paper states it --
heat conduction, vapour diffusion with D proportional to T^1.94 / p (golden
exponent), turbulent diffusion D_t = nu_t / Sc_t with Sc_t = 0.7 (golden) -- and
compares the residual with the flux's exact derivative: the error must fall at
second order under refinement.  Readings where the paper is silent: conductivity
c_p (mu / Pr + mu_t / Pr_t) with Pr = 0.71, Pr_t = 0.9; the vapour diffusivity
constant 2.11e-5 m^2/s at 273.15 K and 101325 Pa (Pruppacher & Klett, the paper's
source for the T^1.94 / p law); the diffused vapour carries the enthalpy difference
h_v - h_a; the algebraic mixing length l_m = kappa_m (delta_0 + s_delta x) in place
of Spalart-Allmaras.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2504_20742_amd import inputs
from tests.test_oracle_pins import _cell

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))

R_A, CP_A, R_V, CP_V, T0, L_VAP0 = 287.0, 1004.5, 461.52, 1846.08, 273.15, 2.5008e6
PR, PR_T = 0.71, 0.9
D0 = GOLD["vapour_diffusivity_m2_s"]["value"]
P0 = GOLD["vapour_diffusivity_m2_s"]["p_Pa"]
SC_T = GOLD["turbulent_schmidt"]["value"]
D_EXP = GOLD["vapour_diffusion_T_exponent"]["value"]
P = 1.0e5
LR = 0.032


def _sutherland(T):
    return 1.716e-5 * (T / 273.15) ** 1.5 * (273.15 + 110.4) / (T + 110.4)


def _deriv(f, r, h=2e-5):
    """Fourth-order central difference of a smooth function of r."""
    return (-f(r + 2 * h) + 8 * f(r + h) - 8 * f(r - h) + f(r - 2 * h)) / (12 * h)


def _channel(orc, nr, T_of_r, Y_of_r, b=0.0, phi_of_r=None, eddy=False):
    """Residual of the planar channel with the given radial profiles; returns the
    interior cell centres, the residual, the case and the column's axial position."""
    nx = 6
    m = inputs.mesh(nx, nr, Lx=6 * LR / nr, Lr=LR, geom=inputs.GEOM_PLANAR,
                    bc=(inputs.BC_COPY, inputs.BC_COPY, inputs.BC_COPY, inputs.BC_COPY))
    c = inputs.case(phase_change=0, kappa_m=0.07 if eddy else 0.0)
    o = orc.Oracle(m, c)
    xf, rf = o.faces()
    rc = 0.5 * (rf[1:] + rf[:-1])
    U = o.empty()
    for j in range(nr):
        ns = phi_of_r(rc[j]) if phi_of_r else 0.0
        Uc = _cell(orc, T=T_of_r(rc[j]), p=P, Y=Y_of_r(rc[j]), u=b * rc[j], ns=ns)
        U[:, j, :] = Uc[:, None]
    R = o.residual(U)
    xc = 0.5 * (xf[1:] + xf[:-1])
    return rc, R, c, xc


def _rho(T, Y):
    return P / (((1 - Y) * R_A + Y * R_V) * T)


def _mu_t(c, x, T, Y, b):
    lm = c["kappa_m"] * (c["delta0_frac"] * c["R_core"] + c["s_delta"] * x)
    return _rho(T, Y) * lm * lm * abs(b)


def _order_check(errs):
    e1, e2 = errs
    assert e2 < 0.3 * e1, errs          # second order: a factor ~4 per halving
    return e2


def _interior(nr):
    return slice(3, nr - 3)


@pytest.mark.parametrize("eddy", [False, True])
def test_heat_conduction_flux(orc, eddy):
    """Energy residual of a quadratic temperature profile T = 250 K + a r^2 (to
    350 K at the wall) at uniform Y: d/dr(lambda_e dT/dr) with
    lambda_e = c_p (mu / Pr + mu_t / Pr_t); in the shear case u = b r also the
    viscous work d/dr(u mu_e du/dr), and the axial momentum residual
    d/dr(mu_e du/dr) with mu_e = mu + mu_t, mu_t = rho l_m^2 |du/dr|."""
    a = 100.0 / LR ** 2
    Y = 0.01
    b = 2.0e3 if eddy else 0.0
    T_of = lambda r: 250.0 + a * r * r
    errs, errs_u = [], []
    for nr in (32, 64):
        rc, R, c, xc = _channel(orc, nr, T_of, lambda r: Y, b=b, eddy=eddy)
        x = xc[3]
        cp = (1 - Y) * CP_A + Y * CP_V
        mut = (lambda r: _mu_t(c, x, T_of(r), Y, b)) if eddy else (lambda r: 0.0 * r)
        mue = lambda r: _sutherland(T_of(r)) + mut(r)
        q = lambda r: cp * (_sutherland(T_of(r)) / PR + mut(r) / PR_T) * 2 * a * r + (b * r) * mue(r) * b
        sl = _interior(nr)
        ex = np.array([_deriv(q, r) for r in rc[sl]])
        got = R[3, sl, 3]
        errs.append(np.abs(got - ex).max() / np.abs(ex).max())
        if eddy:
            exu = np.array([_deriv(lambda r: mue(r) * b, r) for r in rc[sl]])
            errs_u.append(np.abs(R[1, sl, 3] - exu).max() / np.abs(exu).max())
        assert np.abs(R[0, sl, 3]).max() < 1e-12 * np.abs(ex).max()
    e = _order_check(errs)
    assert e < 2e-3, errs
    if eddy:
        assert _order_check(errs_u) < 2e-3, errs_u


@pytest.mark.parametrize("T", [230.0, 300.0])
@pytest.mark.parametrize("eddy", [False, True])
def test_vapour_diffusion_flux(orc, T, eddy):
    """Vapour residual of a quadratic vapour profile Y = 0.005 + c r^2 (to 0.05) at
    uniform T and p: d/dr(rho (D_v + D_t) dY/dr) with
    D_v = D0 (T/273.15)^1.94 (101325/p) (D0 golden, Pruppacher & Klett) and D_t = nu_t / Sc_t, Sc_t = 0.7; the energy
    residual carries the diffused vapour's enthalpy difference,
    d/dr((h_v - h_a) rho (D_v + D_t) dY/dr) (plus the viscous work of the shear); a per-mass scalar phi (the soot number
    per kilogram, quadratic in r) diffuses with rho D_t alone."""
    cY = 0.045 / LR ** 2
    Y_of = lambda r: 0.005 + cY * r * r
    b = 2.0e3 if eddy else 0.0
    phi0, cphi = 1e12, 3e15 / LR ** 2
    phi_of = lambda r: (phi0 + cphi * r * r) * _rho(T, Y_of(r))   # soot number per m^3
    Dv = D0 * (T / T0) ** D_EXP * (P0 / P)
    dh = L_VAP0 + (CP_V - CP_A) * (T - T0)
    errs_v, errs_e, errs_s = [], [], []
    for nr in (32, 64):
        rc, R, c, xc = _channel(orc, nr, lambda r: T, Y_of, b=b, phi_of_r=phi_of, eddy=eddy)
        x = xc[3]
        mut = (lambda r: _mu_t(c, x, T, Y_of(r), b)) if eddy else (lambda r: 0.0 * r)
        Jv = lambda r: (_rho(T, Y_of(r)) * Dv + mut(r) / SC_T) * 2 * cY * r
        sl = _interior(nr)
        exv = np.array([_deriv(Jv, r) for r in rc[sl]])
        # energy: the diffused vapour's enthalpy, and in the shear the viscous work
        work = lambda s: (b * s) * (_sutherland(T) + mut(s)) * b
        exe = np.array([_deriv(lambda s: dh * Jv(s) + work(s), r) for r in rc[sl]])
        errs_v.append(np.abs(R[4, sl, 3] - exv).max() / np.abs(exv).max())
        errs_e.append(np.abs(R[3, sl, 3] - exe).max() / np.abs(exe).max())
        if eddy:
            exs = np.array([_deriv(lambda s: mut(s) / SC_T * 2 * cphi * s, r) for r in rc[sl]])
            errs_s.append(np.abs(R[13, sl, 3] - exs).max() / np.abs(exs).max())
    assert _order_check(errs_v) < 2e-3, errs_v
    assert _order_check(errs_e) < 2e-3, errs_e
    if eddy:
        assert _order_check(errs_s) < 2e-3, errs_s


def test_sutherland_reference_values(orc):
    """Sutherland's law as the flux uses it: mu(273.15 K) = 1.716e-5 Pa s exactly and
    the published air viscosity 1.846e-5 Pa s at 300 K (to 0.1 %)."""
    L = orc.lib()
    assert L.or_mu_sutherland(273.15) == pytest.approx(1.716e-5, rel=1e-14)
    assert L.or_mu_sutherland(300.0) == pytest.approx(1.846e-5, rel=1e-3)
