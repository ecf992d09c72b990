"""Exact steady isentropic flow of a perfect gas through a quasi-1D duct.

Textbook gas dynamics (e.g. Anderson, Modern Compressible Flow, Ch. 5): for a
choked duct with throat area A*, the Mach number at area A solves

    A / A* = (1/M) [ (2/(g+1)) (1 + (g-1)/2 M^2) ]^((g+1)/(2(g-1))),

on the subsonic branch upstream of the throat and the supersonic branch
downstream; the static state follows from the stagnation state by the
isentropic relations.  Written here from those relations alone, for the tests.
"""
import numpy as np
from scipy.optimize import brentq


def area_ratio(M, g):
    return (1.0 / M) * ((2.0 / (g + 1.0)) * (1.0 + 0.5 * (g - 1.0) * M * M)) ** ((g + 1.0) / (2.0 * (g - 1.0)))


def mach(ar, supersonic, g):
    """Mach number at A/A* = ar (>= 1) on the chosen branch."""
    if ar <= 1.0 + 1e-15:
        return 1.0
    f = lambda M: area_ratio(M, g) - ar
    if supersonic:
        return brentq(f, 1.0, 60.0, xtol=1e-15, rtol=1e-15)
    return brentq(f, 1e-8, 1.0, xtol=1e-15, rtol=1e-15)


def static_state(M, p0, T0, g, R):
    """(rho, u, p, T) at Mach M from the stagnation pressure and temperature."""
    T = T0 / (1.0 + 0.5 * (g - 1.0) * M * M)
    p = p0 * (T / T0) ** (g / (g - 1.0))
    return p / (R * T), M * np.sqrt(g * R * T), p, T


def nozzle_area(x):
    """Converging-diverging test duct on [0, 1]: A = 1 + 4 (x - 1/2)^2, throat
    A* = 1 at x = 1/2, inlet and exit area 2 (M = 0.306 in, 2.197 out for g = 1.4)."""
    return 1.0 + 4.0 * (np.asarray(x, dtype=np.float64) - 0.5) ** 2


def nozzle_mach(x, g):
    """Exact Mach number of the choked test duct at positions x."""
    return np.array([mach(float(nozzle_area(xi)), xi > 0.5, g) for xi in np.atleast_1d(x)])


P0, T0 = 1.0e5, 300.0     # stagnation state of the test duct (dry air)


def nozzle_setup(nx, g, R, cfl=0.8):
    """Mesh, case, face areas and the exact cell-centre primitives (rho, u, p) of
    the test duct on nx uniform cells.  The inflow ghost state is the exact state
    at the inlet face; the exit is a zero-gradient (supersonic) outflow."""
    from paper_2504_20742_amd import inputs
    m = inputs.mesh(nx, 1, Lx=1.0, Lr=1.0, geom=inputs.GEOM_QUASI1D,
                    bc=(inputs.BC_INFLOW, inputs.BC_COPY, inputs.BC_WALL, inputs.BC_WALL))
    rho_i, u_i, p_i, T_i = static_state(mach(float(nozzle_area(0.0)), False, g), P0, T0, g, R)
    c = inputs.case(p_amb=p_i, T_amb=T_i, RH_ice=0.0, mach_amb=0.0, R_core=10.0, u_core=u_i,
                    T_core=T_i, Y_core=0.0, R_fan=20.0, u_byp=0.0, T_byp=T_i, Y_byp=0.0, n_soot=0.0,
                    kappa_m=0.0, phase_change=0, cfl=cfl)
    xf = np.linspace(0.0, 1.0, nx + 1)
    xc = 0.5 * (xf[1:] + xf[:-1])
    M = nozzle_mach(xc, g)
    W = np.array([static_state(Mi, P0, T0, g, R)[:3] for Mi in M])
    return m, c, nozzle_area(xf), xc, M, W
