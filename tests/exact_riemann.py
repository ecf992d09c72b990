"""Exact Riemann solver for the 1-D Euler equations of an ideal gas with constant
gamma (Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 4).
Independent of the oracle; used to pin its convective flux on the Sod problem."""
import numpy as np


def _f(p, rho, pk, ck, g):
    if p > pk:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        return (p - pk) * np.sqrt(A / (p + B))
    return 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def star_state(rl, ul, pl, rr, ur, pr, g):
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    lo, hi = 1e-12 * min(pl, pr), 10.0 * max(pl, pr)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        val = _f(mid, rl, pl, cl, g) + _f(mid, rr, pr, cr, g) + (ur - ul)
        if val > 0.0:
            hi = mid
        else:
            lo = mid
    ps = 0.5 * (lo + hi)
    us = 0.5 * (ul + ur) + 0.5 * (_f(ps, rr, pr, cr, g) - _f(ps, rl, pl, cl, g))
    return ps, us


def sample(x, t, x0, left, right, g):
    """Density, velocity, pressure at positions x and time t."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    out = np.zeros((3, len(x)))
    for k, xi in enumerate(x):
        s = (xi - x0) / t
        if s <= us:   # left of contact
            if ps > pl:   # left shock
                sl = ul - cl * np.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= sl:
                    out[:, k] = (rl, ul, pl)
                else:
                    r = rl * ((ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1))
                    out[:, k] = (r, us, ps)
            else:         # left rarefaction
                csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
                if s <= ul - cl:
                    out[:, k] = (rl, ul, pl)
                elif s >= us - csl:
                    out[:, k] = (rl * (ps / pl) ** (1 / g), us, ps)
                else:
                    u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    r = rl * (c / cl) ** (2 / (g - 1))
                    out[:, k] = (r, u, pl * (c / cl) ** (2 * g / (g - 1)))
        else:
            if ps > pr:   # right shock
                sr = ur + cr * np.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= sr:
                    out[:, k] = (rr, ur, pr)
                else:
                    r = rr * ((ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1))
                    out[:, k] = (r, us, ps)
            else:
                csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
                if s >= ur + cr:
                    out[:, k] = (rr, ur, pr)
                elif s <= us + csr:
                    out[:, k] = (rr * (ps / pr) ** (1 / g), us, ps)
                else:
                    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    r = rr * (c / cr) ** (2 / (g - 1))
                    out[:, k] = (r, u, pr * (c / cr) ** (2 * g / (g - 1)))
    return out
