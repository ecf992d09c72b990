"""Seeded synthetic inputs: meshes and operating points as plain numbers.

This module holds only random draws and configuration recipes -- none of the
method's arithmetic.  Derived quantities (ambient humidity from the ice relative
humidity, flight speed from the Mach number, inflow conserved states, mesh
coordinates) are computed independently by the HIP library and by the test
oracle from these numbers.

The workloads take the shape of the paper's three-stream exhaust jet at cruise
(core / bypass / free stream, lognormal soot; Sec. 4.1, Tab. 2) on a 2 m x 0.5 m
axisymmetric domain, plus a hydrogen-like high-water variant (Sec. 4.3) that
activates the phase-change source.
"""
import numpy as np

BC_INFLOW, BC_COPY, BC_WALL, BC_FARFIELD = 0, 1, 2, 3
GEOM_AXI, GEOM_PLANAR, GEOM_QUASI1D = 0, 1, 2

_CASE_DEFAULTS = dict(
    p_amb=23800.0, T_amb=218.0, RH_ice=1.1, mach_amb=0.8,
    R_core=0.3, u_core=450.0, T_core=600.0, Y_core=0.03,
    R_fan=0.9, u_byp=300.0, T_byp=250.0, Y_byp=-1.0,
    n_soot=1.0e13, r_g_soot=15e-9, sigma_g_soot=1.6,
    cfl=0.5, theta_deg=90.0, n_s=1.0e8, k_imm=1.0,
    kappa_m=0.07, s_delta=0.036, delta0_frac=0.02,
    n_sub_max=64, phase_change=1,
)


def mesh(nx, nr, Lx=2.0, Lr=0.5, sx_ratio=1.0, r_cluster=0.0, beta_r=0.0, geom=GEOM_AXI,
         bc=(BC_INFLOW, BC_COPY, BC_WALL, BC_FARFIELD)):
    return dict(nx=int(nx), nr=int(nr), Lx=float(Lx), Lr=float(Lr), sx_ratio=float(sx_ratio),
                r_cluster=float(r_cluster), beta_r=float(beta_r), geom=int(geom),
                bc_xlo=int(bc[0]), bc_xhi=int(bc[1]), bc_rlo=int(bc[2]), bc_rhi=int(bc[3]))


def case(**kw):
    c = dict(_CASE_DEFAULTS)
    for k, v in kw.items():
        if k not in c:
            raise KeyError(k)
        c[k] = v
    return c


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def config1(seed=1):
    """Tiny plain method: 96 x 48 uniform, ambient drawn per seed."""
    g = _rng(seed)
    p = g.uniform(22e3, 25e3)
    T = g.uniform(210.0, 225.0)
    rh = g.uniform(0.6, 1.2)
    return mesh(96, 48), case(p_amb=p, T_amb=T, RH_ice=rh)


def config2(seed=0, nx=2048, nr=512):
    """Production plain method: 2048 x 512, stretched / clustered, fixed ambient."""
    g = _rng(seed)
    ns = 10.0 ** g.uniform(12.0, 14.0)
    return (mesh(nx, nr, sx_ratio=1.002, r_cluster=0.3, beta_r=5.0),
            case(p_amb=23800.0, T_amb=218.0, RH_ice=1.1, n_soot=ns))


def sa1(seed=1, n_soot=None):
    """Source-active twin of config 1: hydrogen-like core water (0.22) and a cold bypass."""
    m, c = config1(seed)
    c["Y_core"] = 0.22
    c["T_byp"] = c["T_amb"]
    if n_soot is not None:
        c["n_soot"] = n_soot
    return m, c


def sa2(seed=0, nx=2048, nr=512):
    """Source-active production mesh (sa1 physics on the config-2 mesh)."""
    m, c = config2(seed, nx, nr)
    c["Y_core"] = 0.22
    c["T_byp"] = c["T_amb"]
    return m, c


def sa0(nx=8, nr=4, Y=0.0045, T=230.0, n_soot=1.0e13):
    """Closed, uniform, source-active box at rest (planar, walls on all sides)."""
    m = mesh(nx, nr, Lx=0.08, Lr=0.04, geom=GEOM_PLANAR, bc=(BC_WALL, BC_WALL, BC_WALL, BC_WALL))
    c = case(p_amb=23800.0, T_amb=T, RH_ice=1.0, mach_amb=0.0, R_core=10.0, u_core=0.0,
             T_core=T, Y_core=Y, n_soot=n_soot)
    return m, c


def config4(seed=0, nplumes=64):
    """Batched operating points: meshes from {256x64, 512x128, 1024x256}."""
    g = _rng(seed)
    sizes = [(256, 64), (512, 128), (1024, 256)]
    out = []
    for _ in range(nplumes):
        nx, nr = sizes[int(g.integers(0, 3))]
        T = g.uniform(205.0, 230.0)
        p = g.uniform(20e3, 30e3)
        rh = g.uniform(0.4, 1.3)
        ei = g.uniform(1.2, 9.0)
        ns = 10.0 ** g.uniform(11.0, 14.0)
        out.append((mesh(nx, nr), case(p_amb=p, T_amb=T, RH_ice=rh, Y_core=0.03 * ei / 1.23,
                                       n_soot=ns)))
    return out


def particle_fields(nr, nx, seed=0, frac=0.05):
    """Seeded particle moments per m^3 on a random fraction of the cells of an
    nr x nx mesh: soot-activated droplets, homogeneously nucleated droplets and
    crystals, each from lognormal draws (N, r_g, sigma_g), so every set is
    realisable.  Returned as arrays of shape (4, nr, nx)."""
    g = _rng(seed)
    n = nr * nx

    def lognormal_moments(has, lo, hi):
        N = np.where(has, 10.0 ** g.uniform(6.0, 11.0, n), 0.0)
        rg = 10.0 ** g.uniform(lo, hi, n)
        sg = g.uniform(1.05, 1.8, n)
        s2 = np.log(sg) ** 2
        return np.stack([N * np.exp(k * np.log(rg) + 0.5 * k * k * s2) for k in range(4)]).reshape(4, nr, nx)

    het = lognormal_moments(g.uniform(size=n) < frac, -7.5, -6.3)
    hom = lognormal_moments(g.uniform(size=n) < frac, -8.5, -7.0)
    ice = lognormal_moments(g.uniform(size=n) < 0.5 * frac, -7.0, -6.0)
    return het, hom, ice


def velocity_noise(nr, nx, seed=0, amp=5.0):
    """Seeded uniform noise in [-amp, amp] (m/s) on an nr x nx mesh, to stir a
    state that is uniform along x so that every face carries a flux."""
    return _rng(seed).uniform(-amp, amp, (nr, nx))


def random_cells(n, seed=0, active=True):
    """Primitive cell states (rho, u, v, p, Y, mu-moments per mass, soot) spanning the
    paper's regimes; returned as a dict of arrays.  Moments come from lognormal draws
    (N, r_g, sigma_g) so they are realisable."""
    g = _rng(seed)
    T = g.uniform(200.0, 320.0, n) if active else g.uniform(200.0, 650.0, n)
    p = g.uniform(18e3, 32e3, n)
    Y = 10.0 ** g.uniform(-4.0, -0.7, n)
    u = g.uniform(-50.0, 500.0, n)
    v = g.uniform(-50.0, 50.0, n)

    def lognormal_moments(has):
        N = np.where(has, 10.0 ** g.uniform(6.0, 12.0, n), 0.0)
        rg = 10.0 ** g.uniform(-9.0, -6.3, n)
        sg = g.uniform(1.05, 2.0, n)
        s2 = np.log(sg) ** 2
        return np.stack([N * np.exp(k * np.log(rg) + 0.5 * k * k * s2) for k in range(4)])

    liq = lognormal_moments(g.uniform(size=n) < 0.6)
    ice = lognormal_moments(g.uniform(size=n) < 0.4)
    ns = np.where(g.uniform(size=n) < 0.7, 10.0 ** g.uniform(10.0, 14.0, n), 0.0)
    na = ns * g.uniform(0.0, 1.0, n) * (g.uniform(size=n) < 0.5)
    return dict(T=T, p=p, Y=Y, u=u, v=v, liq=liq, ice=ice, n_soot=ns, n_act=na)


def extreme_cells(n, seed=0):
    """Primitive cell states over the whole range the source accepts, for stress
    parity: 150 to 700 K (the property range), 5 to 100 kPa, vapour mass fractions
    from 1e-6 to 0.3 with one cell in ten holding no vapour at all, and droplets
    (two sets: soot-activated and homogeneous), crystals and soot with lognormal
    moments from 1 nm to 10 um and up to 1e13 per m^3.  The condensed mass of each
    set is capped at 5 % of p / (287 T) so that the gas stays the carrier.  Returned
    as a dict of arrays like random_cells, plus the second droplet set as 'hom'."""
    g = _rng(seed)
    T = g.uniform(150.0, 700.0, n)
    p = 10.0 ** g.uniform(np.log10(5e3), 5.0, n)
    Y = np.where(g.uniform(size=n) < 0.1, 0.0, 10.0 ** g.uniform(-6.0, -0.5, n))
    u = g.uniform(-50.0, 500.0, n)
    v = g.uniform(-50.0, 50.0, n)
    mu3_cap = 0.05 * p / (287.0 * T) / (4.0 / 3.0 * np.pi * 1000.0)

    def lognormal_moments(has, lg_rmax):
        N = np.where(has, 10.0 ** g.uniform(0.0, 13.0, n), 0.0)
        rg = 10.0 ** g.uniform(-9.0, lg_rmax, n)
        sg = g.uniform(1.01, 2.2, n)
        s2 = np.log(sg) ** 2
        M = np.stack([N * np.exp(k * np.log(rg) + 0.5 * k * k * s2) for k in range(4)])
        scale = np.minimum(1.0, mu3_cap / np.maximum(M[3], 1e-300))
        return M * scale

    liq = lognormal_moments(g.uniform(size=n) < 0.6, -5.0)
    ice = lognormal_moments(g.uniform(size=n) < 0.5, -5.0)
    hom = lognormal_moments(g.uniform(size=n) < 0.5, -6.0)
    ns = np.where(g.uniform(size=n) < 0.7, 10.0 ** g.uniform(8.0, 14.0, n), 0.0)
    na = np.minimum(ns, liq[0]) * g.uniform(0.0, 1.0, n) * (g.uniform(size=n) < 0.5)
    return dict(T=T, p=p, Y=Y, u=u, v=v, liq=liq, ice=ice, hom=hom, n_soot=ns, n_act=na)
