"""FP64 CPU oracle of the contrail-formation finite-volume step -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``contrail_oracle.c`` (plain C,
``-O2 -ffp-contract=off``, OpenMP over rows) through ctypes and shares no code
with the HIP library.  ``mlp.py`` holds the FP64 oracle of the learned source
surrogate.

Every function of the C file cites the section / equation of Tegethoff & Wheeler
(arXiv 2504.20742) that it follows.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "contrail_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
NV = 15          # variables per cell; 19 with two liquid populations (set_bimodal)
NV_BIMODAL = 19

_lib = None


def build(force=True):
    """Compile the oracle with gcc (no contraction, no fast-math)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
           "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


class OrMesh(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("nr", ctypes.c_int),
                ("Lx", ctypes.c_double), ("Lr", ctypes.c_double),
                ("sx_ratio", ctypes.c_double), ("r_cluster", ctypes.c_double),
                ("beta_r", ctypes.c_double),
                ("geom", ctypes.c_int), ("bc_xlo", ctypes.c_int), ("bc_xhi", ctypes.c_int),
                ("bc_rlo", ctypes.c_int), ("bc_rhi", ctypes.c_int)]


_CASE_DOUBLES = ["p_amb", "T_amb", "RH_ice", "mach_amb", "R_core", "u_core", "T_core", "Y_core",
                 "R_fan", "u_byp", "T_byp", "Y_byp", "n_soot", "r_g_soot", "sigma_g_soot", "cfl",
                 "theta_deg", "n_s", "k_imm", "kappa_m", "s_delta", "delta0_frac"]


class OrCase(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in _CASE_DOUBLES] + [
        ("n_sub_max", ctypes.c_int), ("phase_change", ctypes.c_int),
        ("pad0", ctypes.c_int), ("pad1", ctypes.c_int)]


_D = ctypes.c_double
_P = ctypes.POINTER(ctypes.c_double)
_V = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        for name in ["or_ln_psat_liq", "or_ln_psat_ice", "or_sigma_lg", "or_mu_sutherland",
                     "or_koop_delta_aw", "or_koop_rate", "or_contact_factor", "or_cunningham_ac"]:
            getattr(L, name).restype = _D
            getattr(L, name).argtypes = [_D]
        L.or_sn_slip.restype = _D
        L.or_sn_slip.argtypes = [_D, _D, _D, _D]
        for name in ["or_tsat_liq", "or_tsat_ice", "or_cnt_prefactor", "or_kantrowitz_phi",
                     "or_young_nu", "or_barrier_hom", "or_drag_cd"]:
            getattr(L, name).restype = _D
            getattr(L, name).argtypes = [_D, _D]
        L.or_critical_radius.restype = _D
        L.or_critical_radius.argtypes = [_D, _D, _D]
        L.or_gibbs_cluster.restype = _D
        L.or_gibbs_cluster.argtypes = [_D, _D, _D, _D]
        L.or_young_growth.restype = _D
        L.or_young_growth.argtypes = [_D] * 7
        L.or_create.restype = _V
        L.or_create.argtypes = [ctypes.POINTER(OrMesh), ctypes.POINTER(OrCase)]
        L.or_destroy.argtypes = [_V]
        L.or_init.argtypes = [_V, _P]
        L.or_residual.argtypes = [_V, _P, _P]
        L.or_source.restype = ctypes.c_long
        L.or_source.argtypes = [_V, _P, _D, _P]
        L.or_step.argtypes = [_V, _P, _D]
        L.or_cfl_dt.argtypes = [_V, _P, _P]
        L.or_run.restype = _D
        L.or_run.argtypes = [_V, _P, ctypes.c_int]
        L.or_diag.argtypes = [_V, _P, _P]
        L.or_particle_times.argtypes = [_V, _P, _P, _P]
        L.or_mesh_faces.argtypes = [_V, _P, _P]
        L.or_set_equilibrium.restype = ctypes.c_int
        L.or_set_equilibrium.argtypes = [_V, ctypes.c_int]
        L.or_set_drift.restype = ctypes.c_int
        L.or_set_drift.argtypes = [_V, ctypes.c_int]
        L.or_set_bimodal.restype = ctypes.c_int
        L.or_set_bimodal.argtypes = [_V, ctypes.c_int]
        L.or_nvar.restype = ctypes.c_int
        L.or_nvar.argtypes = [_V]
        L.or_property.restype = _D
        L.or_property.argtypes = [_V, ctypes.c_int, _D]
        L.or_property_tsat.restype = _D
        L.or_property_tsat.argtypes = [_V, ctypes.c_int, _D, _D]
        L.or_set_property_table.restype = ctypes.c_int
        L.or_set_property_table.argtypes = [_V, _D]
        L.or_set_area.restype = ctypes.c_int
        L.or_set_area.argtypes = [_V, _P]
        L.or_case_derived.argtypes = [_V, _P]
        L.or_source_cell.restype = ctypes.c_int
        L.or_source_cell.argtypes = [_V, _P, _D, _P]
        L.or_source_rates_cell.argtypes = [_V, _P, _D, _P, _P]
        L.or_prim_to_cons.argtypes = [_P, _P]
        L.or_cons_to_prim.argtypes = [_P, _P]
        _lib = L
    return _lib


def _ptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_P)


def make_mesh(m):
    return OrMesh(**{k: m[k] for k, _ in OrMesh._fields_})


def make_case(c):
    d = {k: c[k] for k in _CASE_DOUBLES}
    d.update(n_sub_max=int(c["n_sub_max"]), phase_change=int(c["phase_change"]), pad0=0, pad1=0)
    return OrCase(**d)


class Oracle:
    """One mesh + case on the host; arrays are float64 ``U[nv][nr][nx]`` with nv = 15,
    or 19 once ``set_bimodal`` splits the liquid into two populations."""

    def __init__(self, mesh, case):
        self.L = lib()
        self.mesh = dict(mesh)
        self.case = dict(case)
        self._m = make_mesh(mesh)
        self._c = make_case(case)
        self.nx, self.nr = int(mesh["nx"]), int(mesh["nr"])
        self.h = self.L.or_create(ctypes.byref(self._m), ctypes.byref(self._c))
        if mesh.get("area_x") is not None:
            self.set_area(mesh["area_x"])

    def __del__(self):
        try:
            if self.h:
                self.L.or_destroy(self.h)
                self.h = None
        except Exception:
            pass

    @property
    def nv(self):
        return self.L.or_nvar(self.h)

    def empty(self):
        return np.zeros((self.nv, self.nr, self.nx), dtype=np.float64)

    def init(self):
        U = self.empty()
        self.L.or_init(self.h, _ptr(U))
        return U

    def residual(self, U):
        R = self.empty()
        self.L.or_residual(self.h, _ptr(U), _ptr(R))
        return R

    def source(self, U, dt, return_nsub=False):
        Q = self.empty()
        n = self.L.or_source(self.h, _ptr(U), float(dt), _ptr(Q))
        return (Q, n) if return_nsub else Q

    def step(self, U, dt):
        self.L.or_step(self.h, _ptr(U), float(dt))
        return U

    def cfl_dt(self, U):
        d = ctypes.c_double()
        self.L.or_cfl_dt(self.h, _ptr(U), ctypes.byref(d))
        return d.value

    def run(self, U, nsteps):
        return self.L.or_run(self.h, _ptr(U), int(nsteps))

    def diag(self, U):
        out = np.zeros(4)
        self.L.or_diag(self.h, _ptr(U), _ptr(out))
        return {"water": out[0], "max_lnS_l": out[1], "ice_number": out[2], "gas_mass": out[3]}

    def particle_times(self, U):
        """Response time tau_p and Stokes number of the droplets and crystals at their
        mean radius r20 (Eq. 24 diagnostics): two arrays [2][nr][nx]."""
        tau = np.zeros((2, self.nr, self.nx))
        St = np.zeros((2, self.nr, self.nx))
        self.L.or_particle_times(self.h, _ptr(U), _ptr(tau), _ptr(St))
        return tau, St

    def set_equilibrium(self, on=True):
        """Switch the phase change between the kinetic model and the equilibrium
        comparison model (instantaneous phase equilibrium per cell)."""
        if self.L.or_set_equilibrium(self.h, 1 if on else 0) != 0:
            raise ValueError("or_set_equilibrium: not with two liquid populations")

    def set_drift(self, on=True):
        """Droplets and crystals drift against the gas with their Stokes-Cunningham
        terminal slip in the pressure gradient (drift-flux reading of Eq. 24)."""
        if self.L.or_set_drift(self.h, 1 if on else 0) != 0:
            raise ValueError("or_set_drift: not with two liquid populations")

    def set_bimodal(self, on=True):
        """Carry the liquid as two populations (Sec. 2.2): soot-activated droplets in
        variables 5..8, homogeneously nucleated ones in 15..18 (arrays of 19 planes)."""
        if self.L.or_set_bimodal(self.h, 1 if on else 0) != 0:
            raise ValueError("or_set_bimodal: not with the equilibrium model or drift")

    def set_property_table(self, h):
        """Water properties from a table of spacing h [K] read by a second-order Taylor
        expansion (h = 0: the closed forms)."""
        if self.L.or_set_property_table(self.h, float(h)) != 0:
            raise ValueError("or_set_property_table: spacing must be >= 0 and give at most 1e6 nodes")

    def property(self, q, T):
        """Water property q (0 ln p_sat,w, 1 ln p_sat,i, 2 sigma) as the source reads it."""
        return self.L.or_property(self.h, int(q), float(T))

    def set_area(self, area):
        """Quasi-1D duct only: cross-section areas at the nx+1 x faces."""
        a = np.ascontiguousarray(area, dtype=np.float64)
        assert a.shape == (self.nx + 1,)
        if self.L.or_set_area(self.h, _ptr(a)) != 0:
            raise ValueError("or_set_area: needs the quasi-1D geometry, nr = 1 and positive areas")

    def faces(self):
        xf = np.zeros(self.nx + 1)
        rf = np.zeros(self.nr + 1)
        self.L.or_mesh_faces(self.h, _ptr(xf), _ptr(rf))
        return xf, rf

    def derived(self):
        out = np.zeros(4)
        self.L.or_case_derived(self.h, _ptr(out))
        return {"Y_amb": out[0], "u_amb": out[1], "f_theta": out[2], "soot_area": out[3]}

    def source_cell(self, Uc, dt):
        Uc = np.ascontiguousarray(Uc, dtype=np.float64)
        assert Uc.shape == (self.nv,)
        Q = np.zeros(self.nv)
        n = self.L.or_source_cell(self.h, _ptr(Uc), float(dt), _ptr(Q))
        return Q, n

    def rates_cell(self, Uc, h=1e-6):
        Uc = np.ascontiguousarray(Uc, dtype=np.float64)
        assert Uc.shape == (self.nv,)
        S = np.zeros(self.nv)
        d = np.zeros(8)
        self.L.or_source_rates_cell(self.h, _ptr(Uc), float(h), _ptr(S), _ptr(d))
        names = ["Gl", "Gs", "Jhom", "Jhet", "rcrit", "lnSl", "lnSi", "mdot_f"]
        return S, dict(zip(names, d))


def prim_to_cons(W):
    """W = (rho, u, v, p, Y, phi5..phi14) -> U (15)."""
    W = np.ascontiguousarray(W, dtype=np.float64)
    U = np.zeros(NV)
    lib().or_prim_to_cons(_ptr(W), _ptr(U))
    return U


def cons_to_prim(U):
    """U (15) -> (rho, u, v, p, Y, phi5..phi14, T, c)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    W = np.zeros(17)
    lib().or_cons_to_prim(_ptr(U), _ptr(W))
    return W
