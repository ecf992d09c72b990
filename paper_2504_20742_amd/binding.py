"""ctypes binding of ``libcontrail.so`` (the C ABI of include/contrail.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
the library.  Arrays are torch CUDA tensors (or raw device pointers) shaped
``(nv, nr, nx)`` (nv = 15, or 19 with two liquid populations); float64 for CP_FP64
contexts, float32 for CP_MIXED contexts.
Loading fails loudly when the library has not been built -- there is no
fallback path.
"""
import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcontrail.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "contrail.h")

CP_OK, CP_EINVAL, CP_EHIP, CP_ENONFINITE, CP_EDT, CP_ESTATE, CP_ENOMEM, CP_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
CP_FP64, CP_MIXED = 0, 1
CP_Q_EXACT, CP_Q_SURROGATE, CP_Q_OFF, CP_Q_EQUILIBRIUM = 0, 1, 2, 3
NV = 15

_lib = None


class ContrailError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("contrail error %d: %s" % (code, msg))
        self.code = code


class CpMesh(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("nr", ctypes.c_int),
                ("Lx", ctypes.c_double), ("Lr", ctypes.c_double),
                ("sx_ratio", ctypes.c_double), ("r_cluster", ctypes.c_double),
                ("beta_r", ctypes.c_double), ("geom", ctypes.c_int),
                ("bc_xlo", ctypes.c_int), ("bc_xhi", ctypes.c_int),
                ("bc_rlo", ctypes.c_int), ("bc_rhi", ctypes.c_int),
                ("area_x", ctypes.POINTER(ctypes.c_double))]


_CASE_D = ["p_amb", "T_amb", "RH_ice", "mach_amb", "R_core", "u_core", "T_core", "Y_core",
           "R_fan", "u_byp", "T_byp", "Y_byp", "n_soot", "r_g_soot", "sigma_g_soot", "cfl",
           "theta_deg", "n_s", "k_imm", "kappa_m", "s_delta", "delta0_frac"]


class CpCase(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in _CASE_D] + [
        ("n_sub_max", ctypes.c_int), ("phase_change", ctypes.c_int),
        ("pad0", ctypes.c_int), ("pad1", ctypes.c_int)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_DP = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "cp_create": (_I, [ctypes.POINTER(CpMesh), ctypes.POINTER(CpCase), _I, _P, ctypes.POINTER(_P)]),
    "cp_destroy": (None, [_P]),
    "cp_init": (_I, [_P, _P]),
    "cp_residual": (_I, [_P, _P, _P]),
    "cp_source": (_I, [_P, _P, _D, _P]),
    "cp_step": (_I, [_P, _P, _D]),
    "cp_cfl_dt": (_I, [_P, _P, _DP]),
    "cp_step_n": (_I, [_P, _P, _I, _DP]),
    "cp_set_qmode": (_I, [_P, _I]),
    "cp_diag": (_I, [_P, _P, _DP]),
    "cp_set_tile": (_I, [_P, _I, _I]),
    "cp_set_property_table": (_I, [_P, _D]),
    "cp_set_drift": (_I, [_P, _I]),
    "cp_set_tile_masks": (_I, [_P, _I]),
    "cp_set_bimodal": (_I, [_P, _I]),
    "cp_nvar": (_I, [_P]),
    "cp_get_tile": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "cp_mesh_faces": (_I, [_P, _DP, _DP]),
    "cp_time_stage": (_I, [_P, _P, _I, _DP]),
    "cp_error_string": (ctypes.c_char_p, [_P]),
    "cp_batch_create": (_I, [_I, _P, _P, _I, _P, ctypes.POINTER(_P)]),
    "cp_batch_destroy": (None, [_P]),
    "cp_batch_init": (_I, [_P, _P]),
    "cp_batch_step_n": (_I, [_P, _P, _I, _DP]),
    "cp_batch_error_string": (ctypes.c_char_p, [_P]),
    "cp_mlp_create": (_I, [_I, _I, _I, _P, ctypes.POINTER(_P)]),
    "cp_mlp_destroy": (None, [_P]),
    "cp_mlp_num_params": (ctypes.c_long, [_P]),
    "cp_mlp_set_params": (_I, [_P, _P]),
    "cp_mlp_get_params": (_I, [_P, _P]),
    "cp_mlp_forward": (_I, [_P, _P, _I, _P]),
    "cp_mlp_forward_static": (_I, [_P, _P, _I, _P]),
    "cp_mlp_loss_grad": (_I, [_P, _P, _P, _I, _DP, _P]),
    "cp_mlp_adam": (_I, [_P, _D, _D, _D, _D]),
    "cp_mlp_error_string": (ctypes.c_char_p, [_P]),
    "cp_sur_set": (_I, [_P, _P, _P, _I]),
    "cp_sur_features": (_I, [_P, _P, _D, _P, _P]),
    "cp_particle_times": (_I, [_P, _P, _P, _P]),
}


def header_functions():
    """Names of the functions declared in include/contrail.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cp_[a-z0-9_]+)\s*\(", txt)))


def load():
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libcontrail.so is not built (run paper_2504_20742_amd/build.py or "
                           "__graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        if hasattr(L, name):
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
    _lib = L
    return L


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def make_mesh(m):
    """cp_mesh from a mesh dict; a quasi-1D mesh carries its nx+1 face areas as
    'area_x'.  The returned struct keeps the area array alive (cp_create copies it)."""
    d = {k: m[k] for k, _ in CpMesh._fields_ if k != "area_x"}
    cm = CpMesh(**d)
    a = m.get("area_x")
    if a is not None:
        import numpy as np
        arr = np.ascontiguousarray(a, dtype=np.float64)
        if arr.shape != (int(m["nx"]) + 1,):
            raise ValueError("area_x needs nx+1 values")
        cm.area_x = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        cm._area_keep = arr
    return cm


def make_case(c):
    d = {k: float(c[k]) for k in _CASE_D}
    d.update(n_sub_max=int(c["n_sub_max"]), phase_change=int(c["phase_change"]), pad0=0, pad1=0)
    return CpCase(**d)


def _current_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


class Solver:
    """One mesh + operating point on the GPU (a cp_ctx)."""

    def __init__(self, mesh, case, precision=CP_FP64, stream=None):
        self.L = load()
        self.mesh, self.case = dict(mesh), dict(case)
        self.nx, self.nr = int(mesh["nx"]), int(mesh["nr"])
        self.precision = precision
        self._m, self._c = make_mesh(mesh), make_case(case)
        h = _P()
        s = _current_stream() if stream is None else stream
        rc = self.L.cp_create(ctypes.byref(self._m), ctypes.byref(self._c), int(precision), s, ctypes.byref(h))
        if rc != CP_OK:
            raise ContrailError(rc, "cp_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.cp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc != CP_OK:
            raise ContrailError(rc, self.L.cp_error_string(self.h).decode())
        return rc

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.precision == CP_FP64 else torch.float32

    @property
    def nv(self):
        """Variables per cell: 15, or 19 with two liquid populations."""
        return self.L.cp_nvar(self.h)

    def set_bimodal(self, on=True):
        """Two liquid populations (soot-activated in 5..8, homogeneously nucleated in
        15..18); arrays then hold 19 planes."""
        self._chk(self.L.cp_set_bimodal(self.h, 1 if on else 0))

    def empty(self):
        import torch
        return torch.empty((self.nv, self.nr, self.nx), dtype=self.dtype, device="cuda")

    def _check(self, U):
        import torch
        if isinstance(U, torch.Tensor):
            n = self.nv * self.nx * self.nr
            if U.dtype != self.dtype or not U.is_cuda or not U.is_contiguous() or U.numel() != n:
                raise ValueError("U must be a contiguous CUDA %s tensor of %d elements" % (self.dtype, n))

    def init(self, U=None):
        U = self.empty() if U is None else U
        self._check(U)
        self._chk(self.L.cp_init(self.h, _ptr(U)))
        return U

    def residual(self, U, R=None):
        R = self.empty() if R is None else R
        self._check(U)
        self._check(R)
        self._chk(self.L.cp_residual(self.h, _ptr(U), _ptr(R)))
        return R

    def source(self, U, dt, Q=None):
        Q = self.empty() if Q is None else Q
        self._check(U)
        self._check(Q)
        self._chk(self.L.cp_source(self.h, _ptr(U), float(dt), _ptr(Q)))
        return Q

    def step(self, U, dt):
        self._check(U)
        self._chk(self.L.cp_step(self.h, _ptr(U), float(dt)))
        return U

    def cfl_dt(self, U):
        self._check(U)
        d = ctypes.c_double()
        self._chk(self.L.cp_cfl_dt(self.h, _ptr(U), ctypes.byref(d)))
        return d.value

    def step_n(self, U, n):
        self._check(U)
        t = ctypes.c_double()
        self._chk(self.L.cp_step_n(self.h, _ptr(U), int(n), ctypes.byref(t)))
        return t.value

    def set_qmode(self, q):
        self._chk(self.L.cp_set_qmode(self.h, int(q)))

    def diag(self, U):
        self._check(U)
        out = (ctypes.c_double * 8)()
        self._chk(self.L.cp_diag(self.h, _ptr(U), out))
        keys = ["water", "max_lnS_l", "ice_number", "gas_mass", "active_cells", "nsub_total",
                "surrogate_cells", "fallback_cells"]
        return dict(zip(keys, list(out)))

    def set_tile(self, tx, ty):
        self._chk(self.L.cp_set_tile(self.h, int(tx), int(ty)))

    def set_tile_masks(self, on=True):
        """Per-tile masks of the non-zero passive scalars (an optimisation with
        identical results); off for comparison."""
        self._chk(self.L.cp_set_tile_masks(self.h, 1 if on else 0))

    def set_drift(self, on=True):
        self._chk(self.L.cp_set_drift(self.h, 1 if on else 0))

    def set_property_table(self, h):
        self._chk(self.L.cp_set_property_table(self.h, float(h)))

    def get_tile(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        self._chk(self.L.cp_get_tile(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def time_stage(self, U, reps=20):
        """Mean duration (ms) of one launch of the fused stage kernel."""
        self._check(U)
        ms = ctypes.c_double()
        self._chk(self.L.cp_time_stage(self.h, _ptr(U), int(reps), ctypes.byref(ms)))
        return ms.value

    def sur_set(self, mlp, norm):
        """Attach a trained network (an MLP) with its 149-float normalisation."""
        import numpy as np
        nm = np.ascontiguousarray(norm, dtype=np.float32)
        self._sur_keep = (mlp, nm)
        self._chk(self.L.cp_sur_set(self.h, mlp.h, nm.ctypes.data, int(nm.size)))

    def sur_features(self, U, dt, s_in, F=None):
        """Per-cell network features [nr*nx][19] (float32 CUDA): 15 scaled states,
        ln dt, log10 N_soot, ln S_l, T."""
        import numpy as np
        import torch
        self._check(U)
        if F is None:
            F = torch.empty((self.nr * self.nx, 19), dtype=torch.float32, device="cuda")
        si = np.ascontiguousarray(s_in, dtype=np.float32)
        assert si.size == NV and F.is_contiguous() and F.numel() == self.nr * self.nx * 19
        self._chk(self.L.cp_sur_features(self.h, _ptr(U), float(dt), si.ctypes.data, _ptr(F)))
        return F

    def particle_times(self, U):
        """Response time and Stokes number of droplets and crystals (Eq. 24
        diagnostics): two float64 CUDA tensors [2][nr][nx]."""
        import torch
        self._check(U)
        tau = torch.empty((2, self.nr, self.nx), dtype=torch.float64, device="cuda")
        St = torch.empty_like(tau)
        self._chk(self.L.cp_particle_times(self.h, _ptr(U), _ptr(tau), _ptr(St)))
        return tau, St

    def faces(self):
        import numpy as np
        xf = np.zeros(self.nx + 1)
        rf = np.zeros(self.nr + 1)
        self._chk(self.L.cp_mesh_faces(self.h, xf.ctypes.data_as(_DP), rf.ctypes.data_as(_DP)))
        return xf, rf


class Batch:
    """Many plumes advanced together (a cp_batch); U[p] are torch CUDA tensors."""

    def __init__(self, meshes, cases, precision=CP_MIXED, stream=None):
        self.L = load()
        self.n = len(meshes)
        self.precision = precision
        self._mesh_structs = [make_mesh(m) for m in meshes]   # keep any area arrays alive
        self._m = (CpMesh * self.n)(*self._mesh_structs)
        self._c = (CpCase * self.n)(*[make_case(c) for c in cases])
        self.shapes = [(int(m["nr"]), int(m["nx"])) for m in meshes]
        h = _P()
        s = _current_stream() if stream is None else stream
        rc = self.L.cp_batch_create(self.n, ctypes.cast(self._m, _P), ctypes.cast(self._c, _P), int(precision), s,
                                    ctypes.byref(h))
        if rc != CP_OK:
            raise ContrailError(rc, "cp_batch_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.cp_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc != CP_OK:
            raise ContrailError(rc, self.L.cp_batch_error_string(self.h).decode())

    def _ptrs(self, Us):
        assert len(Us) == self.n
        return (ctypes.c_void_p * self.n)(*[u.data_ptr() for u in Us])

    def empty(self):
        import torch
        dt = torch.float64 if self.precision == CP_FP64 else torch.float32
        return [torch.empty((NV, nr, nx), dtype=dt, device="cuda") for nr, nx in self.shapes]

    def init(self, Us=None):
        Us = self.empty() if Us is None else Us
        self._keep = self._ptrs(Us)
        self._chk(self.L.cp_batch_init(self.h, ctypes.cast(self._keep, _P)))
        return Us

    def step_n(self, Us, n):
        self._keep = self._ptrs(Us)
        t = (ctypes.c_double * self.n)()
        self._chk(self.L.cp_batch_step_n(self.h, ctypes.cast(self._keep, _P), int(n), t))
        return list(t)


class MLP:
    """BF16 MFMA multilayer perceptron of the C ABI (cp_mlp); X, T, Y are float32
    CUDA tensors [rows][features]; parameters move as float32 numpy arrays."""

    def __init__(self, n_in=17, n_hidden=256, n_out=15, stream=None):
        self.L = load()
        self.dims = (n_in, n_hidden, n_out)
        h = _P()
        s = _current_stream() if stream is None else stream
        rc = self.L.cp_mlp_create(n_in, n_hidden, n_out, s, ctypes.byref(h))
        if rc != CP_OK:
            raise ContrailError(rc, "cp_mlp_create failed")
        self.h = h
        self.n_params = int(self.L.cp_mlp_num_params(h))

    def close(self):
        if getattr(self, "h", None):
            self.L.cp_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc != CP_OK:
            raise ContrailError(rc, self.L.cp_mlp_error_string(self.h).decode())

    def set_params(self, theta):
        import numpy as np
        t = np.ascontiguousarray(theta, dtype=np.float32)
        assert t.size == self.n_params
        self._chk(self.L.cp_mlp_set_params(self.h, t.ctypes.data))

    def get_params(self):
        import numpy as np
        t = np.zeros(self.n_params, dtype=np.float32)
        self._chk(self.L.cp_mlp_get_params(self.h, t.ctypes.data))
        return t

    def forward(self, X):
        import torch
        assert X.dtype == torch.float32 and X.is_cuda and X.is_contiguous()
        Y = torch.empty((X.shape[0], self.dims[2]), dtype=torch.float32, device="cuda")
        self._chk(self.L.cp_mlp_forward(self.h, X.data_ptr(), int(X.shape[0]), Y.data_ptr()))
        return Y

    def forward_static(self, X, Y=None):
        """cp_mlp_forward without any allocation by the library (the call's scratch is
        a static device array shared by every call on the GPU; at most 65536 rows)."""
        import torch
        assert X.dtype == torch.float32 and X.is_cuda and X.is_contiguous()
        if Y is None:
            Y = torch.empty((X.shape[0], self.dims[2]), dtype=torch.float32, device="cuda")
        assert Y.dtype == torch.float32 and Y.is_cuda and Y.is_contiguous()
        self._chk(self.L.cp_mlp_forward_static(self.h, X.data_ptr(), int(X.shape[0]), Y.data_ptr()))
        return Y

    def loss_grad(self, X, T, want_grad=False):
        import numpy as np
        loss = ctypes.c_double()
        g = np.zeros(self.n_params, dtype=np.float32) if want_grad else None
        self._chk(self.L.cp_mlp_loss_grad(self.h, X.data_ptr(), T.data_ptr(), int(X.shape[0]), ctypes.byref(loss),
                                          g.ctypes.data if want_grad else None))
        return (loss.value, g) if want_grad else loss.value

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self._chk(self.L.cp_mlp_adam(self.h, float(lr), float(beta1), float(beta2), float(eps)))
