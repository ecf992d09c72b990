"""Host-side checks of the boundary: the C-ABI library loads without a GPU and
exports every function that include/contrail.h declares (no compute calls)."""
import ctypes
import os

import pytest

from paper_2504_20742_amd import binding


def test_library_exports_header_symbols():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    L = binding.load()
    names = binding.header_functions()
    assert "cp_create" in names and "cp_step_n" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_struct_layouts_match_header():
    """Field counts and sizes of the marshalled structs follow the header."""
    assert ctypes.sizeof(binding.CpMesh) == 2 * 4 + 5 * 8 + 5 * 4 + 4 + 8   # padding, area_x pointer
    assert binding.CpMesh.area_x.offset == 72
    assert ctypes.sizeof(binding.CpCase) == 22 * 8 + 4 * 4


def test_create_rejects_bad_arguments_without_gpu():
    """Argument validation happens before any device call."""
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    L = binding.load()
    from paper_2504_20742_amd import inputs
    m, c = inputs.config1(1)
    m["nx"] = 1
    h = ctypes.c_void_p()
    rc = L.cp_create(ctypes.byref(binding.make_mesh(m)), ctypes.byref(binding.make_case(c)), 0, None,
                     ctypes.byref(h))
    assert rc == binding.CP_EINVAL
    m["nx"] = 16
    rc = L.cp_create(ctypes.byref(binding.make_mesh(m)), ctypes.byref(binding.make_case(c)), 7, None,
                     ctypes.byref(h))
    assert rc == binding.CP_EINVAL


def test_create_rejects_bad_duct_meshes_without_gpu():
    """The quasi-1D duct needs one row, slip walls on both r sides and nx+1 finite
    positive face areas; each violation is rejected before any device call."""
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    import numpy as np
    L = binding.load()
    from paper_2504_20742_amd import inputs
    c = binding.make_case(inputs.case(phase_change=0))
    wall = (inputs.BC_INFLOW, inputs.BC_COPY, inputs.BC_WALL, inputs.BC_WALL)

    def create(m):
        h = ctypes.c_void_p()
        return L.cp_create(ctypes.byref(binding.make_mesh(m)), ctypes.byref(c), 0, None, ctypes.byref(h))

    bad = []
    m = inputs.mesh(16, 2, geom=inputs.GEOM_QUASI1D, bc=wall)            # two rows
    m["area_x"] = np.ones(17)
    bad.append(m)
    m = inputs.mesh(16, 1, geom=inputs.GEOM_QUASI1D, bc=wall)            # no areas
    bad.append(m)
    for v in (0.0, -1.0, np.nan, np.inf):                                 # a bad area
        m = inputs.mesh(16, 1, geom=inputs.GEOM_QUASI1D, bc=wall)
        a = np.ones(17)
        a[5] = v
        m["area_x"] = a
        bad.append(m)
    m = inputs.mesh(16, 1, geom=inputs.GEOM_QUASI1D,                     # far field in r
                    bc=(inputs.BC_INFLOW, inputs.BC_COPY, inputs.BC_WALL, inputs.BC_FARFIELD))
    m["area_x"] = np.ones(17)
    bad.append(m)
    m = inputs.mesh(16, 1, geom=inputs.GEOM_PLANAR, bc=wall)              # one row, not a duct
    bad.append(m)
    m = inputs.mesh(16, 4, geom=3, bc=wall)                               # unknown geometry
    bad.append(m)
    for m in bad:
        assert create(m) == binding.CP_EINVAL, m


def test_batch_rejects_duct_without_gpu():
    """The batch runs axisymmetric and planar plumes; a duct is refused up front."""
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    import numpy as np
    L = binding.load()
    from paper_2504_20742_amd import inputs
    m = inputs.mesh(16, 1, geom=inputs.GEOM_QUASI1D,
                    bc=(inputs.BC_INFLOW, inputs.BC_COPY, inputs.BC_WALL, inputs.BC_WALL))
    m["area_x"] = np.ones(17)
    ms = (binding.CpMesh * 1)(binding.make_mesh(m))
    cs = (binding.CpCase * 1)(binding.make_case(inputs.case(phase_change=0)))
    h = ctypes.c_void_p()
    rc = L.cp_batch_create(1, ctypes.cast(ms, ctypes.c_void_p), ctypes.cast(cs, ctypes.c_void_p), 1, None,
                           ctypes.byref(h))
    assert rc == binding.CP_EUNSUPPORTED


def test_create_rejects_oversized_mesh_without_gpu():
    """At most 2^28 cells per context (a state plane stays below 2 GiB)."""
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    L = binding.load()
    from paper_2504_20742_amd import inputs
    m = inputs.mesh(1 << 15, (1 << 13) + 1)
    h = ctypes.c_void_p()
    rc = L.cp_create(ctypes.byref(binding.make_mesh(m)), ctypes.byref(binding.make_case(inputs.case())), 0, None,
                     ctypes.byref(h))
    assert rc == binding.CP_EINVAL
