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
    assert ctypes.sizeof(binding.CpMesh) == 2 * 4 + 5 * 8 + 5 * 4 + 4   # padded to 8
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
