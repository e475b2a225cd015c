"""The C ABI library loads, exports every symbol include/mproj.h declares and
rejects bad arguments before touching a device (no compute without a GPU)."""
import ctypes
import os
import re

import pytest
import torch

from paper_1908_03634_amd import mproj

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mproj.h")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\s*\*)\s*\*?\s*(mp_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_four_named_entry_points():
    names = declared()
    for n in ("mp_init", "mp_map_base_state", "mp_mac_project", "mp_free"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = mproj.load_library()
    names = declared()
    assert names, "no declarations parsed"
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(mproj.EXPORTS) == names


def _cfg(nx=8, ny=8, nz=8):
    lib = mproj.load_library()
    c = mproj.Config()
    lib.mp_config_default(ctypes.byref(c), nx, ny, nz)
    return lib, c


def _init(c):
    lib = mproj.load_library()
    h = ctypes.c_void_p()
    return lib.mp_init(ctypes.byref(c), ctypes.byref(h)), h


def test_defaults():
    lib, c = _cfg(16, 16, 32)
    assert c.h == pytest.approx(1 / 32) and c.rtol == 1e-10 and c.nu1 == 2 and c.nu2 == 2
    assert list(c.bc) == [0, 0, 1] and c.precision == mproj.MIXED and c.demean == 1


@pytest.mark.parametrize("field,value", [("nx", 0), ("h", 0.0), ("rtol", 0.0), ("rtol", 1.5), ("precision", 7),
                                         ("nu1", -1), ("cycles_per_outer", -1), ("demean", 3),
                                         ("bottom_max_iter", 0), ("smoother", 9), ("coarse_cycle", 2),
                                         ("blocked", 2)])
def test_bad_config_is_rejected_before_any_device_call(field, value):
    lib, c = _cfg()
    setattr(c, field, value)
    code, h = _init(c)
    assert code == 1 and not h.value


def test_bad_bc_and_uncoarsenable_grid_are_rejected():
    lib, c = _cfg()
    c.bc[1] = 5
    assert _init(c)[0] == 1
    lib, c = _cfg(129, 129, 129)  # odd: the coarsest grid would hold 129^3 cells
    assert _init(c)[0] == 1


def test_null_arguments():
    lib = mproj.load_library()
    assert lib.mp_init(None, None) == 1
    assert lib.mp_free(None) == 0
    assert isinstance(lib.mp_last_error(None), bytes)
    assert lib.mp_map_base_state(None, 0, None, 0, 0.0, None, None, None, None, None) == 1
    assert lib.mp_mac_project(None, None, None, None, None, None, 0, None) == 1
    assert lib.mp_solve(None, None, None, 0, None) == 1
    assert lib.mp_nodal_project(None, None, None, None, None, None, 0, None) == 1
    assert lib.mp_nodal_apply(None, None, None) == 1
    assert lib.mp_nodal_shape(None, None, None, None) == 1
    assert lib.mp_base_radii(None, None, None) == 1
    assert lib.mp_enforce_hse(None, 0, None, None, None, 0.0, 0.0, None, None) == 1
    assert lib.mp_beta0_from_p0(None, 0, 1.0, None, None, None) == 1
    assert lib.mp_w0(None, 0, 0, None, None, None, None, None, None) == 1
    assert lib.mp_set_coefs(None, None, None, None) == 1
    assert lib.mp_set_kernel_timing(None, 1) == 1
    assert lib.mp_radius_count(None, None) == 1
    assert lib.mp_mac_project_split(None, None, None, None, None, None, 0, None, None) == 1
    assert lib.mp_average(None, None, None, None) == 1
    assert lib.mp_apply(None, None, None) == 1
    assert lib.mp_coef_grad(None, None, None, None, None, None) == 1
    assert lib.mp_version().startswith(b"mproj")


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-device path")
def test_init_reports_missing_device():
    lib, c = _cfg()
    code, h = _init(c)
    assert code == 2 and not h.value
