"""Host-side checks of the C-ABI library (no GPU needed, no compute calls).

The library must build for gfx950, load, and export exactly the entry points
that include/gpaw_fd.h declares; argument validation that precedes any device
call must reject bad descriptors.
"""
import ctypes
import os
import re

import pytest

import paper_2310_14776_amd as lib_pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpaw_fd.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"GPAW_API\s+[\w\s\*]*?\b(gpaw_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lib_pkg.library_path()):
        from paper_2310_14776_amd.build import build
        build()
    return lib_pkg.load()


def test_header_declares_the_step_calls():
    names = _declared()
    for required in ("gpaw_fd_apply_H", "gpaw_fd_apply_S", "gpaw_project",
                     "gpaw_subspace_matrices", "gpaw_rotate", "gpaw_subspace_diag"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(_declared()) == sorted(lib_pkg.ENTRY_POINTS)


def test_only_abi_symbols_are_exported():
    out = os.popen(f"nm -D --defined-only {lib_pkg.library_path()}").read()
    exported = sorted(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert exported == _declared()


def test_version_matches_header(lib):
    m = re.search(r"#define GPAW_FD_VERSION (\d+)", open(HEADER).read())
    assert lib.gpaw_version() == int(m.group(1))


def test_create_rejects_bad_descriptors_before_any_device_call(lib):
    from paper_2310_14776_amd._binding import SysDesc
    out = ctypes.c_void_p()
    assert lib.gpaw_sys_create(None, ctypes.byref(out)) == -1
    d = SysDesc()
    d.n[:] = (0, 4, 4)
    d.h[:] = (0.2, 0.2, 0.2)
    d.max_bands = 1
    assert lib.gpaw_sys_create(ctypes.byref(d), ctypes.byref(out)) == -1
    assert b"grid sizes" in lib.gpaw_last_error()
    d.n[:] = (4, 4, 4)
    d.k[:] = (0.25, 0.0, 0.0)
    d.dtype = 0
    assert lib.gpaw_sys_create(ctypes.byref(d), ctypes.byref(out)) == -2   # real needs k = 0
    d.k[:] = (0.0, 0.0, 0.0)
    d.dtype = 7
    assert lib.gpaw_sys_create(ctypes.byref(d), ctypes.byref(out)) == -2
    assert out.value is None


def test_compute_calls_reject_null_system(lib):
    assert lib.gpaw_project(None, None, 1, None, None) == -1
    assert lib.gpaw_fd_apply_H(None, None, 1, None, None, None) == -1
    assert lib.gpaw_rotate(None, None, None, 1, None, None, None, None) == -1
    assert b"NULL" in lib.gpaw_last_error()
