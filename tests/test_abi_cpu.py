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


def _atoms_desc(natoms, n=(12, 12, 12), h=0.2, rc=0.5):
    """Descriptor of natoms atoms stacked on one site (every point of the
    sphere then carries natoms entries); keeps its host arrays alive."""
    import numpy as np
    from paper_2310_14776_amd._binding import SysDesc, Channel
    chans = (Channel * 1)(Channel(0, rc / 3.0, rc))
    pos = np.ascontiguousarray(np.tile([[1.2, 1.2, 1.2]], (natoms, 1)))
    dH = np.zeros((natoms, 1, 1))
    dS = np.zeros((natoms, 1, 1))
    v = np.zeros(n)
    dp = ctypes.POINTER(ctypes.c_double)
    d = SysDesc()
    d.n[:] = n
    d.h[:] = (h, h, h)
    d.dtype = 0
    d.natoms = natoms
    d.pos = pos.ctypes.data_as(dp)
    d.nchan = 1
    d.chan = chans
    d.dH = dH.ctypes.data_as(dp)
    d.dS = dS.ctypes.data_as(dp)
    d.v = v.ctypes.data_as(dp)
    d.max_bands = 1
    return d, (chans, pos, dH, dS, v)


def test_too_many_entries_at_one_point_is_rejected_on_the_host(lib):
    # 256 spheres through one grid point exceed the 8-bit per-point count;
    # the check runs while the tables are built on the host, before any
    # device call, so it holds without a GPU
    d, keep = _atoms_desc(256)
    out = ctypes.c_void_p()
    assert lib.gpaw_sys_create(ctypes.byref(d), ctypes.byref(out)) == -1
    assert b"255 projector entries" in lib.gpaw_last_error()
    assert out.value is None


def test_counts_above_127_pass_the_host_table_check(lib):
    # 200 entries per point used to wrap through a signed shift; the host
    # check must accept it (with no GPU the call then stops at the device)
    d, keep = _atoms_desc(200)
    out = ctypes.c_void_p()
    rc = lib.gpaw_sys_create(ctypes.byref(d), ctypes.byref(out))
    if rc != 0:
        assert b"255 projector entries" not in lib.gpaw_last_error()
    else:
        lib.gpaw_sys_destroy(out)
