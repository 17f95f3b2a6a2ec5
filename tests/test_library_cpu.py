"""Host-side checks of libcbs that need no GPU: the library loads, exports
every symbol include/cbs.h declares, and rejects bad arguments before any
device call."""

import ctypes
import os
import re

import pytest

from paper_2506_15411_amd import libcbs as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "cbs.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cbs_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libcbs.so is not built (python -m paper_2506_15411_amd.build)")
    return L.load()


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), f"missing export {n}"
    assert set(names) <= set(L.SYMBOLS)


@pytest.mark.parametrize("n", [2, 3, 5, 8, 16, 29, 64, 128, 192, 256, 261, 275, 315, 621])
def test_supported_axis_lengths(lib, n):
    assert L.cbs_axis_supported(0, n) and L.cbs_axis_supported(1, n)


def test_unsupported_lengths(lib):
    assert not L.cbs_axis_supported(0, 1)
    assert not L.cbs_axis_supported(0, 37 * 41)
    assert not L.cbs_axis_supported(2, 621)      # x/y only
    assert not L.cbs_axis_supported(3, 64)
    assert L.cbs_plan_workspace_bytes(621, 621, 621) == 0
    assert L.cbs_plan_workspace_bytes(1, 8, 8) == 0


def test_workspace_bytes_cover_fields():
    # W (24 B/voxel, row pitch padded to 8) + V0 (8 B/voxel) + tables, partial
    # sums and the lens-metric scratch (five FP64 complex planes)
    for (nx, ny, nz) in [(64, 64, 64), (275, 275, 315), (621, 621, 261)]:
        b = L.cbs_plan_workspace_bytes(nx, ny, nz)
        nxp = (nx + 7) // 8 * 8
        assert b >= 24 * nxp * ny * nz + 8 * nx * ny * nz + 5 * 16 * nx * ny
        assert b < (24 * nxp * ny * nz + 8 * nx * ny * nz + 4 * 2 ** 20 + 16 * ny * nz
                    + 5 * 16 * nx * ny + 16 * (nx + ny))


def _create(nx, ny, nz, pitch=1e-7, lam=1e-6, nbg=1.0, pml=(0, 0, 0), ws=None, wsb=0):
    h = ctypes.c_void_p()
    rc = L.load().cbs_plan_create(ctypes.byref(h), nx, ny, nz, pitch, lam, nbg,
                                  (ctypes.c_int * 3)(*pml), ws, wsb, None)
    return rc, L.cbs_last_error()


@pytest.mark.parametrize("args,code,frag", [
    (dict(nx=1, ny=8, nz=8), L.CBS_E_INVALID, ">= 2"),
    (dict(nx=37 * 41, ny=8, nz=8), L.CBS_E_INVALID, "specialisation"),
    (dict(nx=8, ny=8, nz=8, pitch=0.0), L.CBS_E_INVALID, "pitch"),
    (dict(nx=8, ny=8, nz=8, lam=-1.0), L.CBS_E_INVALID, "lambda0"),
    (dict(nx=8, ny=8, nz=8, nbg=0.0), L.CBS_E_INVALID, "n_bg"),
    (dict(nx=8, ny=8, nz=8, pml=(4, 0, 0)), L.CBS_E_INVALID, "pml"),
    (dict(nx=8, ny=8, nz=8), L.CBS_E_WORKSPACE, "NULL"),
    (dict(nx=8, ny=8, nz=8, ws=256, wsb=16), L.CBS_E_WORKSPACE, "required"),
    (dict(nx=8, ny=8, nz=8, ws=100, wsb=1 << 30), L.CBS_E_WORKSPACE, "aligned"),
])
def test_plan_create_rejects_bad_arguments(lib, args, code, frag):
    rc, msg = _create(**args)
    assert rc == code
    assert frag in msg


def test_calls_on_null_plan_fail(lib):
    assert lib.cbs_set_permittivity(None, None, 0) == L.CBS_E_INVALID
    assert lib.cbs_solve(None, None, None, None, None) == L.CBS_E_INVALID
    assert lib.cbs_eps_shift(None) < 0
    assert lib.cbs_plan_destroy(None) == L.CBS_OK


def test_static_solve_checks_before_any_device_call(lib):
    """cbs_solve_static validates the grid and its scratch size on the host."""
    hdr = open(os.path.join(ROOT, "include", "cbs.h")).read()
    m = re.search(r"#define CBS_STATIC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", hdr)
    assert m and int(m.group(1)) << int(m.group(2)) == L.CBS_STATIC_SCRATCH_BYTES
    opts = L.cbs_opts(1e-4, 10, 10, 0)
    st = L.cbs_stats()
    pml = (ctypes.c_int * 3)(8, 8, 48)
    rc = lib.cbs_solve_static(275, 275, 315, 66.5e-9, 1.064e-6, 1.0, pml, None, 0, None, None,
                              ctypes.byref(opts), ctypes.byref(st), None)
    assert rc == L.CBS_E_WORKSPACE and b"static scratch" in lib.cbs_last_error()
    rc = lib.cbs_solve_static(37 * 41, 8, 8, 1e-7, 1e-6, 1.0, None, None, 0, None, None,
                              ctypes.byref(opts), ctypes.byref(st), None)
    assert rc == L.CBS_E_INVALID
    assert L.cbs_plan_workspace_bytes(128, 128, 128) <= L.CBS_STATIC_SCRATCH_BYTES


def test_stretched_layer_workspace_bytes(lib):
    """cbs_scpml_workspace_bytes is host arithmetic: restart + 4 vector fields,
    two scalar fields and 3 n^2 complex64 per axis, or 0 out of range."""
    nx, ny, nz = 24, 20, 32
    n = nx * ny * nz
    b1 = L.cbs_scpml_workspace_bytes(nx, ny, nz, 1)
    b40 = L.cbs_scpml_workspace_bytes(nx, ny, nz, 40)
    assert b1 >= (2 + 2) * 3 * n * 8 + 2 * n * 8 + 3 * 8 * (nx * nx + ny * ny + nz * nz)
    assert b40 - b1 >= 39 * 3 * n * 8
    assert L.cbs_scpml_workspace_bytes(nx, ny, nz, 0) == 0
    assert L.cbs_scpml_workspace_bytes(nx, ny, nz, 65) == 0
    assert L.cbs_scpml_workspace_bytes(37 * 41, ny, nz, 4) == 0
    opts = L.cbs_opts(1e-4, 10, 10, 0)
    layer = L.cbs_scpml(1.5, 2, 8)
    rc = lib.cbs_solve_scpml(None, None, None, ctypes.byref(opts), ctypes.byref(layer), None,
                             None, 0)
    assert rc == L.CBS_E_INVALID
