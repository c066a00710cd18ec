"""The C-ABI library loads and exports every symbol include/abba.h declares.

These run without a GPU: only argument validation that fails before any HIP
call is exercised.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "abba.h")
LIB = os.path.join(ROOT, "paper_2602_17892_amd", "libabba.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(abba_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.fail("libabba.so is not built (python paper_2602_17892_amd/build.py)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("abba_project", "abba_backproject", "abba_solve", "abba_solve_workspace", "abba_op_create"):
        assert n in names


def test_every_declared_symbol_is_exported(L):
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings_and_version(L):
    L.abba_status_str.restype = ctypes.c_char_p
    L.abba_version.restype = ctypes.c_char_p
    assert L.abba_status_str(0) == b"ok"
    assert L.abba_status_str(-2) == b"shape mismatch"
    assert b"gfx950" in L.abba_version()


def test_validation_before_any_device_call():
    import paper_2602_17892_amd as pk
    h = ctypes.c_void_p()
    # NULL geometry
    assert pk.lib.abba_op_create(ctypes.byref(h), 0, None, 1, 1) == -1
    g = pk.Geometry(8, 8, 12, 13)
    cg, keep = g._c()
    # unknown op kind
    assert pk.lib.abba_op_create(ctypes.byref(h), 7, ctypes.byref(cg), 1, 1) == -1
    # unsupported dtype pair (F64 image with F32 sinogram)
    assert pk.lib.abba_op_create(ctypes.byref(h), 0, ctypes.byref(cg), 0, 1) == -3
    # bad sizes
    bad = pk.Geometry(0, 8, 12, 13)._c()[0]
    assert pk.lib.abba_op_create(ctypes.byref(h), 0, ctypes.byref(bad), 1, 1) == -1
    bad = pk.Geometry(8, 8, 12, 13, det_pitch_u=-1.0)._c()[0]
    assert pk.lib.abba_op_create(ctypes.byref(h), 0, ctypes.byref(bad), 1, 1) == -1
    # exact transpose is 2D only
    cone = pk.Geometry(8, 8, 12, 13, kind="cone3d", nz=8, det_v=9, sid=30.0, sdd=60.0)._c()[0]
    assert pk.lib.abba_op_create(ctypes.byref(h), 2, ctypes.byref(cone), 1, 1) == -7
    bad = pk.Geometry(8, 8, 12, 13, kind="cone3d", nz=8, det_v=9, sid=60.0, sdd=30.0)._c()[0]
    assert pk.lib.abba_op_create(ctypes.byref(h), 0, ctypes.byref(bad), 1, 1) == -1
    # NULL handles
    nb0 = ctypes.c_size_t()
    assert pk.lib.abba_project(None, None, None, 1, None, 0, None) == -1
    assert pk.lib.abba_backproject(None, None, None, 1, None, 0, None) == -1
    assert pk.lib.abba_project_workspace(None, 1, ctypes.byref(nb0)) == -1
    assert pk.lib.abba_backproject_workspace(None, 1, ctypes.byref(nb0)) == -1
    assert pk.lib.abba_autotune_workspace(None, 1, ctypes.byref(nb0)) == -1
    assert pk.lib.abba_mlp_loss_grad_workspace(0, ctypes.byref(nb0)) == -1
    assert pk.lib.abba_mlp_loss_grad_workspace(64, None) == -1
    assert pk.lib.abba_mlp_loss_grad_workspace(64, ctypes.byref(nb0)) == 0 and nb0.value > 64 * 4
    nb = ctypes.c_size_t()
    assert pk.lib.abba_solve_workspace(None, None, 1, 0, 5, None, None, ctypes.byref(nb)) == -1
    lay = pk._Layout()
    assert pk.lib.abba_solve_layout(None, None, 1, 0, 5, None, None, ctypes.byref(lay)) == -1
    assert pk.lib.abba_solve_layout(None, None, 1, 0, 5, None, None, None) == -1
    assert pk.lib.abba_solve(None, None, None, None, 1, 0, 5, None, None, None, None, None, 0, None) == -1
    assert b"required" in pk.lib.abba_last_error()
    # concurrent sub-batches: a negative count is an argument error, and the
    # layout query covers one stream's workspace only
    ex = pk._Exec()
    ex.streams = -1
    assert pk.lib.abba_solve_workspace(None, None, 4, 0, 5, None, ctypes.byref(ex), ctypes.byref(nb)) == -1
    assert b"streams" in pk.lib.abba_last_error()
    assert pk.lib.abba_solve(None, None, None, None, 4, 0, 5, None, None, None, ctypes.byref(ex), None, 0,
                             None) == -1
    ex.streams = 2
    assert pk.lib.abba_solve_layout(None, None, 4, 0, 5, None, ctypes.byref(ex), ctypes.byref(lay)) == -7
    assert b"one stream" in pk.lib.abba_last_error()
    assert pk.lib.abba_solve(None, None, None, None, 4, 0, 5, None, None, None, ctypes.byref(ex), None, 0,
                             None) == -1
    assert b"required" in pk.lib.abba_last_error()
    del keep


def test_validation_of_the_newer_entry_points():
    import paper_2602_17892_amd as pk
    h = ctypes.c_void_p()
    # fan beam: the source must lie outside the image and before the detector
    bad = pk.Geometry(64, 64, 12, 13, kind="fan2d", sid=20.0, sdd=80.0)._c()[0]
    assert pk.lib.abba_op_create(ctypes.byref(h), 0, ctypes.byref(bad), 1, 1) == -1
    bad = pk.Geometry(8, 8, 12, 13, kind="fan2d", sid=60.0, sdd=30.0)._c()[0]
    assert pk.lib.abba_op_create(ctypes.byref(h), 0, ctypes.byref(bad), 1, 1) == -1
    fan = pk.Geometry(8, 8, 12, 13, kind="fan2d", sid=30.0, sdd=60.0)._c()[0]
    assert pk.lib.abba_op_create(ctypes.byref(h), 2, ctypes.byref(fan), 1, 1) == -7   # no exact transpose
    bad = pk.Geometry(8, 8, 12, 13, kind="fan2d", nz=3, sid=30.0, sdd=60.0)._c()[0]
    assert pk.lib.abba_op_create(ctypes.byref(h), 0, ctypes.byref(bad), 1, 1) == -1
    # learned network calls
    assert pk.lib.abba_mlp_forward(None, None, 5, None, None) == -1
    assert pk.lib.abba_mlp_forward(None, None, 0, None, None) == 0          # nothing to do
    assert pk.lib.abba_mlp_forward(None, None, -1, None, None) == -1
    assert pk.lib.abba_mlp_loss_grad(None, None, None, 4, None, 4, None, None, None, 0, None) == -1
    assert pk.lib.abba_mlp_adam(None, None, None, None, 1, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert pk.lib.abba_mlp_labels(None, 1, 5, None, None, None, None) == -1
    # tuning
    t = pk._Tune()
    assert pk.lib.abba_autotune(None, 4, 3, None, 0, None, ctypes.byref(t)) == -1
    assert pk.lib.abba_op_set_tuning(None, 4, ctypes.byref(t)) == -1
    assert pk.lib.abba_op_get_tuning(None, 4, ctypes.byref(t)) == -1


# ctypes field name -> C field name where they differ (`lambda` is a Python keyword)
_C_NAMES = {("abba_reg", "lam"): "lambda", ("abba_out", "lam"): "lambda"}


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structures have the sizes and field offsets of the
    C structures in include/abba.h (compiled here by gcc)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    if not os.path.exists(LIB):
        pytest.fail("libabba.so is not built (python paper_2602_17892_amd/build.py)")
    import paper_2602_17892_amd as pk
    structs = {"abba_geometry": pk._Geometry, "abba_reg": pk._Reg, "abba_stop": pk._Stop, "abba_out": pk._Out,
               "abba_exec": pk._Exec, "abba_tune": pk._Tune, "abba_basis_layout": pk._Layout}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "abba.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            c = _C_NAMES.get((cname, fname), fname)
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {c}));')
    lines.append("return 0; }")
    src, exe = tmp_path / "layout.c", tmp_path / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
