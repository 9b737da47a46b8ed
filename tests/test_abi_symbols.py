"""The C-ABI library loads on a CPU-only host and exports every entry point
include/ultima.h declares (no compute calls: those need the GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ultima.h")
LIB = os.path.join(ROOT, "paper_2303_13435_amd", "libultima.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ur_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def built_lib():
    if not os.path.exists(LIB):
        from paper_2303_13435_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_path_entry_points():
    syms = declared_symbols()
    for name in ("ur_plan_create", "ur_rho_generate", "ur_fft3d_exec", "ur_intensity_bin",
                 "ur_merge_zooms", "ur_simulate", "ur_adjoint", "ur_simulate_host"):
        assert name in syms


def test_library_exports_every_declared_symbol(built_lib):
    missing = [s for s in declared_symbols() if not hasattr(built_lib, s)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    import paper_2303_13435_amd as ur
    assert sorted(ur.EXPORTS) == declared_symbols()


def test_version_and_errors_without_gpu(built_lib):
    built_lib.ur_version.restype = ctypes.c_char_p
    assert built_lib.ur_version().startswith(b"ultima")
    # argument validation happens before any device call
    built_lib.ur_plan_create.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_uint32,
                                         ctypes.POINTER(ctypes.c_void_p)]
    h = ctypes.c_void_p()
    assert built_lib.ur_plan_create(120, 1.0, 0, 0, ctypes.byref(h)) == 1       # neither 2^a nor a mixed-radix edge
    built_lib.ur_last_error.restype = ctypes.c_char_p
    assert b"power of two" in built_lib.ur_last_error()
    assert built_lib.ur_plan_create(100, 1.0, 0, 2, ctypes.byref(h)) == 1       # unknown flag
    assert built_lib.ur_plan_create(64, -1.0, 0, 0, ctypes.byref(h)) == 1       # bad voxel
    assert built_lib.ur_plan_create(64, 1.0, 7, 0, ctypes.byref(h)) == 1        # bad precision
    # box limits: 4096^3 only in FP32 real, nothing above; complex only up to 1024^3
    assert built_lib.ur_plan_create(8192, 1.0, 0, 0, ctypes.byref(h)) == 2
    assert built_lib.ur_plan_create(4096, 1.0, 1, 0, ctypes.byref(h)) == 2      # FP64
    assert built_lib.ur_plan_create(4096, 1.0, 0, 1, ctypes.byref(h)) == 2      # complex
    assert built_lib.ur_plan_create(2048, 1.0, 0, 1, ctypes.byref(h)) == 2      # complex above 1024
    assert not h.value


def test_struct_layouts_match_the_header(tmp_path):
    """Every struct the binding passes by pointer has the header's size and
    field offsets (a C program built with gcc from include/ultima.h prints
    them)."""
    import shutil
    import subprocess
    import paper_2303_13435_amd as ur
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    pairs = {"ur_cell": ur.UrCell, "ur_mask": ur.UrMask, "ur_zoom": ur.UrZoom, "ur_hist": ur.UrHist,
             "ur_ewald": ur.UrEwald}
    lines = ['#include <stdio.h>', '#include "ultima.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_peak_integrals_argument_checks_without_gpu(built_lib):
    """ur_peak_integrals validates before any device call: null pointers, a
    bin or window count out of range and windows that are empty or not
    finite are refused (UR_ERR_INVALID) on a host without a GPU."""
    f = built_lib.ur_peak_integrals
    f.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                  ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.c_void_p]
    buf = (ctypes.c_double * 16)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    win = (ctypes.c_double * 4)(1.0, 2.0, 3.0, 4.0)
    assert f(8, None, p, 1, win, p, None) == 1
    assert f(0, p, p, 1, win, p, None) == 1
    assert f(8, p, p, 0, win, p, None) == 1
    assert f(8, p, p, 65, win, p, None) == 1
    assert f(8, p, p, 1, (ctypes.c_double * 2)(2.0, 2.0), p, None) == 1
    assert f(8, p, p, 2, (ctypes.c_double * 4)(1.0, 2.0, float("nan"), 4.0), p, None) == 1
