"""The C-ABI library loads and exports every symbol include/nuht.h declares,
and rejects invalid arguments before touching the GPU (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "nuht.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nuht_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_2411_09583_amd as nuht
    return nuht.load_library()


def test_header_declares_the_boundary():
    names = declared_symbols()
    for n in ("nuht_plan", "nuht_execute", "nuht_adjoint", "nuht_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    import paper_2411_09583_amd as nuht
    names = declared_symbols()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(nuht.EXPORTS) == names


def test_strerror(lib):
    assert lib.nuht_strerror(0) == b"success"
    for code in (-1, -2, -3, -4, -5, -6, -7):
        assert lib.nuht_strerror(code) != b"unknown error"


def test_invalid_arguments_rejected_without_gpu(lib):
    import paper_2411_09583_amd as nuht
    h = ctypes.c_void_p()
    plan = lib.nuht_plan
    assert plan(ctypes.byref(h), 101, 1e-12, 0, None, 0, None, None, None) == -1      # |nu| > 100
    assert plan(ctypes.byref(h), 0, 1e-16, 0, None, 0, None, None, None) == -1        # eps too small
    assert plan(ctypes.byref(h), 0, 0.5, 0, None, 0, None, None, None) == -1          # eps too large
    assert plan(ctypes.byref(h), 0, 1e-12, -1, None, 0, None, None, None) == -1       # n < 0
    assert plan(ctypes.byref(h), 0, 1e-12, 10, None, 10, None, None, None) == -1      # null with n > 0
    assert plan(None, 0, 1e-12, 0, None, 0, None, None, None) == -1
    o = nuht.NuhtOpts(0, 0, 0, nuht.NUHT_FP32_SPREAD, 0)
    assert plan(ctypes.byref(h), 0, 1e-12, 0, None, 0, None, ctypes.byref(o), None) == -3   # FP32 below 1e-7
    assert plan(ctypes.byref(h), 0, 1e-8, 0, None, 0, None, ctypes.byref(o), None) == -3
    o = nuht.NuhtOpts(0, 21, 0, 0, 0)                                                 # M > 20
    assert plan(ctypes.byref(h), 0, 1e-12, 0, None, 0, None, ctypes.byref(o), None) == -1
    assert lib.nuht_execute(None, None, None, None) == -1
    assert lib.nuht_adjoint(None, None, None, None) == -1
    assert lib.nuht_destroy(None) == 0
    assert lib.nuht_direct(0, 1e-12, 5, None, None, 5, None, None, None) == -1


def test_new_entry_points_reject_invalid_arguments_without_gpu(lib):
    import paper_2411_09583_amd as nuht
    h = ctypes.c_void_p()
    # gradient, tuning and batches on a null plan / batch
    assert lib.nuht_gradient(None, None, None, None, None, None, None) == -1
    assert lib.nuht_gradient_noalloc(None, None, None, None, None, None, None) == -1
    best = nuht.NuhtOpts()
    assert lib.nuht_tune(None, None, 3, ctypes.byref(best), None, None) == -1
    assert lib.nuht_execute_many(None, None, None, None) == -1
    assert lib.nuht_batch_info(None, 0, None) == -1
    assert lib.nuht_batch_destroy(None) == 0
    assert lib.nuht_plan_set_order(None, 1, None) == -1
    assert lib.nuht_plan_order(None, None, None, None, None, None) == -1
    assert lib.nuht_profile_stages(None, 1) == -1
    assert lib.nuht_profile(None, 1) == -1
    # batch arguments are validated before anything is created
    many = lib.nuht_plan_many
    one = lambda t, v: (t * 1)(v)
    assert many(None, 0, None, 1e-12, None, None, None, None, None, None) == -1
    assert many(ctypes.byref(h), -1, None, 1e-12, None, None, None, None, None, None) == -1
    assert many(ctypes.byref(h), 1, None, 1e-12, None, None, None, None, None, None) == -1     # null arrays
    vp = ctypes.c_void_p
    nu = one(ctypes.c_int, 200)                                                                 # |nu| > 100
    n = one(ctypes.c_int64, 0)
    m = one(ctypes.c_int64, 0)
    r = (vp * 1)(None)
    w = (vp * 1)(None)
    assert many(ctypes.byref(h), 1, nu, 1e-12, n, r, m, w, None, None) == -1
    nu = one(ctypes.c_int, 0)
    n = one(ctypes.c_int64, 5)                                                                  # null r with n > 0
    assert many(ctypes.byref(h), 1, nu, 1e-12, n, r, m, w, None, None) == -1
    o = nuht.NuhtOpts(0, 0, 0, 0, 0, 17, 0)                                                     # spread_chunk < 64
    n = one(ctypes.c_int64, 0)
    assert many(ctypes.byref(h), 1, nu, 1e-12, n, r, m, w, ctypes.byref(o), None) == -1


def test_disk_solver_rejects_invalid_arguments_without_gpu(lib):
    h = ctypes.c_void_p()
    p = ctypes.c_void_p(8)              # a non-null stand-in, never dereferenced
    fbp = lib.nuht_fb_plan
    assert fbp(None, 2, 8, p, p, 8, 4, p, 1e-10, 0, None) == -1                       # no handle
    assert fbp(ctypes.byref(h), -1, 8, p, p, 8, 4, p, 1e-10, 0, None) == -1           # L < 0
    assert fbp(ctypes.byref(h), 101, 8, p, p, 256, 4, p, 1e-10, 0, None) == -1        # L > 100
    assert fbp(ctypes.byref(h), 2, 0, p, p, 8, 4, p, 1e-10, 0, None) == -1            # m = 0
    assert fbp(ctypes.byref(h), 2, 8, p, p, 12, 4, p, 1e-10, 0, None) == -1           # t not a power of two
    assert fbp(ctypes.byref(h), 2, 8, p, p, 8192, 4, p, 1e-10, 0, None) == -1         # t > 4096
    assert fbp(ctypes.byref(h), 4, 8, p, p, 8, 4, p, 1e-10, 0, None) == -1            # 2L + 1 > t
    assert fbp(ctypes.byref(h), 2, 8, p, p, 8, 0, p, 1e-10, 0, None) == -1            # J = 0
    assert fbp(ctypes.byref(h), 2, 8, None, p, 8, 4, p, 1e-10, 0, None) == -1         # null radii
    assert fbp(ctypes.byref(h), 2, 8, p, p, 8, 4, None, 1e-10, 0, None) == -1         # null zeros
    assert fbp(ctypes.byref(h), 2, 8, p, p, 8, 4, p, 1e-16, 0, None) == -1            # eps out of range
    assert fbp(ctypes.byref(h), 2, 8, p, p, 8, 4, p, 1e-10, 2, None) == -1            # unknown method
    assert fbp(ctypes.byref(h), 2, 8, p, p, 8, 4, p, 1e-10, -1, None) == -1
    assert h.value is None
    assert lib.nuht_fb_analysis(None, p, p, None) == -1
    assert lib.nuht_fb_synthesis(None, p, p, None) == -1
    assert lib.nuht_fb_helmholtz(None, 1.0, p, None, None, p, None) == -1
    assert lib.nuht_fb_destroy(None) == 0


def test_ctypes_structs_match_the_header(tmp_path):
    # The binding's ctypes mirrors of nuht_opts and nuht_info must have the
    # C layout: a C program compiled against include/nuht.h prints the size
    # and every field offset, which are compared with ctypes' own.
    import shutil
    import subprocess
    import paper_2411_09583_amd as nuht
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include "nuht.h"', "#include <stdio.h>", "#include <stddef.h>", "int main(void) {"]
    for cname, cls in (("nuht_opts", nuht.NuhtOpts), ("nuht_info", nuht.NuhtInfo)):
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'    printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in (("nuht_opts", nuht.NuhtOpts), ("nuht_info", nuht.NuhtInfo)):
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
