"""The C ABI library loads and exports every function inrct.h declares
(no compute; runs without a GPU)."""
import ctypes
import os
import re

from paper_2604_09884_amd import lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "inrct.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\s*\*?\s*(\w+)\s*\(", src, re.M)))


def test_header_declares_the_five_named_calls():
    names = _declared()
    for n in ("inr_eval_grid", "ct_project", "ct_backproject", "inr_vjp_subsampled",
              "inr_grad_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(L.LIB_PATH):
        from paper_2604_09884_amd import build
        build.build()
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(L.EXPORTED) == sorted(_declared())


def test_errors_are_reported_without_a_gpu():
    lib = L.load()
    h = ctypes.c_void_p()
    grid = L.InrGrid(2, 0)
    a = L.InrArch(1, 2, 8, 128, 2, 30.0, 0)
    rc = lib.inrct_model_create(ctypes.byref(a), ctypes.byref(grid), 10, ctypes.byref(h))
    assert rc == -1
    assert b"grid n" in lib.inrct_last_error()


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stdout


def test_hash_arch_is_checked_before_any_device_call():
    lib = L.load()
    h = ctypes.c_void_p()
    grid = L.InrGrid(2, 16)
    # width 128 is not a hash-INR width
    a = L.InrArch(L.INRCT_HASH, 2, 0, 128, 2, 30.0, L.INRCT_FP32, 4, 10, 4, 16)
    rc = lib.inrct_model_create(ctypes.byref(a), ctypes.byref(grid), 10, ctypes.byref(h))
    assert rc != 0 and b"width" in lib.inrct_last_error()
    # BF16 is refused for the hash INR
    a = L.InrArch(L.INRCT_HASH, 2, 0, 64, 2, 30.0, L.INRCT_BF16, 4, 10, 4, 16)
    rc = lib.inrct_model_create(ctypes.byref(a), ctypes.byref(grid), 10, ctypes.byref(h))
    assert rc != 0 and b"FP32" in lib.inrct_last_error()


def test_fan_geometry_checks_on_the_host():
    lib = L.load()
    angles = (ctypes.c_double * 4)(0.0, 0.5, 1.0, 1.5)
    grid = L.InrGrid(2, 32)
    h = ctypes.c_void_p()

    def make(n_u, du, sid, idd, n_v=1):
        g = L.CtGeometry()
        g.kind, g.n_views, g.n_u, g.n_v = L.INRCT_FAN2D, 4, n_u, n_v
        g.du, g.dv, g.sid, g.idd = du, du, sid, idd
        g.angles = ctypes.cast(angles, ctypes.POINTER(ctypes.c_double))
        return lib.inrct_geom_create(ctypes.byref(g), ctypes.byref(grid), ctypes.byref(h))

    assert make(64, 0.05, 1.2, 1.0) != 0          # source inside the image
    assert b"outside" in lib.inrct_last_error()
    assert make(64, 0.05, 3.0, 1.0, n_v=2) != 0   # a fan has one detector row
    assert make(101, 1.0, 3.0, 1.0) != 0          # a fan wider than 90 degrees
    assert b"90" in lib.inrct_last_error()
