"""The C-ABI library loads and exports every symbol the public header
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hsrom.h")
LIB = os.path.join(ROOT, "paper_2301_01718_amd", "libhsrom.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:hs_status|const char\*)\s+(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("hdm_step", "sample_select", "rom_hybrid_step", "basis_update"):
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (python -m paper_2301_01718_amd.build)"
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2301_01718_amd import exported_symbols
    assert set(exported_symbols()) >= set(declared_functions())


def test_status_strings_without_gpu():
    from paper_2301_01718_amd import lib
    assert lib().hs_status_string(0) == b"ok"
    assert lib().hs_status_string(-3) == b"not converged"


def test_create_rejects_bad_arguments_without_gpu():
    from paper_2301_01718_amd import _lib as L
    p = L.Problem(kind=7, nx=4, ny=1, bc=0, dx=0.25, dy=1, dt=0.1, gamma=1.4, inflow=1,
                  m_max=4, w_max=4)
    h = ctypes.c_void_p()
    assert L.lib().hs_create(ctypes.byref(p), None, ctypes.byref(h)) == -1
    p.kind = 0
    p.m_max = 0
    assert L.lib().hs_create(ctypes.byref(p), None, ctypes.byref(h)) == -1
