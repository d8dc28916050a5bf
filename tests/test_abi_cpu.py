"""CPU-side checks of the C ABI: the library loads and exports every function
that include/vif.h declares, and the workspace query behaves (no GPU work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vif.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(vif_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_expected_api():
    fns = declared_functions()
    for f in ("vif_workspace_bytes", "vif_neighbors", "vif_factor", "vif_nll", "vif_nll_terms",
              "vif_last_error"):
        assert f in fns


def test_library_exports_every_declared_symbol():
    import paper_2602_03609_amd as vif
    lib = vif.load()
    for f in declared_functions():
        assert hasattr(lib, f), f


def test_workspace_bytes():
    import paper_2602_03609_amd as vif
    assert vif.vif_workspace_bytes(0, 10, 0, 0, 2) == 0
    assert vif.vif_workspace_bytes(100, 64, 0, 0, 2) == 0          # m above VIF_MAX_M
    assert vif.vif_workspace_bytes(100, 10, 5000, 0, 2) == 0       # k above VIF_MAX_K
    a = vif.vif_workspace_bytes(1000, 10, 100, 0, 2)
    b = vif.vif_workspace_bytes(1000, 10, 100, 2, 2)
    assert a > b > 0                                               # FP32 U and W are half size
    assert vif.vif_workspace_bytes(1000, 10, 0, 0, 0) > 0


def test_argument_errors_before_any_launch():
    """Host-side validation returns VIF_E_ARG without touching device pointers."""
    import paper_2602_03609_amd._lib as L
    lib = L.load()
    K = L.make_kernel({"kind": 1, "sigma2": 1.0, "nugget": 0.1, "a": 0.5, "c": 20.0, "alpha": 0.75,
                       "beta": 0.5, "gamma": 0.5, "tau": 1.0})
    P = L.Points()
    P.n = 10
    P.sx = P.sy = P.t = ctypes.c_void_p(0x1000)
    # NULL workspace
    st = lib.vif_neighbors(ctypes.byref(P), ctypes.byref(K), 5, ctypes.c_void_p(0x1000), None, 0, None)
    assert st == L.VIF_E_ARG
    # bad hyperparameter
    K.alpha = 1.5
    st = lib.vif_neighbors(ctypes.byref(P), ctypes.byref(K), 5, ctypes.c_void_p(0x1000),
                           ctypes.c_void_p(0x100000), 1 << 30, None)
    assert st == L.VIF_E_ARG and b"alpha" in lib.vif_last_error()
    K.alpha = 0.75
    # m too large
    st = lib.vif_neighbors(ctypes.byref(P), ctypes.byref(K), 64, ctypes.c_void_p(0x1000),
                           ctypes.c_void_p(0x100000), 1 << 30, None)
    assert st == L.VIF_E_UNSUPPORTED
    # workspace too small
    st = lib.vif_neighbors(ctypes.byref(P), ctypes.byref(K), 5, ctypes.c_void_p(0x1000),
                           ctypes.c_void_p(0x100000), 16, None)
    assert st == L.VIF_E_WORKSPACE
    # unknown kernel kind
    K.kind = 9
    st = lib.vif_nll(ctypes.byref(P), ctypes.c_void_p(0x1000), ctypes.byref(K), 5,
                     ctypes.c_void_p(0x1000), None, 0, ctypes.byref(ctypes.c_double()),
                     ctypes.c_void_p(0x100000), 1 << 30, None)
    assert st == L.VIF_E_ARG
    # nu outside the closed forms
    K.kind = 2
    K.nu = 1.0
    st = lib.vif_nll(ctypes.byref(P), ctypes.c_void_p(0x1000), ctypes.byref(K), 5,
                     ctypes.c_void_p(0x1000), None, 0, ctypes.byref(ctypes.c_double()),
                     ctypes.c_void_p(0x100000), 1 << 30, None)
    assert st == L.VIF_E_UNSUPPORTED
