"""CPU-side checks of the C ABI: the library loads and exports every function
that the headers in include/ declare, and the workspace query behaves (no GPU
work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    fns = set()
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        fns |= set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(vif_\w+)\s*\(", src, flags=re.M))
    return sorted(fns)


def test_header_declares_expected_api():
    fns = declared_functions()
    for f in ("vif_workspace_bytes", "vif_neighbors", "vif_factor", "vif_nll", "vif_nll_terms",
              "vif_last_error", "vif_mlp_forward", "vif_mlp_backward", "vif_mlp_pair_loss",
              "vif_mlp_adam", "vif_mlp_batch", "vif_mlp_features", "vif_propose_neighbors"):
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


def test_neighbors_nll_argument_errors():
    """The combined search + NLL entry point: workspace is the search's (256-byte
    aligned) followed by the NLL's; host-side validation precedes any launch."""
    import paper_2602_03609_amd._lib as L
    lib = L.load()
    n, m, k = 5000, 30, 200
    for prec in (0, 2, 3):
        a = L.vif_workspace_bytes(n, m, 0, 0, L.VIF_OP_NEIGHBORS)
        b = L.vif_workspace_bytes(n, m, k, prec, L.VIF_OP_NLL)
        assert L.vif_workspace_bytes(n, m, k, prec, L.VIF_OP_NEIGHBORS_NLL) == ((a + 255) // 256) * 256 + b
    assert lib.vif_workspace_bytes(n, m, k, 0, 4) == 0
    K = L.make_kernel({"kind": 1, "sigma2": 1.0, "nugget": 0.1, "a": 0.5, "c": 20.0, "alpha": 0.75,
                       "beta": 0.5, "gamma": 0.5, "tau": 1.0})
    P = L.Points()
    P.n = n
    P.sx = P.sy = P.t = ctypes.c_void_p(0x1000)
    Z = L.Points()
    Z.n = k
    Z.sx = Z.sy = Z.t = ctypes.c_void_p(0x2000)
    dev, big = ctypes.c_void_p(0x1000), 1 << 40
    out = ctypes.c_double()
    need = L.vif_workspace_bytes(n, m, k, 2, L.VIF_OP_NEIGHBORS_NLL)

    def call(y=dev, nbr=dev, prec=2, res=ctypes.byref(out), ws_bytes=big):
        return lib.vif_neighbors_nll(ctypes.byref(P), y, ctypes.byref(K), m, nbr, ctypes.byref(Z), prec,
                                     res, ctypes.c_void_p(0x100000), ws_bytes, None)

    assert call(ws_bytes=need - 1) == L.VIF_E_WORKSPACE
    assert call(y=None) == L.VIF_E_ARG and b"y is NULL" in lib.vif_last_error()
    assert call(nbr=None) == L.VIF_E_ARG and b"nbr is NULL" in lib.vif_last_error()
    assert call(res=None) == L.VIF_E_ARG and b"nll is NULL" in lib.vif_last_error()
    assert call(prec=7) == L.VIF_E_ARG and b"precision" in lib.vif_last_error()


def test_learned_proposal_argument_errors():
    import paper_2602_03609_amd._lib as L
    lib = L.load()
    assert lib.vif_mlp_pair_loss(None, 4, 0, 3, 1.0, None, None, None) == L.VIF_E_ARG
    assert lib.vif_mlp_pair_loss(None, 4, 100, 30, 1.0, None, None, None) == L.VIF_E_ARG
    assert lib.vif_mlp_adam(None, None, None, None, 10, 0, 1e-3, 0.9, 0.999, 1e-8, None) == L.VIF_E_ARG
    assert lib.vif_mlp_forward(None, None, 5, None, None, None) == L.VIF_E_ARG
    assert lib.vif_mlp_backward_ws(1000) >= 16 * 9936 * 4
    assert lib.vif_propose_ws(0) == 0 and lib.vif_propose_ws(1000) > 0
    K = L.make_kernel({"kind": 1, "sigma2": 1.0, "nugget": 0.1, "a": 0.5, "c": 20.0, "alpha": 0.75,
                       "beta": 0.5, "gamma": 0.5, "tau": 1.0})
    P = L.Points()
    P.n = 10
    P.sx = P.sy = P.t = ctypes.c_void_p(0x1000)
    nfb = ctypes.c_int64(0)
    # ncand above 128 and a NULL workspace are host-side errors
    st = lib.vif_propose_neighbors(ctypes.byref(P), ctypes.byref(K), 5, None, 200, 1.0, 1, 0, 1,
                                   64, ctypes.c_void_p(0x1000), ctypes.byref(nfb), None, 0, None)
    assert st == L.VIF_E_ARG
    centre = (ctypes.c_double * 10)(*([0.0] * 10))
    st = lib.vif_mlp_features(ctypes.byref(P), ctypes.byref(K), centre, ctypes.c_void_p(0x1000), None)
    assert st == L.VIF_E_ARG and b"scale" in lib.vif_last_error()


def test_batch_argument_errors():
    """Batch planning rejects bad arguments before any device call."""
    import paper_2602_03609_amd._lib as L
    lib = L.load()
    assert lib.vif_batch_create(None, 1, 0, ctypes.c_void_p(0x1000), 16384, None) is None
    assert b"at least one problem" in lib.vif_last_error()
    probs = (L.Problem * 1)()
    assert lib.vif_batch_create(probs, 1, 7, ctypes.c_void_p(0x1000), 16384, None) is None
    assert b"precision" in lib.vif_last_error()
    assert lib.vif_batch_create(probs, 1, 1, ctypes.c_void_p(0x1000), 100, None) is None
    assert b"scratch" in lib.vif_last_error()
    assert lib.vif_batch_create(probs, 1, 1, ctypes.c_void_p(0x1001), 16384, None) is None
    assert b"aligned" in lib.vif_last_error()
    probs[0].points.n = 10
    probs[0].points.sx = probs[0].points.sy = probs[0].points.t = 0x1000
    probs[0].y = 0x1000
    probs[0].kern = L.make_kernel({"kind": 1, "sigma2": 1.0, "nugget": 0.1, "a": 0.5, "c": 20.0,
                                   "alpha": 0.75, "beta": 0.5, "gamma": 0.5, "tau": 1.0})
    probs[0].m = 70
    probs[0].nbr = 0x1000
    assert lib.vif_batch_create(probs, 1, 1, ctypes.c_void_p(0x1000), 16384, None) is None
    assert b"VIF_MAX_M" in lib.vif_last_error()
    probs[0].m = 5
    probs[0].nbr = None
    assert lib.vif_batch_create(probs, 1, 1, ctypes.c_void_p(0x1000), 16384, None) is None
    assert b"nbr is NULL" in lib.vif_last_error()
    assert lib.vif_batch_workspace_bytes(None) == 0
    assert lib.vif_batch_enqueue(None, None, 0, None, None) == L.VIF_E_ARG
    assert lib.vif_batch_set_schedule(None, 1, 4096) == L.VIF_E_ARG
    lib.vif_batch_destroy(None)


def test_residual_argument_errors():
    import paper_2602_03609_amd._lib as L
    lib = L.load()
    assert lib.vif_residual_ws(0, 10) == 0
    assert lib.vif_residual_ws(100, 5000) == 0
    assert lib.vif_residual_ws(1000, 50) > lib.vif_residual_ws(1000, 0) > 0
    K = L.make_kernel({"kind": 1, "sigma2": 1.0, "nugget": 0.1, "a": 0.5, "c": 20.0, "alpha": 0.75,
                       "beta": 0.5, "gamma": 0.5, "tau": 1.0})
    P = L.Points()
    P.n = 10
    P.sx = P.sy = P.t = ctypes.c_void_p(0x1000)
    big = lib.vif_residual_ws(10, 0)
    st = lib.vif_residual_neighbors(ctypes.byref(P), ctypes.byref(K), 0, None,
                                    ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), big, None)
    assert st == L.VIF_E_ARG and b"m must be" in lib.vif_last_error()
    st = lib.vif_residual_neighbors(ctypes.byref(P), ctypes.byref(K), 5, None, None,
                                    ctypes.c_void_p(0x1000), big, None)
    assert st == L.VIF_E_ARG and b"nbr" in lib.vif_last_error()
    st = lib.vif_residual_neighbors(ctypes.byref(P), ctypes.byref(K), 5, None,
                                    ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), 16, None)
    assert st == L.VIF_E_WORKSPACE


def test_gradient_argument_errors():
    import paper_2602_03609_amd._lib as L
    lib = L.load()
    assert lib.vif_grad_params(1) == 8 and lib.vif_grad_params(2) == 7
    assert lib.vif_grad_params(3) == 4 and lib.vif_grad_params(9) == 0
    assert lib.vif_grad_ws(0) == 0 and lib.vif_grad_ws(1000) > 0
    K = L.make_kernel({"kind": 2, "sigma2": 1.0, "nugget": 0.1, "a": 0.5, "c": 20.0, "alpha": 0.4,
                       "gamma": 0.4, "delta": 0.2, "nu": 1.0})
    P = L.Points()
    P.n = 10
    P.sx = P.sy = P.t = ctypes.c_void_p(0x1000)
    out = ctypes.c_double()
    g = (ctypes.c_double * 8)()

    def call(y=ctypes.c_void_p(0x1000)):
        return lib.vif_nll_grad(ctypes.byref(P), y, ctypes.byref(K), 5, ctypes.c_void_p(0x1000),
                                ctypes.byref(out), g, ctypes.c_void_p(0x1000), lib.vif_grad_ws(10), None)

    assert call() == L.VIF_E_UNSUPPORTED          # nu without a closed form
    K.nu = 1.5
    assert call(y=None) == L.VIF_E_ARG


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr


def test_noalloc_neighbors_rejects_sizes_beyond_its_scratch():
    """vif_neighbors_noalloc refuses, before any launch, an n whose search
    workspace exceeds its static device scratch."""
    import paper_2602_03609_amd._lib as L
    lib = L.load()
    K = L.make_kernel({"kind": 1, "sigma2": 1.0, "nugget": 0.1, "a": 0.5, "c": 20.0, "alpha": 0.75,
                       "beta": 0.5, "gamma": 0.5, "tau": 1.0})
    P = L.Points()
    P.n = 50_000_000
    P.sx = P.sy = P.t = ctypes.c_void_p(0x1000)
    st = lib.vif_neighbors_noalloc(ctypes.byref(P), ctypes.byref(K), 10, ctypes.c_void_p(0x1000), None)
    assert st == L.VIF_E_WORKSPACE and b"static scratch" in lib.vif_last_error()
    st = lib.vif_neighbors_noalloc(None, ctypes.byref(K), 10, ctypes.c_void_p(0x1000), None)
    assert st == L.VIF_E_ARG
    P.n = 100
    st = lib.vif_neighbors_noalloc(ctypes.byref(P), ctypes.byref(K), 64, ctypes.c_void_p(0x1000), None)
    assert st == L.VIF_E_UNSUPPORTED


def test_library_binds_to_the_callers_hip_runtime():
    """Loading the package before torch still leaves one HIP runtime in the
    process, torch's: PyTorch ships its libamdhip64 under the system's soname, so
    whichever is mapped first is the one libvif.so uses, and a second runtime
    mapped later shares no devices or streams with the first."""
    import subprocess
    import sys
    code = ("import paper_2602_03609_amd as v\n"
            "v.load()\n"
            "import torch, os\n"
            "libs = sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l})\n"
            "tdir = os.path.realpath(os.path.join(os.path.dirname(torch.__file__), 'lib'))\n"
            "print(len(libs), all(os.path.realpath(p).startswith(tdir) for p in libs))\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                       cwd=ROOT)
    assert r.returncode == 0, r.stderr
    assert r.stdout.split() == ["1", "True"], r.stdout
