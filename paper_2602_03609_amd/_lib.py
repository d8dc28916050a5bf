"""ctypes binding of libvif.so (the C ABI in include/vif.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI. Tensors must be CUDA (HIP) tensors on one device;
PyTorch provides the device memory and the stream. There is no CPU fallback:
if the library or a GPU is missing, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libvif.so")

VIF_OK, VIF_E_ARG, VIF_E_NOT_PD, VIF_E_DEVICE, VIF_E_WORKSPACE, VIF_E_UNSUPPORTED = range(6)
VIF_KERNEL_GNEITING, VIF_KERNEL_GNEITING_MATERN, VIF_KERNEL_MATERN_ANISO = 1, 2, 3
VIF_PREC_FP64, VIF_PREC_FP32, VIF_PREC_BF16X3, VIF_PREC_BF16X6 = 0, 1, 2, 3
VIF_OP_NEIGHBORS, VIF_OP_FACTOR, VIF_OP_NLL, VIF_OP_NEIGHBORS_NLL = 0, 1, 2, 3
PREC_NAMES = {"fp64": VIF_PREC_FP64, "fp32": VIF_PREC_FP32, "bf16x3": VIF_PREC_BF16X3,
              "bf16x6": VIF_PREC_BF16X6}

EXPORTS = ("vif_workspace_bytes", "vif_neighbors", "vif_factor", "vif_nll", "vif_nll_terms",
           "vif_neighbors_nll",
           "vif_last_error", "vif_profile", "vif_profile_read",
           "vif_mlp_features", "vif_mlp_forward", "vif_mlp_backward_ws", "vif_mlp_backward",
           "vif_mlp_pair_loss", "vif_mlp_adam", "vif_mlp_batch", "vif_propose_ws",
           "vif_propose_neighbors", "vif_batch_create", "vif_batch_workspace_bytes",
           "vif_batch_enqueue", "vif_batch_graph_launch", "vif_batch_autotune",
           "vif_batch_schedule", "vif_batch_set_schedule", "vif_batch_status",
           "vif_batch_destroy", "vif_residual_ws", "vif_residual_neighbors",
           "vif_grad_params", "vif_grad_ws", "vif_nll_grad", "vif_neighbors_noalloc",
           "vif_grad_vif_ws", "vif_nll_grad_vif")
BATCH_PLAN_SCRATCH = 16384
MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_PARAMS = 8, 64, 16, 9936
STAGES = ("neighbors", "sigma_k", "crosscov", "trmm", "point_factor", "syrk", "assembly")


class VifError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"vif error {status}: {message}")
        self.status = status
        self.message = message


class Kernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32)] + [
        (f, ctypes.c_double) for f in ("sigma2", "nugget", "a", "c", "alpha", "beta", "gamma", "tau",
                                       "nu", "delta", "range_s", "range_t", "jitter")]


class Points(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sx", ctypes.c_void_p), ("sy", ctypes.c_void_p),
                ("t", ctypes.c_void_p)]


class Problem(ctypes.Structure):
    _fields_ = [("points", Points), ("y", ctypes.c_void_p), ("kern", Kernel),
                ("m", ctypes.c_int32), ("nbr", ctypes.c_void_p), ("ind", Points)]


_lib = None
_lock = threading.Lock()


def load(path=LIB_PATH):
    """Load libvif.so and declare the C signatures. Raises if it is not built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise ImportError(f"{path} is not built; run `python -m paper_2602_03609_amd.build`")
        # The library has to run on the HIP runtime that owns the device memory and the
        # streams it is given. PyTorch ships its own libamdhip64 under the system's soname:
        # mapped first, it is the one libvif.so binds to; mapped after libvif.so, it would
        # be a second runtime in the process, sharing no devices, streams or memory with
        # the library's (whose first call then finds no device).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(path)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        pP, pK = ctypes.POINTER(Points), ctypes.POINTER(Kernel)
        pd = ctypes.POINTER(ctypes.c_double)
        lib.vif_workspace_bytes.argtypes = [i64, i32, i32, i32, i32]
        lib.vif_workspace_bytes.restype = sz
        lib.vif_neighbors.argtypes = [pP, pK, i32, vp, vp, sz, vp]
        lib.vif_neighbors.restype = i32
        lib.vif_factor.argtypes = [pP, pK, i32, vp, pP, i32, vp, vp, vp, sz, vp]
        lib.vif_factor.restype = i32
        lib.vif_nll.argtypes = [pP, vp, pK, i32, vp, pP, i32, pd, vp, sz, vp]
        lib.vif_nll.restype = i32
        lib.vif_nll_terms.argtypes = [pP, vp, pK, i32, vp, pP, i32, pd, pd, vp, sz, vp]
        lib.vif_nll_terms.restype = i32
        lib.vif_neighbors_nll.argtypes = [pP, vp, pK, i32, vp, pP, i32, pd, vp, sz, vp]
        lib.vif_neighbors_nll.restype = i32
        lib.vif_last_error.argtypes = []
        lib.vif_last_error.restype = ctypes.c_char_p
        lib.vif_profile.argtypes = [i32]
        lib.vif_profile.restype = i32
        lib.vif_profile_read.argtypes = [pd, ctypes.POINTER(i32), i32]
        lib.vif_profile_read.restype = i32
        f32 = ctypes.c_float
        lib.vif_mlp_features.argtypes = [pP, pK, pd, vp, vp]
        lib.vif_mlp_features.restype = i32
        lib.vif_mlp_forward.argtypes = [vp, vp, i64, vp, vp, vp]
        lib.vif_mlp_forward.restype = i32
        lib.vif_mlp_backward_ws.argtypes = [i64]
        lib.vif_mlp_backward_ws.restype = sz
        lib.vif_mlp_backward.argtypes = [vp, vp, vp, vp, i64, vp, vp, sz, vp]
        lib.vif_mlp_backward.restype = i32
        lib.vif_mlp_pair_loss.argtypes = [vp, i64, i32, i32, f32, vp, vp, vp]
        lib.vif_mlp_pair_loss.restype = i32
        lib.vif_mlp_adam.argtypes = [vp, vp, vp, vp, i64, i32, f32, f32, f32, f32, vp]
        lib.vif_mlp_adam.restype = i32
        lib.vif_mlp_batch.argtypes = [vp, vp, i64, vp, i32, i32, i32, i32, vp, i32, vp, vp]
        lib.vif_mlp_batch.restype = i32
        lib.vif_propose_ws.argtypes = [i64]
        lib.vif_propose_ws.restype = sz
        lib.vif_propose_neighbors.argtypes = [pP, pK, i32, vp, i32, ctypes.c_double, i32, i32,
                                              i32, i32, vp, ctypes.POINTER(i64), vp, sz, vp]
        lib.vif_propose_neighbors.restype = i32
        pi32 = ctypes.POINTER(i32)
        lib.vif_batch_create.argtypes = [ctypes.POINTER(Problem), i32, i32, vp, sz, vp]
        lib.vif_batch_create.restype = vp
        lib.vif_batch_workspace_bytes.argtypes = [vp]
        lib.vif_batch_workspace_bytes.restype = sz
        lib.vif_batch_enqueue.argtypes = [vp, vp, sz, vp, vp]
        lib.vif_batch_enqueue.restype = i32
        lib.vif_batch_graph_launch.argtypes = [vp, vp, sz, vp, vp]
        lib.vif_batch_graph_launch.restype = i32
        lib.vif_batch_autotune.argtypes = [vp, vp, sz, vp, i32, pd, vp]
        lib.vif_batch_autotune.restype = i32
        lib.vif_batch_schedule.argtypes = [vp, pi32, pi32]
        lib.vif_batch_schedule.restype = i32
        lib.vif_batch_set_schedule.argtypes = [vp, i32, i32]
        lib.vif_batch_set_schedule.restype = i32
        lib.vif_batch_status.argtypes = [vp, vp, pi32, vp]
        lib.vif_batch_status.restype = i32
        lib.vif_residual_ws.argtypes = [i64, i32]
        lib.vif_residual_ws.restype = sz
        lib.vif_residual_neighbors.argtypes = [pP, pK, i32, pP, vp, vp, sz, vp]
        lib.vif_residual_neighbors.restype = i32
        lib.vif_grad_params.argtypes = [i32]
        lib.vif_grad_params.restype = i32
        lib.vif_grad_ws.argtypes = [i64]
        lib.vif_grad_ws.restype = sz
        lib.vif_nll_grad.argtypes = [pP, vp, pK, i32, vp, pd, pd, vp, sz, vp]
        lib.vif_nll_grad.restype = i32
        lib.vif_grad_vif_ws.argtypes = [i64, i32, i32]
        lib.vif_grad_vif_ws.restype = sz
        lib.vif_nll_grad_vif.argtypes = [pP, vp, pK, i32, vp, pP, pd, pd, vp, sz, vp]
        lib.vif_nll_grad_vif.restype = i32
        lib.vif_neighbors_noalloc.argtypes = [pP, pK, i32, vp, vp]
        lib.vif_neighbors_noalloc.restype = i32
        lib.vif_batch_destroy.argtypes = [vp]
        lib.vif_batch_destroy.restype = None
        _lib = lib
        return lib


def _check(st):
    if st != VIF_OK:
        msg = load().vif_last_error().decode(errors="replace")
        raise VifError(st, msg)


def make_kernel(kern):
    """vif_kernel from a dict with keys kind, sigma2, nugget, ... (missing keys = 0)."""
    k = Kernel()
    k.kind = int(kern["kind"])
    for f, _ in Kernel._fields_[1:]:
        setattr(k, f, float(kern.get(f, 0.0)))
    return k


def _torch():
    import torch
    return torch


def _dev_ptr(x, dtype, name):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if x.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {x.dtype}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return x.data_ptr()


def make_points(sx, sy, t, name="points"):
    torch = _torch()
    n = sx.shape[0]
    if sy.shape[0] != n or t.shape[0] != n:
        raise ValueError(f"{name}: sx, sy, t must have the same length")
    p = Points()
    p.n = n
    p.sx = _dev_ptr(sx, torch.float64, name + ".sx")
    p.sy = _dev_ptr(sy, torch.float64, name + ".sy")
    p.t = _dev_ptr(t, torch.float64, name + ".t")
    return p


_ws_cache = {}


def workspace(n, m, k, prec, op, device):
    """Cached caller-owned workspace (a uint8 CUDA tensor) for one operation shape."""
    torch = _torch()
    nbytes = vif_workspace_bytes(n, m, k, prec, op)
    if nbytes == 0:
        raise VifError(VIF_E_ARG, "invalid workspace request")
    key = (str(device), op, prec)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        _ws_cache.pop(key, None)
        buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def release_workspaces():
    _ws_cache.clear()


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _prec(prec):
    return PREC_NAMES[prec] if isinstance(prec, str) else int(prec)


def vif_workspace_bytes(n, m, k, prec, op):
    return int(load().vif_workspace_bytes(int(n), int(m), int(k), _prec(prec), int(op)))


def vif_neighbors(sx, sy, t, kern, m, nbr=None, stream=None):
    """Exact correlation-based neighbors; returns int32 [n, m] (-1 padded)."""
    torch = _torch()
    lib = load()
    n = sx.shape[0]
    if nbr is None:
        nbr = torch.empty((n, m), dtype=torch.int32, device=sx.device)
    p = make_points(sx, sy, t)
    K = make_kernel(kern)
    ws = workspace(n, m, 0, 0, VIF_OP_NEIGHBORS, sx.device)
    _check(lib.vif_neighbors(ctypes.byref(p), ctypes.byref(K), int(m),
                             _dev_ptr(nbr, torch.int32, "nbr") if m > 0 else None,
                             ws.data_ptr(), ws.numel(), _stream(stream)))
    return nbr


def vif_neighbors_noalloc(sx, sy, t, kern, m, nbr, stream=None):
    """vif_neighbors with the library's static device scratch as workspace (no
    allocation inside the call); nbr: int32 [n, m] CUDA tensor, written."""
    torch = _torch()
    lib = load()
    p = make_points(sx, sy, t)
    K = make_kernel(kern)
    _check(lib.vif_neighbors_noalloc(ctypes.byref(p), ctypes.byref(K), int(m),
                                     _dev_ptr(nbr, torch.int32, "nbr") if m > 0 else None,
                                     _stream(stream)))
    return nbr


def _ind(ind):
    if ind is None:
        return None, 0
    zx, zy, zt = ind
    return make_points(zx, zy, zt, "ind"), int(zx.shape[0])


def vif_factor(sx, sy, t, kern, m, nbr, ind=None, prec="fp64", stream=None):
    """Per-point factor; returns (B [n, m] = -A_i, D [n]) as float64 tensors."""
    torch = _torch()
    lib = load()
    n = sx.shape[0]
    p = make_points(sx, sy, t)
    K = make_kernel(kern)
    ip, k = _ind(ind)
    B = torch.empty((n, m), dtype=torch.float64, device=sx.device)
    D = torch.empty(n, dtype=torch.float64, device=sx.device)
    ws = workspace(n, m, k, _prec(prec), VIF_OP_FACTOR, sx.device)
    _check(lib.vif_factor(ctypes.byref(p), ctypes.byref(K), int(m),
                          _dev_ptr(nbr, torch.int32, "nbr") if m > 0 else None,
                          ctypes.byref(ip) if ip is not None else None, _prec(prec),
                          B.data_ptr() if m > 0 else None, D.data_ptr(), ws.data_ptr(), ws.numel(),
                          _stream(stream)))
    return B, D


def vif_nll_terms(sx, sy, t, y, kern, m, nbr, ind=None, prec="fp64", stream=None):
    """(nll, [sum log D, z'z, log det M, q'M^-1 q])."""
    torch = _torch()
    lib = load()
    n = sx.shape[0]
    p = make_points(sx, sy, t)
    K = make_kernel(kern)
    ip, k = _ind(ind)
    ws = workspace(n, m, k, _prec(prec), VIF_OP_NLL, sx.device)
    out = ctypes.c_double(0.0)
    terms = (ctypes.c_double * 4)()
    _check(lib.vif_nll_terms(ctypes.byref(p), _dev_ptr(y, torch.float64, "y"), ctypes.byref(K),
                             int(m), _dev_ptr(nbr, torch.int32, "nbr") if m > 0 else None,
                             ctypes.byref(ip) if ip is not None else None, _prec(prec),
                             ctypes.byref(out), terms, ws.data_ptr(), ws.numel(), _stream(stream)))
    return out.value, list(terms)


def vif_nll(sx, sy, t, y, kern, m, nbr, ind=None, prec="fp64", stream=None):
    """Negative log-likelihood (float)."""
    torch = _torch()
    lib = load()
    n = sx.shape[0]
    p = make_points(sx, sy, t)
    K = make_kernel(kern)
    ip, k = _ind(ind)
    ws = workspace(n, m, k, _prec(prec), VIF_OP_NLL, sx.device)
    out = ctypes.c_double(0.0)
    _check(lib.vif_nll(ctypes.byref(p), _dev_ptr(y, torch.float64, "y"), ctypes.byref(K), int(m),
                       _dev_ptr(nbr, torch.int32, "nbr") if m > 0 else None,
                       ctypes.byref(ip) if ip is not None else None, _prec(prec),
                       ctypes.byref(out), ws.data_ptr(), ws.numel(), _stream(stream)))
    return out.value


def vif_neighbors_nll(sx, sy, t, y, kern, m, nbr=None, ind=None, prec="fp64", stream=None):
    """Neighbor search and NLL in one call (the search overlaps the low-rank
    stages); returns (nll, nbr int32 [n, m])."""
    torch = _torch()
    lib = load()
    n = sx.shape[0]
    if nbr is None:
        nbr = torch.empty((n, m), dtype=torch.int32, device=sx.device)
    p = make_points(sx, sy, t)
    K = make_kernel(kern)
    ip, k = _ind(ind)
    ws = workspace(n, m, k, _prec(prec), VIF_OP_NEIGHBORS_NLL, sx.device)
    out = ctypes.c_double(0.0)
    _check(lib.vif_neighbors_nll(ctypes.byref(p), _dev_ptr(y, torch.float64, "y"), ctypes.byref(K),
                                 int(m), _dev_ptr(nbr, torch.int32, "nbr") if m > 0 else None,
                                 ctypes.byref(ip) if ip is not None else None, _prec(prec),
                                 ctypes.byref(out), ws.data_ptr(), ws.numel(), _stream(stream)))
    return out.value, nbr


def vif_profile(enable):
    """Turn the library's stage timing on or off (both reset the totals)."""
    _check(load().vif_profile(1 if enable else 0))


def vif_profile_read():
    """{stage: (total_ms, calls)} accumulated since the last vif_profile()."""
    n = len(STAGES)
    ms = (ctypes.c_double * n)()
    calls = (ctypes.c_int32 * n)()
    _check(load().vif_profile_read(ms, calls, n))
    return {STAGES[i]: (ms[i], calls[i]) for i in range(n)}


# ---------------------------------------------------------------- NLL gradient ----
GRAD_PARAMS = {VIF_KERNEL_GNEITING: ("sigma2", "nugget", "a", "c", "alpha", "beta", "gamma", "tau"),
               VIF_KERNEL_GNEITING_MATERN: ("sigma2", "nugget", "a", "c", "alpha", "gamma", "delta"),
               VIF_KERNEL_MATERN_ANISO: ("sigma2", "nugget", "range_s", "range_t")}


def vif_nll_grad(sx, sy, t, y, kern, m, nbr, stream=None):
    """(NLL, gradient list) of the plain Vecchia NLL (include/vif_grad.h); the
    gradient follows GRAD_PARAMS[kern["kind"]]."""
    torch = _torch()
    lib = load()
    n = sx.shape[0]
    p = make_points(sx, sy, t)
    K = make_kernel(kern)
    P = int(lib.vif_grad_params(int(kern["kind"])))
    nbytes = int(lib.vif_grad_ws(int(n)))
    if nbytes == 0:
        raise VifError(VIF_E_ARG, "invalid sizes")
    ws = _scratch(("grad", str(sx.device)), nbytes, sx.device)
    out = ctypes.c_double(0.0)
    g = (ctypes.c_double * 8)()
    _check(lib.vif_nll_grad(ctypes.byref(p), _dev_ptr(y, torch.float64, "y"), ctypes.byref(K),
                            int(m), _dev_ptr(nbr, torch.int32, "nbr") if m > 0 else None,
                            ctypes.byref(out), g, ws.data_ptr(), ws.numel(), _stream(stream)))
    return out.value, [g[q] for q in range(P)]


# ---------------------------------------------------------- residual neighbors ----
def vif_nll_grad_vif(sx, sy, t, y, kern, m, nbr, ind, stream=None):
    """(NLL, gradient as a numpy array) of the VIF NLL in FP64; ind = (zx, zy, zt)."""
    import numpy as np
    torch = _torch()
    lib = load()
    n = sx.shape[0]
    p = make_points(sx, sy, t)
    K = make_kernel(kern)
    ip, k = _ind(ind)
    P = int(lib.vif_grad_params(int(kern["kind"])))
    nbytes = int(lib.vif_grad_vif_ws(int(n), int(m), int(k)))
    if nbytes == 0:
        raise VifError(VIF_E_ARG, "invalid workspace request")
    ws = _scratch(("grad_vif", str(sx.device)), nbytes, sx.device)
    nll = ctypes.c_double()
    g = (ctypes.c_double * max(P, 1))()
    _check(lib.vif_nll_grad_vif(ctypes.byref(p), _dev_ptr(y, torch.float64, "y"), ctypes.byref(K),
                                int(m), _dev_ptr(nbr, torch.int32, "nbr") if m > 0 else None,
                                ctypes.byref(ip) if ip is not None else None, ctypes.byref(nll), g,
                                ws.data_ptr(), ws.numel(), _stream(stream)))
    return nll.value, np.array([g[i] for i in range(P)])


def vif_residual_neighbors(sx, sy, t, kern, m, ind=None, nbr=None, stream=None):
    """Residual-correlation neighbors for VIF (include/vif_residual.h); int32 [n, m]."""
    torch = _torch()
    lib = load()
    n = sx.shape[0]
    if nbr is None:
        nbr = torch.empty((n, m), dtype=torch.int32, device=sx.device)
    p = make_points(sx, sy, t)
    K = make_kernel(kern)
    ip, k = _ind(ind)
    nbytes = int(lib.vif_residual_ws(int(n), int(k)))
    if nbytes == 0:
        raise VifError(VIF_E_ARG, "invalid sizes")
    ws = _scratch(("resid", str(sx.device)), nbytes, sx.device)
    _check(lib.vif_residual_neighbors(ctypes.byref(p), ctypes.byref(K), int(m),
                                      ctypes.byref(ip) if ip is not None else None,
                                      _dev_ptr(nbr, torch.int32, "nbr"), ws.data_ptr(), ws.numel(),
                                      _stream(stream)))
    return nbr


# ------------------------------------------------------------ learned proposal ----
def _scratch(key, nbytes, device):
    torch = _torch()
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        _ws_cache.pop(key, None)
        buf = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def vif_mlp_features(sx, sy, t, kern, centre, stream=None):
    """Network inputs [n, 8] (float32) for the points under kernel `kern`."""
    torch = _torch()
    lib = load()
    n = sx.shape[0]
    X = torch.empty((n, MLP_IN), dtype=torch.float32, device=sx.device)
    c = (ctypes.c_double * 10)(*[float(v) for v in centre])
    p = make_points(sx, sy, t)
    K = make_kernel(kern)
    _check(lib.vif_mlp_features(ctypes.byref(p), ctypes.byref(K), c, X.data_ptr(),
                                _stream(stream)))
    return X


def vif_mlp_forward(params, X, want_hidden=False, stream=None):
    """(E [rows, 16], H [rows, 3, 64] or None)."""
    torch = _torch()
    lib = load()
    rows = X.shape[0]
    E = torch.empty((rows, MLP_OUT), dtype=torch.float32, device=X.device)
    H = (torch.empty((rows, 3, MLP_HIDDEN), dtype=torch.float32, device=X.device)
         if want_hidden else None)
    _check(lib.vif_mlp_forward(_dev_ptr(params, torch.float32, "params"),
                               _dev_ptr(X, torch.float32, "X"), int(rows), E.data_ptr(),
                               H.data_ptr() if H is not None else None, _stream(stream)))
    return E, H


def vif_mlp_backward(params, X, H, dE, stream=None):
    """Gradient [9936] of sum(dE * E) with respect to the parameters."""
    torch = _torch()
    lib = load()
    rows = X.shape[0]
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device)
    nb = int(lib.vif_mlp_backward_ws(int(rows)))
    ws = _scratch(("mlp_bwd", str(X.device)), nb, X.device)
    _check(lib.vif_mlp_backward(_dev_ptr(params, torch.float32, "params"),
                                _dev_ptr(X, torch.float32, "X"), _dev_ptr(H, torch.float32, "H"),
                                _dev_ptr(dE, torch.float32, "dE"), int(rows), grad.data_ptr(),
                                ws.data_ptr(), ws.numel(), _stream(stream)))
    return grad


def vif_mlp_pair_loss(E, npos, nneg, tau, stream=None):
    """(loss [groups], dE [rows, 16]) for groups of 1 + npos + nneg rows."""
    torch = _torch()
    lib = load()
    G = 1 + npos + nneg
    groups = E.shape[0] // G
    loss = torch.empty(groups, dtype=torch.float32, device=E.device)
    dE = torch.zeros_like(E)
    _check(lib.vif_mlp_pair_loss(_dev_ptr(E, torch.float32, "E"), int(groups), int(npos),
                                 int(nneg), float(tau), dE.data_ptr(), loss.data_ptr(),
                                 _stream(stream)))
    return loss, dE


def vif_mlp_adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """One in-place Adam step (step counts from 1)."""
    torch = _torch()
    lib = load()
    _check(lib.vif_mlp_adam(_dev_ptr(params, torch.float32, "params"),
                            _dev_ptr(grad, torch.float32, "grad"), _dev_ptr(m, torch.float32, "m"),
                            _dev_ptr(v, torch.float32, "v"), int(params.numel()), int(step),
                            float(lr), float(beta1), float(beta2), float(eps), _stream(stream)))


def vif_mlp_batch(X, queries, nbr_ext, npos, nhard, nrand, rnd, rand_window, stream=None):
    """Training rows [nq * (1 + npos + nhard + nrand), 8]."""
    torch = _torch()
    lib = load()
    nq = queries.shape[0]
    G = 1 + npos + nhard + nrand
    Xb = torch.empty((nq * G, MLP_IN), dtype=torch.float32, device=X.device)
    _check(lib.vif_mlp_batch(_dev_ptr(X, torch.float32, "X"),
                             _dev_ptr(queries, torch.int32, "queries"), int(nq),
                             _dev_ptr(nbr_ext, torch.int32, "nbr_ext"), int(nbr_ext.shape[1]),
                             int(npos), int(nhard), int(nrand),
                             _dev_ptr(rnd, torch.int32, "rnd") if nrand > 0 else None,
                             int(rand_window), Xb.data_ptr(), _stream(stream)))
    return Xb


def vif_propose_neighbors(sx, sy, t, kern, m, E, ncand, cell, lags, cmax=1024, nbr=None,
                          stream=None, wmin=0, rmax=1):
    """Proposal search (embedding or, with E=None, spatial candidates + exact rerank).
    Returns (nbr int32 [n, m], number of rows that took the exact search)."""
    torch = _torch()
    lib = load()
    n = sx.shape[0]
    if nbr is None:
        nbr = torch.empty((n, m), dtype=torch.int32, device=sx.device)
    p = make_points(sx, sy, t)
    K = make_kernel(kern)
    ws = _scratch(("propose", str(sx.device)), int(lib.vif_propose_ws(int(n))), sx.device)
    nfb = ctypes.c_int64(0)
    _check(lib.vif_propose_neighbors(ctypes.byref(p), ctypes.byref(K), int(m),
                                     _dev_ptr(E, torch.float32, "E") if E is not None else None,
                                     int(ncand), float(cell), int(lags), int(wmin), int(rmax),
                                     int(cmax),
                                     _dev_ptr(nbr, torch.int32, "nbr") if m > 0 else None,
                                     ctypes.byref(nfb), ws.data_ptr(), ws.numel(),
                                     _stream(stream)))
    return nbr, int(nfb.value)


# --------------------------------------------------------------------- batches ----
class Batch:
    """Many NLL evaluations planned once and enqueued together (include/vif_batch.h).

    problems: sequence of dicts with device tensors sx, sy, t, y, nbr (int32
    [n, m]), optional ind = (zx, zy, zt), and a kernel dict `kern`. The tensors
    are kept referenced for the batch's lifetime. Results land in `self.nll`
    (float64 CUDA tensor [count]).
    """

    def __init__(self, problems, prec="fp32", stream=None):
        torch = _torch()
        lib = load()
        self._keep = []
        arr = (Problem * len(problems))()
        for i, d in enumerate(problems):
            pr = arr[i]
            pr.points = make_points(d["sx"], d["sy"], d["t"])
            pr.y = _dev_ptr(d["y"], torch.float64, "y")
            pr.kern = make_kernel(d["kern"])
            m = int(d["nbr"].shape[1]) if d.get("nbr") is not None else 0
            pr.m = m
            pr.nbr = _dev_ptr(d["nbr"], torch.int32, "nbr") if m > 0 else None
            ind = d.get("ind")
            if ind is not None:
                pr.ind = make_points(*ind, name="ind")
            self._keep.append(d)
        dev = problems[0]["sx"].device
        scratch = torch.empty(BATCH_PLAN_SCRATCH, dtype=torch.uint8, device=dev)
        h = lib.vif_batch_create(arr, len(problems), _prec(prec), scratch.data_ptr(),
                                 scratch.numel(), _stream(stream))
        if not h:
            raise VifError(VIF_E_ARG, lib.vif_last_error().decode(errors="replace"))
        self._h = ctypes.c_void_p(h)
        self.count = len(problems)
        self.ws = torch.empty(int(lib.vif_batch_workspace_bytes(self._h)), dtype=torch.uint8,
                              device=dev)
        self.nll = torch.zeros(self.count, dtype=torch.float64, device=dev)

    def _args(self):
        return self._h, self.ws.data_ptr(), self.ws.numel(), self.nll.data_ptr()

    def enqueue(self, stream=None):
        _check(load().vif_batch_enqueue(*self._args(), _stream(stream)))
        return self.nll

    def graph_launch(self, stream=None):
        _check(load().vif_batch_graph_launch(*self._args(), _stream(stream)))
        return self.nll

    def autotune(self, reps=3, stream=None):
        best = ctypes.c_double(0.0)
        _check(load().vif_batch_autotune(*self._args(), int(reps), ctypes.byref(best),
                                         _stream(stream)))
        return best.value

    def schedule(self):
        a, b = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(load().vif_batch_schedule(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_schedule(self, streams, chunk_rows):
        _check(load().vif_batch_set_schedule(self._h, int(streams), int(chunk_rows)))

    def status(self, stream=None):
        """Per-problem status list (VIF_OK or VIF_E_*) of the last evaluation."""
        st = (ctypes.c_int32 * self.count)()
        load().vif_batch_status(self._h, self.ws.data_ptr(), st, _stream(stream))
        return list(st)

    def close(self):
        if getattr(self, "_h", None):
            load().vif_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
