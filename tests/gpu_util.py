"""Helpers shared by the GPU parity tests: device transfer and problem setup."""
import os

import numpy as np
import pytest

import synth


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def lib():
    import paper_2602_03609_amd as vif
    vif.load()  # raises if libvif.so is not built
    return vif


def dev(a, dtype=None):
    torch = torch_cuda()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def problem_on_device(d):
    torch = torch_cuda()
    X = tuple(dev(d[k], torch.float64) for k in ("sx", "sy", "t"))
    y = dev(d["y"], torch.float64)
    Z = None
    if d.get("k", 0) > 0:
        Z = tuple(dev(d[k], torch.float64) for k in ("zx", "zy", "zt"))
    return X, y, Z


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def log(msg):
    print(msg, flush=True)
    sys_log = os.environ.get("VIF_TEST_LOG")
    if sys_log:
        with open(sys_log, "a") as f:
            f.write(msg + "\n")
