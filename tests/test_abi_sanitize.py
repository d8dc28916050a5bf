"""The host code of the C ABI (argument validation, workspace layout, the
neighbor search's host tables) built with AddressSanitizer and
UndefinedBehaviorSanitizer and exercised by tests/native/abi_sanitize.cpp on a
machine without a GPU: the instrumented api.cpp is linked ahead of libvif.so,
whose kernels and launchers it calls (none is reached: every call is refused by
the host-side checks). Skipped where a GPU is present or hipcc is missing."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2602_03609_amd")
HIPCC = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


@pytest.mark.skipif(HIPCC is None, reason="hipcc not found")
def test_host_abi_under_asan_and_ubsan(tmp_path):
    if not os.path.exists(os.path.join(PKG, "libvif.so")):
        pytest.skip("libvif.so is not built")
    # host code only (no device pass), each sanitizer flag for the host side
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-host-only", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]
    api_o, drv_o, exe = (str(tmp_path / f) for f in ("api.o", "drv.o", "abi_sanitize"))
    _run([HIPCC, *flags, "-c", os.path.join(PKG, "csrc", "api.cpp"), "-o", api_o])
    _run([HIPCC, *flags, "-c", os.path.join(ROOT, "tests", "native", "abi_sanitize.cpp"), "-o", drv_o])
    _run([HIPCC, "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          drv_o, api_o, "-L", PKG, "-lvif", f"-Wl,-rpath,{PKG}", "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    if r.returncode == 77:
        pytest.skip(r.stdout.strip())
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
