"""The host side of the C ABI under AddressSanitizer (CPU only).

Builds liblbm.so with the host code instrumented (the device code is built
as usual), links a small C driver (asan_driver.c) against it, and runs every
entry point that must answer without a GPU: size queries, the velocity set,
status strings and the argument checks that reject a call before any device
work.  Any heap, stack or global-buffer error in that host code aborts the
driver with an AddressSanitizer report.
"""

import glob
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="HIP toolchain not installed")
def test_host_abi_under_address_sanitizer(tmp_path):
    from paper_1601_01237_amd import build
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("clang AddressSanitizer runtime not found")
    lib = build.build(out=str(tmp_path / "liblbm.so"), objdir=str(tmp_path / "obj"), host_asan=True)
    clang = "/opt/rocm/llvm/bin/clang"
    exe = str(tmp_path / "asan_driver")
    cmd = [clang, "-fsanitize=address", "-shared-libasan", "-fno-omit-frame-pointer", "-g",
           "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "asan_driver.c"),
           "-L", str(tmp_path), "-llbm", f"-Wl,-rpath,{tmp_path}", f"-Wl,-rpath,{os.path.dirname(rt)}",
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "all host-side checks passed" in r.stdout
    assert os.path.exists(lib)
