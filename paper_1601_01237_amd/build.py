"""Build liblbm.so (HIP, gfx950) in-tree with hipcc.

Usage: ``python -m paper_1601_01237_amd.build`` or ``build()`` from Python.
The library lands next to this file as ``liblbm.so``.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = ["march.hip", "march_pair.hip", "adjoint_march.hip", "adjoint.hip", "aux.hip", "api.hip"]

ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # no implicit multiply-add fusion: every instance of a kernel template
    # rounds identically (fused operations are written out with fmaf)
    "-ffp-contract=off",
    # packed FP32 VALU forms are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE,
    "-I", CSRC,
]


def _hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the HIP toolchain is required to build liblbm.so")
    return exe


def _compile(src, extra, objdir=OBJDIR):
    obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj, r.stderr


# AddressSanitizer on the host code only (the device code is built as usual).
HOST_ASAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def build(verbose=False, extra=(), out=None, objdir=None, host_asan=False):
    """Compile every source and link liblbm.so; returns the library path.

    ``host_asan`` instruments the host code with AddressSanitizer (for the
    host-side checks of the C ABI); ``out``/``objdir`` place such a build
    away from the product library."""
    out = out or LIB
    objdir = objdir or OBJDIR
    flags = list(extra) + (HOST_ASAN if host_asan else [])
    os.makedirs(objdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        results = list(ex.map(lambda s: _compile(s, flags, objdir), SOURCES))
    objs = [o for o, _ in results]
    if verbose:
        for _, err in results:
            if err.strip():
                print(err, file=sys.stderr)
    tmp = out + ".tmp"
    link = ["-Xarch_host", "-fsanitize=address", "-shared-libasan"] if host_asan else []
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *link, *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
