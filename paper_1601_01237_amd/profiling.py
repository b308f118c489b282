"""Plain device-to-device copy for calibrating rocprofv3 byte counters.

``python -m paper_1601_01237_amd.profiling --gib 2 --reps 3`` runs the
library's reference streaming copy (lbm_stream_copy) on a buffer of known
size; the counters of those dispatches divided by the known bytes give the
scale between the counters and the bytes actually moved on this device.
"""

import argparse
import ctypes

import torch

from . import _lib


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gib", type=float, default=2.0)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    lib = _lib.load()
    n = (int(args.gib * (1 << 30)) // 16) * 16
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    h = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    for _ in range(args.reps):
        _lib.check("lbm_stream_copy", lib.lbm_stream_copy(ctypes.c_void_p(src.data_ptr()),
                                                           ctypes.c_void_p(dst.data_ptr()), n, h))
    torch.cuda.synchronize()
    print(f"copied {args.reps} x {n} bytes", flush=True)


if __name__ == "__main__":
    main()
