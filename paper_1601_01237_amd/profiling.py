"""Plain device-to-device copy for calibrating rocprofv3 byte counters.

``python -m paper_1601_01237_amd.profiling --gib 2 --reps 3`` copies a buffer
of the given size with torch's copy kernel; FETCH_SIZE / WRITE_SIZE of those
dispatches divided by the known bytes gives the scale between the counters
and real HBM bytes on this device.
"""

import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gib", type=float, default=2.0)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    n = int(args.gib * (1 << 30)) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(args.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {args.reps} x {n * 4} bytes", flush=True)


if __name__ == "__main__":
    main()
