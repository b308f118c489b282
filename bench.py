"""Throughput of the fused two-component D3Q19 step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extra] [--no-cpu]

Headline workload: 128^3 periodic box, two species, D3Q19 BGK with
tau_A = tau_B = 1.0, third-order equilibrium, Shan-Chen G^AB = G^BA = -1.0,
one droplet of species A with R = 16 (rho_A = 1.0 / 0.03, mirrored for B,
+-1e-3 seeded noise), FP32 storage and arithmetic.  One step = one fused
kernel launch updating every cell of both species.  MLUPS = cells * steps /
seconds / 1e6.  The state lives in HBM before the timed region starts.  The
K timed steps run back to back in 5 consecutive windows split by HIP events;
``value`` is taken at the median per-step time over the windows (the
windows, their spread and the mean over all K steps are printed too).

Prints ONE JSON line.  ``roofline`` prices the fused kernel against HBM: 304
algorithmic bytes per cell-step (19 populations x 2 species x 4 B, read once
and written once) divided by the launch duration measured with HIP events on
the stream the kernel runs on.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL = {"fp32": 304, "fp16": 160, "bf16": 160}
ADJOINT_BYTES_PER_CELL = 456
ALGO_BYTES_NOTE = ("2 species x 19 populations x element size (plus the 2 rest-population residuals of the "
                   "16-bit forms), read + write, per cell-step")


def stored_traffic(workload, storage):
    """HBM bytes per launch from committed rocprofv3 counter runs, if the kernel is unchanged."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    key = f"{workload}:{storage}"
    ent = rec.get(key)
    from paper_1601_01237_amd.profiling import kernel_source_hash
    if not ent or ent.get("kernel_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def time_steps(sim, steps, warmup, windows=5):
    """ms per step (= per launch) of ``steps`` steps after ``warmup`` untimed ones.

    The K timed steps run back to back on the context's stream, split into
    ``windows`` consecutive windows of (nearly) equal length with a HIP event
    between windows (no synchronisation inside the timed region).  Returns the
    median over the windows of the per-step time, the per-window times and the
    mean over all K steps."""
    import torch
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = sim.stream
    nwin = max(1, min(windows, steps))
    sizes = [steps // nwin + (1 if k < steps % nwin else 0) for k in range(nwin)]
    events = [torch.cuda.Event(enable_timing=True) for _ in range(nwin + 1)]
    events[0].record(stream)
    for k, m in enumerate(sizes):
        sim.step(m)
        events[k + 1].record(stream)
    torch.cuda.synchronize()
    per = [events[k].elapsed_time(events[k + 1]) / sizes[k] for k in range(nwin)]
    total = events[0].elapsed_time(events[nwin]) / steps
    return float(np.median(per)), per, total


# Tile shapes the tuned cases try besides the automatic one (64 x 12 rows:
# measured fastest on the walls channel, 0.86 against 0.90 ms for 64 x 8).
TUNE_TILES = (-1, 1)


def run_case(shape, storage, steps, warmup, rho0=None, solid=None, tau=1.0, G=-1.0, tile=None, zchunk=None,
             collision="bgk", tune=False):
    from paper_1601_01237_amd import inputs
    from paper_1601_01237_amd.sim import Sim
    if rho0 is None:
        rho0 = inputs.sphere_droplet(shape, radius=shape[0] / 8.0, seed=0)
    sim = Sim(rho0, tau=(tau, tau), G=G, storage=storage, solid=solid, tile=tile, zchunk=zchunk,
              collision=collision)
    tuned = {}
    if tune:
        # tile shape (automatic or 64 x 12) and z chunk measured on this state
        # (restored afterwards), before the warmup
        tile, best, _ = sim.tune(tiles=TUNE_TILES)
        tuned = dict(tile=tile, zchunk=best)
    if solid is not None:
        tuned["wall_classes"] = sim.wall_classes()  # 0: the marches read 4-byte link words
    ms, per, mean_ms = time_steps(sim, steps, warmup)
    _, _, diag = sim.moments(want_fields=False)
    n = int(np.prod(shape))
    sim.close()
    mlups = n / (ms * 1e-3) / 1e6
    gbs = BYTES_PER_CELL[storage] * n / (ms * 1e-3) / 1e9
    return dict(ms_per_step=ms, mlups=mlups, gbs=gbs, nonfinite=diag["nonfinite"], n=n,
                window_ms=[round(v, 5) for v in per], mean_ms_per_step=mean_ms, **tuned)


def adjoint_cost(n=96, steps=20, adjoint_tile=None, collision="bgk"):
    """Forward step vs one reverse step on the differentiation workload (n^3, R = 20 n / 96).

    The reverse sweep recomputes each forward step with lbm_step_fields
    (the step plus the densities and velocity the reverse step reads) and
    runs lbm_adjoint_step_fields; the reverse step that pulls those itself
    (lbm_adjoint_step) is timed too.  Both at the library's automatic tiling
    unless ``adjoint_tile`` names the reverse march's shape; ``collision`` is
    the operator of both."""
    import torch
    from paper_1601_01237_amd import inputs
    from paper_1601_01237_amd.autograd import Reverse
    from paper_1601_01237_amd.sim import Sim
    rho0 = inputs.sphere_droplet((n, n, n), radius=20.0 * n / 96.0, seed=0)
    sim = Sim(rho0, tau=(1.0, 1.0), G=-1.0, collision=collision)
    fwd_ms = time_steps(sim, steps, 5)[0]
    if adjoint_tile is not None:
        sim.set_adjoint_tiling(adjoint_tile, 0)
    fields = torch.empty(5 * n ** 3, dtype=torch.float32, device=sim.device)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(sim.stream)
        for _ in range(steps):
            fn()
        end.record(sim.stream)
        torch.cuda.synchronize()
        return start.elapsed_time(end) / steps

    x_t = sim.state.clone()
    fwd_fields_ms = timed(lambda: sim.step_fields(fields))
    # fields of x_t (the state the reverse steps below differentiate at)
    sim.restore((x_t, sim.t))
    sim.step_fields(fields)
    rev = Reverse(sim)
    grad = torch.ones((2, n, n, n), dtype=torch.float32, device=sim.device)
    lam0 = rev.seed(grad)
    box = {"lam": lam0}

    def rstep(f):
        box["lam"], _ = rev.step(x_t, box["lam"], fields=f)

    adj_ms = timed(lambda: rstep(fields))
    box["lam"] = lam0
    adj_pull_ms = timed(lambda: rstep(None))
    sim.close()
    # one reverse step reads X_t and lam_{t+1} and writes lam_t: 456 B per cell
    gbs = ADJOINT_BYTES_PER_CELL * n ** 3 / (adj_ms * 1e-3) / 1e9
    return dict(forward_ms=round(fwd_ms, 4), forward_fields_ms=round(fwd_fields_ms, 4),
                adjoint_step_ms=round(adj_ms, 4), adjoint_step_pull_ms=round(adj_pull_ms, 4),
                ratio=round(adj_ms / fwd_ms, 3),
                ratio_with_recompute=round((adj_ms + fwd_fields_ms) / fwd_ms, 3),
                algorithmic_bytes_per_cell=ADJOINT_BYTES_PER_CELL, gbs=round(gbs, 1),
                frac=round(gbs / HBM_PEAK_GBS, 4))


def copy_ceiling(gib=4.0, reps=10):
    """Read + write bandwidth of the library's plain streaming copy (GB/s)."""
    import ctypes
    import torch
    from paper_1601_01237_amd import _lib
    lib = _lib.load()
    n = int(gib * (1 << 30))
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    h = ctypes.c_void_p(stream.cuda_stream)
    for _ in range(2):
        _lib.check("lbm_stream_copy", lib.lbm_stream_copy(ctypes.c_void_p(src.data_ptr()),
                                                           ctypes.c_void_p(dst.data_ptr()), n, h))
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        _lib.check("lbm_stream_copy", lib.lbm_stream_copy(ctypes.c_void_p(src.data_ptr()),
                                                           ctypes.c_void_p(dst.data_ptr()), n, h))
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / reps
    del src, dst
    return 2.0 * n / (ms * 1e-3) / 1e9


def pattern_ceiling(shape, storage="fp32", reps=20):
    """Rate (GB/s of algorithmic bytes) of lbm_march_copy on ``shape``: the
    step's access pattern (tiles, z march, 38 loads then 38 stores per cell)
    with no arithmetic, halo or re-read."""
    import torch
    from paper_1601_01237_amd import inputs
    from paper_1601_01237_amd.sim import Sim
    sim = Sim(inputs.sphere_droplet(shape, radius=4.0, seed=0), storage=storage)
    src = sim.bufs[0]
    dst = torch.empty_like(sim.bufs[1])
    for _ in range(2):
        _lib_call(sim, src, dst)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(sim.stream)
    for _ in range(reps):
        _lib_call(sim, src, dst)
    end.record(sim.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / reps
    n = int(np.prod(shape))
    sim.close()
    del dst
    return BYTES_PER_CELL[storage] * n / (ms * 1e-3) / 1e9


def _rounded(r):
    return {k: (v if isinstance(v, list) else round(v, 3)) for k, v in r.items() if k != "n"}


def _lib_call(sim, src, dst):
    import ctypes
    from paper_1601_01237_amd import _lib
    _lib.check("lbm_march_copy", sim.lib.lbm_march_copy(sim.ctx, ctypes.c_void_p(src.data_ptr()),
                                                         ctypes.c_void_p(dst.data_ptr())))


def cpu_baseline(shape, seconds_budget=12.0, max_steps=8):
    """The FP64 oracle on whole steps of the headline workload, one thread.

    Steps until ``seconds_budget`` has passed (at most ``max_steps``); any
    BLAS the oracle reaches is limited to one thread."""
    from threadpoolctl import threadpool_limits
    from oracle import lbm as olbm
    from paper_1601_01237_amd import inputs
    rho0 = inputs.sphere_droplet(shape, radius=16.0, seed=0)
    p = olbm.Params(tau=(1.0, 1.0), G=((0.0, -1.0), (-1.0, 0.0)))
    f = olbm.init_state(rho0)
    steps = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while True:
            f = olbm.step(f, p)
            steps += 1
            if time.perf_counter() - t0 > seconds_budget or steps >= max_steps:
                break
        dt = time.perf_counter() - t0
    n = int(np.prod(shape))
    return dict(value=n * steps / dt / 1e6, unit="MLUPS", cores=1, kind="oracle",
                sample=f"{steps} step(s) of the {shape[2]}x{shape[1]}x{shape[0]} workload, FP64 NumPy, "
                       f"{dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--tile", type=int, default=None, help="tile shape of the step kernel (0..9, see lbm_set_tiling)")
    ap.add_argument("--zchunk", type=int, default=None, help="z planes per workgroup (0 = default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the z-slab decomposition is a design note).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1601_01237_amd import _lib, inputs
    _lib.load()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)

    n = args.n
    shape = (n, n, n)
    rho0 = inputs.sphere_droplet(shape, radius=16.0, seed=0)
    print(f"[bench] headline {n}^3 fp32 steps={args.steps} warmup={args.warmup}", file=sys.stderr, flush=True)
    head = run_case(shape, "fp32", args.steps, args.warmup, rho0=rho0, tile=args.tile, zchunk=args.zchunk)
    ncell = head["n"]
    achieved = BYTES_PER_CELL["fp32"] * ncell / (head["ms_per_step"] * 1e-3) / 1e9
    workload = f"{n}^3"
    traffic = stored_traffic(workload, "fp32")

    extra = {}
    print("[bench] copy ceiling", file=sys.stderr, flush=True)
    ceiling = copy_ceiling()
    pattern = pattern_ceiling(shape)
    if not args.no_extra:
        steps_big = max(10, args.steps // 10)
        big = (512, 512, 512)
        rho_big, _, _ = inputs.random_droplets(big, count=64, rmin=8.0, rmax=24.0, seed=0)
        for storage in ("fp32", "fp16", "bf16"):
            print(f"[bench] 512^3 {storage}", file=sys.stderr, flush=True)
            r = run_case(big, storage, steps_big, 5, rho0=rho_big, tau=0.6)
            extra[f"512^3_{storage}"] = _rounded(r)
        extra["fp16_over_fp32_512^3"] = round(extra["512^3_fp32"]["ms_per_step"]
                                              / extra["512^3_fp16"]["ms_per_step"], 3)
        print("[bench] 512^3 fp32 regularized", file=sys.stderr, flush=True)
        r = run_case(big, "fp32", steps_big, 5, rho0=rho_big, tau=0.6, collision="regularized")
        extra["512^3_fp32_regularized"] = _rounded(r)
        del rho_big
        print("[bench] walls 384x192x192", file=sys.stderr, flush=True)
        rho_w, solid = inputs.inclined_channel((192, 192, 384), angle_deg=30.0, radius=32.0, seed=0)
        r = run_case((192, 192, 384), "fp32", steps_big, 5, rho0=rho_w, solid=solid, tau=0.7, tune=True)
        fluid = int((~solid).sum())
        r["mlups_fluid_only"] = fluid / (r["ms_per_step"] * 1e-3) / 1e6
        # with walls only fluid cells move populations: the algorithmic bytes
        # are 304 per fluid cell
        r["fluid_fraction"] = fluid / r["n"]
        r["gbs_fluid"] = BYTES_PER_CELL["fp32"] * fluid / (r["ms_per_step"] * 1e-3) / 1e9
        r["frac_fluid"] = r["gbs_fluid"] / HBM_PEAK_GBS
        extra["384x192x192_walls_fp32"] = _rounded(r)
        print("[bench] adjoint 96^3", file=sys.stderr, flush=True)
        extra["adjoint_96^3"] = adjoint_cost()
        extra["adjoint_96^3_regularized"] = adjoint_cost(collision="regularized")
        extra["adjoint_96^3_regularized3"] = adjoint_cost(collision="regularized3")

    cpu = None
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(shape)

    out = {
        "metric": "MLUPS (2-species D3Q19) + % HBM roofline; FP16-storage & adjoint vs FP32",
        "value": round(head["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "timing": {"windows": len(head["window_ms"]), "window_ms_per_step": head["window_ms"],
                   "statistic": "median over windows", "mean_ms_per_step": round(head["mean_ms_per_step"], 5),
                   "spread": round((max(head["window_ms"]) - min(head["window_ms"])) / head["ms_per_step"], 4)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded droplet, +-1e-3 noise)",
        "config": {"workload": f"{n}^3 periodic, 2 species D3Q19 BGK, tau=1.0, G_AB=G_BA=-1.0, "
                               f"droplet R=16, FP32", "cells": ncell, "storage": "fp32",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "algorithmic_bytes_per_cell": BYTES_PER_CELL["fp32"],
                     "algorithmic_bytes_note": ALGO_BYTES_NOTE,
                     "copy_ceiling_gbs": round(ceiling, 1),
                     "frac_of_copy_ceiling": round(achieved / ceiling, 4),
                     "pattern_ceiling_gbs": round(pattern, 1),
                     "frac_of_pattern_ceiling": round(achieved / pattern, 4),
                     "kernel": "march_kernel<F32, no walls, Step, 128x4 tile>"},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
