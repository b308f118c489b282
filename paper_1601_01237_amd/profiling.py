"""Counter runs and their summaries for the fused step (rocprofv3 helpers).

Five subcommands:

``run-adjoint``
    Forward then reverse steps of the differentiation workload (n^3 droplet).

``run``
    The program profiled: the library's reference streaming copy
    (``lbm_stream_copy``) on a buffer of known size, then ``--steps`` fused steps
    of one workload.  Each step is one launch of the step kernel.

``traffic``
    Reads the ``counter_collection.csv`` of two ``rocprofv3 --pmc`` runs of
    ``run`` (one with FETCH_SIZE, one with WRITE_SIZE; both in KiB per
    dispatch).  The copy moves a known number of bytes each way, so the ratio
    of that to what the counter reads for it is the counter's scale on this
    device; the step kernel's counters times that scale are its HBM bytes
    per launch.  Writes a text summary and an entry of ``profiles/traffic.json``
    tied to a hash of the kernel sources.

``counters``
    Mean per dispatch of any counters (one or more ``--pmc`` runs of ``run``)
    for the reference copy, the pattern copy (``--march-copy``) and the step.

``stats``
    Formats the ``kernel_stats.csv`` of a ``rocprofv3 --kernel-trace --stats``
    run as a short text table.

    python -m paper_1601_01237_amd.profiling run --workload 128 --storage fp32
    python -m paper_1601_01237_amd.profiling traffic --fetch F.csv --write W.csv ...
    python -m paper_1601_01237_amd.profiling stats --csv kernel_stats.csv ...
"""

from __future__ import annotations

import argparse
import csv
import ctypes
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
# Sources each kernel is built from, with the launch choices (api.hip).
COMMON_SOURCES = ("pull.h", "cell.h", "buffer.h", "lattice.h", "launch.h", "api.hip")
KERNEL_SOURCES = {"step": ("march.hip", "march_pair.hip") + COMMON_SOURCES,
                  "reverse": ("adjoint_march.hip", "adjoint_cell.h") + COMMON_SOURCES}
BYTES_PER_CELL = {"fp32": 304, "fp16": 160, "bf16": 160}
SHAPES = {"128": (128, 128, 128), "512": (512, 512, 512), "walls": (192, 192, 384), "adjoint96": (96, 96, 96),
          "adjoint256": (256, 256, 256)}
# Algorithmic bytes per cell of one reverse step: X_t and lam_{t+1} read once,
# lam_t written once (FP32).
ADJOINT_BYTES_PER_CELL = 456


def _code_only(text):
    """Source text without comments and blank space (comment edits keep the hash)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(kind="step"):
    """Hash of the code (comments removed) of the sources a kernel is built from."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kind]:
        with open(os.path.join(HERE, "csrc", name)) as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def workload(name, storage, collision="bgk"):
    """(shape, kwargs of Sim) of a named benchmark workload."""
    shape, kw = _workload(name, storage)
    kw["collision"] = collision
    return shape, kw


def _workload(name, storage):
    from . import inputs
    if name == "128":
        shape = (128, 128, 128)
        return shape, dict(rho0=inputs.sphere_droplet(shape, radius=16.0, seed=0), tau=(1.0, 1.0), G=-1.0,
                           storage=storage)
    if name == "512":
        shape = (512, 512, 512)
        rho0, _, _ = inputs.random_droplets(shape, count=64, rmin=8.0, rmax=24.0, seed=0)
        return shape, dict(rho0=rho0, tau=(0.6, 0.6), G=-1.0, storage=storage)
    if name == "walls":
        shape = (192, 192, 384)
        rho0, solid = inputs.inclined_channel(shape, angle_deg=30.0, radius=32.0, seed=0)
        return shape, dict(rho0=rho0, solid=solid, tau=(0.7, 0.7), G=-1.0, storage=storage)
    raise ValueError(name)


def copy_bytes(gib):
    return (int(gib * (1 << 30)) // 16) * 16


def _reference_copy(args):
    """The calibration copy: ``--copy-reps`` launches of lbm_stream_copy over
    ``--copy-gib`` GiB."""
    import torch
    from . import _lib
    lib = _lib.load()
    n = copy_bytes(args.copy_gib)
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    h = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    for _ in range(args.copy_reps):
        _lib.check("lbm_stream_copy", lib.lbm_stream_copy(ctypes.c_void_p(src.data_ptr()),
                                                           ctypes.c_void_p(dst.data_ptr()), n, h))
    torch.cuda.synchronize()
    del src, dst
    print(f"[profiling] copied {args.copy_reps} x {n} bytes", flush=True)


def cmd_run(args):
    import torch
    from . import _lib
    from .sim import Sim
    lib = _lib.load()
    _reference_copy(args)
    shape, kw = workload(args.workload, args.storage, args.collision)
    sim = Sim(**kw)
    if args.zchunk or args.tile >= 0:
        sim.set_tiling(args.tile, args.zchunk)
    sim.set_placement(args.order, args.xoff)
    if args.march_copy:
        # the step's access pattern without arithmetic, on a copy of the state
        dst = torch.empty_like(sim.state)
        for _ in range(args.march_copy):
            _lib.check("lbm_march_copy", lib.lbm_march_copy(sim.ctx, ctypes.c_void_p(sim.state.data_ptr()),
                                                             ctypes.c_void_p(dst.data_ptr())))
        torch.cuda.synchronize()
        del dst
    sim.step(args.steps)
    torch.cuda.synchronize()
    sim.close()
    print(f"[profiling] {args.workload} {args.storage}: {args.steps} steps of {shape}", flush=True)


def cmd_run_adjoint(args):
    """Forward steps and reverse steps of the 96^3 differentiation workload."""
    import torch
    from . import inputs
    from .autograd import Reverse
    from .sim import Sim
    _reference_copy(args)
    n = args.n
    rho0 = inputs.sphere_droplet((n, n, n), radius=20.0 * n / 96.0, seed=0)
    sim = Sim(rho0, tau=(1.0, 1.0), G=-1.0, collision=args.collision)
    if args.shape >= 0 or args.zchunk:
        sim.set_adjoint_tiling(args.shape, args.zchunk)
    sim.step(args.steps)
    rev = Reverse(sim)
    lam = rev.seed(torch.ones((2, n, n, n), dtype=torch.float32, device=sim.device))
    x_t = sim.state.clone()
    fields = None
    if args.fields:
        # the reverse sweep's path: the recomputed forward step writes the
        # densities and velocity the reverse step reads
        fields = torch.empty(5 * n ** 3, dtype=torch.float32, device=sim.device)
        for _ in range(args.steps):
            sim.restore((x_t, sim.t))
            sim.step_fields(fields)
    for _ in range(args.steps):
        lam, _ = rev.step(x_t, lam, fields=fields)
    torch.cuda.synchronize()
    sim.close()
    print(f"[profiling] adjoint {n}^3: {args.steps} forward and {args.steps} reverse steps", flush=True)


def _rows(path, counter):
    with open(path, newline="") as f:
        return [r for r in csv.DictReader(f) if r["Counter_Name"] == counter]


def _mean_kib(rows, pick):
    vals = [float(r["Counter_Value"]) for r in rows if pick(r["Kernel_Name"])]
    if not vals:
        raise SystemExit("no dispatch matched")
    return sum(vals) / len(vals), len(vals)


def _is_copy(name):
    return "stream_copy_kernel" in name


def _is_step(name):
    # single-cell march in Step mode, or the paired march (Step only)
    return ("march_kernel" in name and "(lbm::Mode)0" in name) or "march_pair_kernel" in name


def _is_step_fields(name):
    # the step that also writes the forward fields of the reverse step
    return "march_kernel" in name and "(lbm::Mode)2" in name


def _is_adjoint(name):
    return "adjoint_march_kernel" in name


def cmd_traffic(args):
    known = copy_bytes(args.copy_gib)
    fetch, write = _rows(args.fetch, "FETCH_SIZE"), _rows(args.write, "WRITE_SIZE")
    c_rd, n_c = _mean_kib(fetch, _is_copy)
    c_wr, _ = _mean_kib(write, _is_copy)
    pick = _is_adjoint if args.workload.startswith("adjoint") else _is_step
    s_rd, n_s = _mean_kib(fetch, pick)
    s_wr, _ = _mean_kib(write, pick)
    f_rd = known / (c_rd * 1024.0)
    f_wr = known / (c_wr * 1024.0)
    rd = s_rd * 1024.0 * f_rd
    wr = s_wr * 1024.0 * f_wr
    shape = SHAPES[args.workload]
    cells = shape[0] * shape[1] * shape[2]
    algo = (ADJOINT_BYTES_PER_CELL if args.workload.startswith("adjoint") else BYTES_PER_CELL[args.storage]) * cells
    # With walls a step reads and writes the populations of fluid cells only:
    # that is the algorithmic traffic; the all-cell figure is kept beside it.
    fluid = cells
    if args.workload == "walls":
        _, kw = _workload("walls", args.storage)
        fluid = int((~kw["solid"]).sum())
    algo_fluid = BYTES_PER_CELL[args.storage] * fluid
    entry = {
        "kernel_hash": kernel_source_hash("reverse" if pick is _is_adjoint else "step"),
        "bytes_per_launch": round(rd + wr),
        "read_bytes_per_launch": round(rd),
        "write_bytes_per_launch": round(wr),
        "algorithmic_bytes_per_launch": algo,
        "traffic_over_algorithmic": round((rd + wr) / algo, 4),
        "fluid_cells": fluid,
        "algorithmic_bytes_fluid": algo_fluid,
        "traffic_over_algorithmic_fluid": round((rd + wr) / algo_fluid, 4),
        "read_over_algorithmic_fluid": round(rd / (algo_fluid / 2), 4),
        "fetch_scale": round(f_rd, 4),
        "write_scale": round(f_wr, 4),
        "step_dispatches": n_s,
        "copy_dispatches": n_c,
        "command": args.command,
    }
    key = f"{args.workload_key}:{args.storage}"
    rec = {}
    if os.path.exists(args.json):
        with open(args.json) as f:
            rec = json.load(f)
    rec[key] = entry
    with open(args.json, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
        f.write("\n")
    rfrac = 2.0 / 3.0 if pick is _is_adjoint else 0.5  # share of the algorithmic bytes that are reads
    lines = [
        f"HBM traffic of the {'fused reverse step' if pick is _is_adjoint else 'fused step'}, "
        f"{args.workload_key} {args.storage} ({cells} cells)",
        "",
        f"command: {args.command}",
        "",
        f"calibration (lbm_stream_copy, {known} bytes read and written per dispatch, {n_c} dispatches):",
        f"  FETCH_SIZE  {c_rd:14.1f} KiB/dispatch -> scale {f_rd:.4f}",
        f"  WRITE_SIZE  {c_wr:14.1f} KiB/dispatch -> scale {f_wr:.4f}",
        f"{'reverse-march' if pick is _is_adjoint else 'step'} kernel ({n_s} dispatches):",
        f"  FETCH_SIZE  {s_rd:14.1f} KiB/dispatch -> read  {rd / 1e6:10.2f} MB",
        f"  WRITE_SIZE  {s_wr:14.1f} KiB/dispatch -> write {wr / 1e6:10.2f} MB",
        f"  total {(rd + wr) / 1e6:.2f} MB per launch vs algorithmic {algo / 1e6:.2f} MB "
        f"({(rd + wr) / algo:.3f}x); read {rd / (algo * rfrac):.3f}x, write {wr / (algo * (1 - rfrac)):.3f}x",
        f"kernel source hash {entry['kernel_hash']}",
    ]
    if fluid != cells:
        lines.insert(-1, f"  fluid cells {fluid} ({fluid / cells:.3f} of all): algorithmic {algo_fluid / 1e6:.2f} MB; "
                         f"total {(rd + wr) / algo_fluid:.3f}x, read {rd / (algo_fluid / 2):.3f}x, "
                         f"write {wr / (algo_fluid / 2):.3f}x of it")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _kernel_class(name):
    if _is_copy(name):
        return "lbm_stream_copy"
    if _is_adjoint(name):
        return "reverse"
    if "march_copy_kernel" in name:
        return "lbm_march_copy"
    if _is_step(name):
        return "step"
    if _is_step_fields(name):
        return "step+fields"
    return None


XCDS, CUS, SIMDS = 8, 256, 1024


def _derived(m):
    """Ratios that name a bound, from the mean counters of one kernel."""
    out = []
    cyc = m.get("GRBM_GUI_ACTIVE", 0.0) / XCDS  # cycles of the dispatch (per XCD)
    if cyc > 0:
        out.append(f"{cyc:.4g} cycles")
        if "SQ_ACTIVE_INST_VALU" in m:
            out.append(f"VALU busy {100.0 * m['SQ_ACTIVE_INST_VALU'] * 4 / SIMDS / cyc:.1f}%")
        if "TA_ADDR_STALLED_BY_TC_CYCLES_sum" in m:
            out.append(f"TA address stalled by L1 {100.0 * m['TA_ADDR_STALLED_BY_TC_CYCLES_sum'] / CUS / cyc:.1f}%")
        if "TA_DATA_STALLED_BY_TC_CYCLES_sum" in m:
            out.append(f"TA data stalled by L1 {100.0 * m['TA_DATA_STALLED_BY_TC_CYCLES_sum'] / CUS / cyc:.1f}%")
        if "TCP_PENDING_STALL_CYCLES_sum" in m:
            out.append(f"L1 pending stall {100.0 * m['TCP_PENDING_STALL_CYCLES_sum'] / CUS / cyc:.1f}%")
        if "TCP_TCC_READ_REQ_LATENCY_sum" in m:
            out.append(f"L1->L2 reads in flight {m['TCP_TCC_READ_REQ_LATENCY_sum'] / cyc:.4g}")
        if "TCP_TCC_READ_REQ_sum" in m:
            out.append(f"L1->L2 read requests/cycle {m['TCP_TCC_READ_REQ_sum'] / cyc:.3g}")
    if m.get("TCP_TCC_READ_REQ_sum", 0.0) > 0 and "TCP_TCC_READ_REQ_LATENCY_sum" in m:
        out.append(f"mean L1->L2 read latency {m['TCP_TCC_READ_REQ_LATENCY_sum'] / m['TCP_TCC_READ_REQ_sum']:.0f} cycles")
    if m.get("TCC_HIT_sum", 0.0) + m.get("TCC_MISS_sum", 0.0) > 0:
        out.append(f"L2 hit rate {100.0 * m['TCC_HIT_sum'] / (m['TCC_HIT_sum'] + m['TCC_MISS_sum']):.1f}%")
    if m.get("SQ_WAVE_CYCLES", 0.0) > 0 and "SQ_WAIT_INST_ANY" in m:
        out.append(f"waves waiting on an instruction {100.0 * m['SQ_WAIT_INST_ANY'] / m['SQ_WAVE_CYCLES']:.1f}% of wave cycles")
    return out


def cmd_counters(args):
    """Mean per dispatch of every counter in one or more counter_collection.csv
    files, for the reference copy, the pattern copy and the step kernel."""
    table = {}
    for path in args.csv:
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                cls = _kernel_class(r["Kernel_Name"])
                if cls is None:
                    continue
                key = (r["Counter_Name"], cls)
                table.setdefault(key, []).append(float(r["Counter_Value"]))
    counters = sorted({k[0] for k in table})
    classes = [c for c in ("lbm_stream_copy", "lbm_march_copy", "step", "step+fields", "reverse")
               if any(k[1] == c for k in table)]
    lines = [args.title, "", f"command: {args.command}", "",
             f"{'counter (mean per dispatch)':32} " + " ".join(f"{c:>18}" for c in classes)]
    for name in counters:
        cells = []
        for c in classes:
            v = table.get((name, c))
            cells.append(f"{sum(v) / len(v):18.6g}" if v else f"{'-':>18}")
        lines.append(f"{name:32} " + " ".join(cells))
    lines += ["", "derived (per dispatch; the GRBM counter is summed over the 8 XCDs, the TA/TCP ones over the",
              "256 CUs, SQ_ACTIVE_INST_VALU counts 4-cycle issue slots over the 1024 SIMDs):"]
    for c in classes:
        d = _derived({name: sum(v) / len(v) for (name, cls), v in table.items() if cls == c})
        if d:
            lines.append(f"  {c}: " + "; ".join(d))
    for note in args.note or ():
        lines.append(note)
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cmd_stats(args):
    with open(args.csv, newline="") as f:
        rows = list(csv.DictReader(f))
    lines = [args.title, "", f"command: {args.command}", "",
             f"{'calls':>7} {'avg us':>10} {'min us':>10} {'max us':>10} {'total %':>8}  kernel"]
    for r in rows:
        name = r["Name"]
        if len(name) > 110:
            name = name[:107] + "..."
        lines.append(f"{int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.2f} {float(r['MinNs']) / 1e3:10.2f} "
                     f"{float(r['MaxNs']) / 1e3:10.2f} {float(r['Percentage']):8.2f}  {name}")
    if args.bench and os.path.exists(args.bench):
        with open(args.bench) as f:
            tail = [ln for ln in f.read().splitlines() if ln.startswith("{")]
        if tail:
            lines += ["", "bench line of the same run:", tail[-1]]
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--workload", default="128", choices=["128", "512", "walls"])
    r.add_argument("--storage", default="fp32", choices=["fp32", "fp16", "bf16"])
    r.add_argument("--steps", type=int, default=5)
    r.add_argument("--collision", default="bgk", choices=["bgk", "regularized"])
    r.add_argument("--copy-gib", type=float, default=2.0)
    r.add_argument("--copy-reps", type=int, default=3)
    r.add_argument("--zchunk", type=int, default=0, help="z planes per workgroup (0 = the library's default)")
    r.add_argument("--tile", type=int, default=-1, help="tile shape (-1 = automatic)")
    r.add_argument("--order", type=int, default=0, help="block order (0 = automatic, see lbm_set_placement)")
    r.add_argument("--xoff", type=int, default=-1, help="x shift of the tile grid (-1 = automatic)")
    r.add_argument("--march-copy", type=int, default=0,
                   help="launches of lbm_march_copy (the step's access pattern) before the steps")
    ra = sub.add_parser("run-adjoint")
    ra.add_argument("--n", type=int, default=96)
    ra.add_argument("--steps", type=int, default=20)
    ra.add_argument("--collision", default="bgk", choices=["bgk", "regularized"])
    ra.add_argument("--shape", type=int, default=-1, help="reverse-march tile shape (-1 = automatic)")
    ra.add_argument("--zchunk", type=int, default=0)
    ra.add_argument("--fields", action="store_true", help="reverse steps read the forward fields (lbm_step_fields)")
    ra.add_argument("--copy-gib", type=float, default=2.0)
    ra.add_argument("--copy-reps", type=int, default=3)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--workload", default="128", choices=["128", "512", "walls", "adjoint96", "adjoint256"])
    t.add_argument("--workload-key", default="128^3")
    t.add_argument("--storage", default="fp32")
    t.add_argument("--copy-gib", type=float, default=2.0)
    t.add_argument("--json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    t.add_argument("--out", required=True)
    t.add_argument("--command", default="")
    s = sub.add_parser("stats")
    s.add_argument("--csv", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--title", default="rocprofv3 kernel statistics")
    s.add_argument("--command", default="")
    s.add_argument("--bench", default=None)
    k = sub.add_parser("counters")
    k.add_argument("--csv", nargs="+", required=True)
    k.add_argument("--out", required=True)
    k.add_argument("--title", default="rocprofv3 counters")
    k.add_argument("--command", default="")
    k.add_argument("--note", action="append")
    args = ap.parse_args(argv)
    {"run": cmd_run, "run-adjoint": cmd_run_adjoint, "traffic": cmd_traffic, "stats": cmd_stats,
     "counters": cmd_counters}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())
