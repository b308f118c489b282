"""The five benchmark workloads as named presets, run end to end on the GPU.

Each preset runs its workload with seeded synthetic inputs through the
library and returns one flat record (config, seeds, steps, time per step,
MLUPS, diagnostics); ``--jsonl`` appends the records to a file.

* ``C1``  32^3 droplet R = 8, tau = 1, G = -1: 200 FP32 steps.
* ``C2``  128^3 droplets R in {12, 16, 24, 32} at tau in {0.55, 0.8, 1.0,
  1.5}, 5000 steps each: Young-Laplace fit of Delta p against 1/R per tau
  (Eq. 12).  ``--physics`` takes the demixing coupling G = -2.6 instead of the
  configured |G| = 1, at which the droplets dissolve; ``--collision
  regularized`` takes the operator of Sec. 3, stable there down to tau ~ 0.65.
* ``C3``  512^3 field of 64 droplets (R ~ U[8, 24]), tau = 0.6, 2000 steps in
  FP32, FP16 and BF16: time per step and mass drift of each form.
* ``C4``  384 x 192 x 192 channel with the 30-degree inclined wall and a
  sessile droplet R = 32, tau = 0.7, 10000 steps: drift of the droplet's
  centre of mass over the last 1000 steps (Sec. 4.2.3).
* ``C5``  96^3 droplet R = 20: 500 forward steps with a checkpoint every 50,
  then the adjoint sweep for L = 1/2 sum (rho_A(T) - target)^2: dL/dG,
  dL/dtau, |dL/drho0| and the time of both sweeps.

    python -m paper_1601_01237_amd.configs C1 [C2 ...] [--physics | --G G] [--collision regularized]
        [--jsonl runs.jsonl]
"""

from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import experiments, inputs
from .sim import Sim


def _timed_steps(sim, steps):
    import torch
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(sim.stream)
    sim.step(steps)
    end.record(sim.stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def _record(name, shape, steps, ms, d0, d1, **extra):
    n = int(np.prod(shape))
    rec = dict(config=name, shape=list(shape), steps=steps, ms_per_step=ms, mlups=n / (ms * 1e-3) / 1e6,
               mass_drift_a=abs(d1["mass_a"] - d0["mass_a"]) / d0["mass_a"],
               mass_drift_b=abs(d1["mass_b"] - d0["mass_b"]) / d0["mass_b"],
               max_uf=d1["max_uf"], nonfinite=d1["nonfinite"])
    rec.update(extra)
    return rec


def c1():
    shape = (32, 32, 32)
    sim = Sim(inputs.sphere_droplet(shape, radius=8.0, seed=0), tau=(1.0, 1.0), G=-1.0)
    d0 = sim.moments(want_fields=False)[2]
    ms = _timed_steps(sim, 200)
    d1 = sim.moments(want_fields=False)[2]
    sim.close()
    return [_record("C1", shape, 200, ms, d0, d1, seed=0, storage="fp32")]


def c2(physics=False, collision="bgk", G=None):
    G = G if G is not None else (experiments.G_PHYS if physics else -1.0)
    res = experiments.laplace_sweep(n=128, radii=(12.0, 16.0, 24.0, 32.0), taus=(0.55, 0.8, 1.0, 1.5), G=G,
                                    steps=5000, collision=collision)
    recs = []
    for tau, fit in res["fits"].items():
        recs.append(dict(config="C2", shape=[128, 128, 128], steps=5000, G=G, tau=tau, collision=collision, **fit))
    for q in res["points"]:
        recs.append(dict(config="C2-point", G=G, **{k: q[k] for k in ("R0", "tau", "R_eq", "dp", "nonfinite",
                                                                      "max_uf", "mass_drift") if k in q}))
    return recs


def c3(steps=2000):
    shape = (512, 512, 512)
    rho0, _, _ = inputs.random_droplets(shape, count=64, rmin=8.0, rmax=24.0, seed=0)
    recs = []
    for storage in ("fp32", "fp16", "bf16"):
        sim = Sim(rho0, tau=(0.6, 0.6), G=-1.0, storage=storage)
        d0 = sim.moments(want_fields=False)[2]
        ms = _timed_steps(sim, steps)
        d1 = sim.moments(want_fields=False)[2]
        sim.close()
        recs.append(_record("C3", shape, steps, ms, d0, d1, seed=0, storage=storage))
    return recs


def c4(physics=False, collision="bgk", G=None):
    # As configured (G = -1, tau = 0.7) the droplet dissolves.  The physics
    # run uses the demixing coupling at tau = 1: at tau = 0.7 and G = -2.3 a
    # growing flow develops even in a periodic box without walls (max |u_F|
    # 0.16 after 3000 steps, R = 32), i.e. a bulk instability at low
    # viscosity, not a wall effect.
    G = G if G is not None else (-2.3 if physics else -1.0)
    tau = 1.0 if physics else 0.7
    t0 = time.perf_counter()
    res = experiments.incline_drift(shape=(192, 192, 384), angle=30.0, radius=32.0, G=G, tau=tau, steps=10000,
                                    collision=collision)
    res.update(config="C4", shape=[192, 192, 384], wall_seconds=time.perf_counter() - t0)
    return [res]


def c5(n=96, steps=500, every=50):
    import torch
    from .autograd import LBMFunction
    radius = 20.0 * n / 96.0
    rho0 = torch.tensor(inputs.sphere_droplet((n, n, n), radius=radius, seed=0), device="cuda",
                        requires_grad=True)
    target = torch.tensor(inputs.target_ellipsoid((n, n, n), radius=radius, seed=1), device="cuda",
                          dtype=torch.float64)
    G = torch.tensor(-1.0, dtype=torch.float64, requires_grad=True)
    tau = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rho = LBMFunction.apply(rho0, G, tau, steps, every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L = 0.5 * ((rho[0].double() - target) ** 2).sum()
    L.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return [dict(config="C5", shape=[n, n, n], steps=steps, checkpoint_every=every, loss=float(L.detach()),
                 dL_dG=float(G.grad), dL_dtau=float(tau.grad), dL_drho0_norm=float(rho0.grad.norm()),
                 forward_seconds=t1 - t0, backward_seconds=t2 - t1)]


RUNNERS = {"C1": c1, "C2": c2, "C3": c3, "C4": c4, "C5": c5}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("configs", nargs="+", choices=sorted(RUNNERS))
    ap.add_argument("--physics", action="store_true", help="C2/C4 at the demixing coupling G = -2.6")
    ap.add_argument("--collision", default="bgk", choices=["bgk", "regularized"], help="C2/C4 collision operator")
    ap.add_argument("--G", type=float, default=None, help="C2/C4 coupling G^AB = G^BA (overrides --physics)")
    ap.add_argument("--jsonl", default=None, help="append the records to this file")
    args = ap.parse_args(argv)
    for name in args.configs:
        fn = RUNNERS[name]
        if name in ("C2", "C4"):
            recs = fn(physics=args.physics, collision=args.collision, G=args.G)
        else:
            recs = fn()
        for r in recs:
            line = json.dumps(r, default=float)
            print(line, flush=True)
            if args.jsonl:
                with open(args.jsonl, "a") as f:
                    f.write(line + "\n")


if __name__ == "__main__":
    main()
