"""Write the oracle references of the long-horizon parity cases.

Every value stored here comes from the FP64 oracle (``oracle/``) run on the
seeded inputs of ``paper_1601_01237_amd.inputs``; nothing is taken from the
HIP path.  Cases (step of Eq. 1 with the collision of Eq. 2 or Eqs. 10-11 and
the force of Eq. 7; walls by halfway bounce-back, Sec. 4):

``c1_32cube``
    32^3 periodic box, sphere R = 8 of species A (1.0 inside, 0.03 outside,
    mirrored for B, +-1e-3 noise, seed 0), tau = 1, G^{AB} = G^{BA} = -1,
    BGK, 200 steps: the configured plain-method case.
``walls_48x24x24_bgk`` / ``walls_48x24x24_regularized``
    The inclined-channel geometry scaled from 384 x 192 x 192 to
    48 x 24 x 24 (x, y, z): walls on z = 0 and z = 23 plus the half space
    below the 30 degree plane through (x, z) = (24, 8), sessile sphere of
    radius 4 centred on the plane, tau = 0.7, G = -1, 200 steps.
``droplet_48cube_g26``
    A droplet that stays: 48^3 periodic box, sphere R = 12 with a tanh
    interface of width 1.5 (seed 0), tau = 1, G = -2.6 (above the demixing
    threshold |G| rho > 2 of the bulk-pressure reading), BGK, 2000 steps.

Stored per case in ``long_<case>.npz``:

* ``rho``, ``uf``: rho^A, rho^B and the three components of u_F (Eqs. 8-9)
  on every cell at the last step, rounded to float32 (a relative change of
  at most 2^-24, far below the 1e-5 parity tolerance);
* ``idx`` and, per checkpoint step t, ``rho_<t>``/``uf_<t>`` at those sample
  cells (float64) and ``max_<t>`` = (max |rho^A|, max |rho^B|, max |u_F|)
  over all cells, for the error against step;
* ``diag_<t>``: the oracle's diagnostic vector at every checkpoint with the
  region ``center``, ``r_in``, ``r_out``, ``thr`` stored alongside;
* ``mass0``: the species masses at t = 0.

    python tests/golden/make_long_goldens.py [case ...]
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import diagnostics as odiag  # noqa: E402
from oracle import lbm  # noqa: E402
from paper_1601_01237_amd import inputs  # noqa: E402

N_RANDOM = 1024
N_BAND = 1024


def _case(name):
    """(rho0, solid, Params, steps, checkpoints, region) of a named case."""
    if name == "c1_32cube":
        shape = (32, 32, 32)
        rho0 = inputs.sphere_droplet(shape, radius=8.0, seed=0)
        p = lbm.Params(tau=(1.0, 1.0), G=((0.0, -1.0), (-1.0, 0.0)))
        region = dict(center=(15.5, 16.25, 17.0), r_in=4.0, r_out=11.0, thr=0.3)
        return rho0, None, p, 200, (1, 10, 100, 200), region
    if name.startswith("walls_48x24x24_"):
        collision = name.rsplit("_", 1)[1]
        shape = (24, 24, 48)
        rho0, solid = inputs.inclined_channel(shape, angle_deg=30.0, radius=4.0, seed=0)
        p = lbm.Params(tau=(0.7, 0.7), G=((0.0, -1.0), (-1.0, 0.0)), collision=collision)
        region = dict(center=(24.0, 12.0, 8.0), r_in=3.0, r_out=6.0, thr=0.4)
        return rho0, solid, p, 200, (1, 10, 100, 200), region
    if name == "droplet_48cube_g26":
        shape = (48, 48, 48)
        rho0 = inputs.sphere_droplet(shape, radius=12.0, seed=0, width=1.5)
        p = lbm.Params(tau=(1.0, 1.0), G=((0.0, -2.6), (-2.6, 0.0)))
        region = dict(center=(24.0, 24.0, 24.0), r_in=6.0, r_out=18.0, thr=0.515)
        return rho0, None, p, 2000, (1, 10, 100, 500, 1000, 2000), region
    raise ValueError(name)


CASES = ("c1_32cube", "walls_48x24x24_bgk", "walls_48x24x24_regularized", "droplet_48cube_g26")


def sample_cells(rho0, solid):
    """Seeded sample: cells drawn uniformly, plus cells of the initial interface."""
    rng = np.random.default_rng(321)
    n = rho0[0].size
    fluid = np.ones(n, bool) if solid is None else ~solid.reshape(-1)
    ra = rho0[0].reshape(-1)
    cand = np.nonzero(fluid)[0]
    band = np.nonzero(fluid & (ra > 0.1) & (ra < 0.9))[0]
    if band.size < 16:  # sharp interfaces: the cells next to the droplet
        band = np.nonzero(fluid & (ra > 0.5))[0]
    a = rng.choice(cand, size=min(N_RANDOM, cand.size), replace=False)
    b = rng.choice(band, size=min(N_BAND, band.size), replace=False)
    return np.unique(np.concatenate([a, b]))


def main(names):
    for name in names:
        rho0, solid, p, steps, ckpts, region = _case(name)
        idx = sample_cells(rho0, solid)
        f = lbm.init_state(rho0, solid)
        fluid = lbm.fluid_mask(rho0.shape[1:], solid)
        out = {"steps": np.array(ckpts), "idx": idx, "n_steps": np.array(steps),
               "center": np.array(region["center"]), "r_in": np.array(region["r_in"]),
               "r_out": np.array(region["r_out"]), "thr": np.array(region["thr"]),
               "mass0": np.array([rho0[0][fluid].sum(), rho0[1][fluid].sum()])}
        t0 = time.time()
        for t in range(1, steps + 1):
            f = lbm.step(f, p, solid)
            if t in ckpts:
                rho_s, uF = lbm.observables(f, p, solid)
                flat = lambda a: a.reshape(a.shape[0], -1)[:, idx]
                out[f"rho_{t}"] = flat(rho_s)
                out[f"uf_{t}"] = flat(uF)
                out[f"max_{t}"] = np.array([np.abs(rho_s[0]).max(), np.abs(rho_s[1]).max(),
                                            np.sqrt((uF ** 2).sum(axis=0)).max()])
                out[f"diag_{t}"] = odiag.diagnostics(f, p, solid, **region)
                if t == steps:
                    out["rho"] = rho_s.astype(np.float32)
                    out["uf"] = uF.astype(np.float32)
                print(f"{name} t={t} {time.time() - t0:.0f}s", flush=True)
        np.savez_compressed(os.path.join(HERE, f"long_{name}.npz"), **out)


if __name__ == "__main__":
    main(sys.argv[1:] or CASES)
