"""FP64 CPU oracle: global diagnostics of a two-component state (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may use this module.  Quantities (arXiv 1601.01237):

* species mass sum_x rho^a and mixture momentum sum_x rho u_F (Eqs. 4-9);
* maximum |u_F|, the spurious-velocity measure of Sec. 3;
* bulk pressure p = T0 (rho^A + rho^B) - G T0 rho^A rho^B averaged inside and
  outside a droplet, for the Young-Laplace law of Eq. (12).  This pressure is
  the leading-order continuum form of Eq. (7) (G the symmetric inter-component
  coupling); the paper states no pressure formula;
* count and centre of mass of the cells whose droplet-species density exceeds
  a threshold (the droplet-drift protocol of Sec. 4.2.3).

The layout of the returned vector is the one the GPU diagnostic uses, so the
two can be compared entry by entry.
"""

from __future__ import annotations

import numpy as np

from . import lbm

DIAG_LEN = 16
MASS_A, MASS_B, MOM_X, MOM_Y, MOM_Z, MAX_UF, NONFINITE, N_FLUID = range(8)
P_IN_SUM, N_IN, P_OUT_SUM, N_OUT, N_THR, SDX_THR, SDY_THR, SDZ_THR = range(8, 16)


def _min_image(d, n):
    return d - n * np.round(d / n)


def pressure(rho_a, rho_b, G_ab):
    return lbm.T0 * (rho_a + rho_b) - G_ab * lbm.T0 * rho_a * rho_b


def diagnostics(f, p: lbm.Params, solid=None, center=None, r_in=0.0, r_out=1e30,
                thr=0.515):
    """Diagnostic vector of length DIAG_LEN for pre-collision state ``f``."""
    nz, ny, nx = f.shape[2:]
    fluid = lbm.fluid_mask((nz, ny, nx), solid)
    rho_s, uF = lbm.observables(f, p, solid)
    rho = rho_s[0] + rho_s[1]
    out = np.zeros(DIAG_LEN)
    out[MASS_A] = np.sum(np.where(fluid, rho_s[0], 0.0))
    out[MASS_B] = np.sum(np.where(fluid, rho_s[1], 0.0))
    for a in range(3):
        out[MOM_X + a] = np.sum(np.where(fluid, rho * uF[a], 0.0))
    speed = np.sqrt(uF[0] ** 2 + uF[1] ** 2 + uF[2] ** 2)
    out[MAX_UF] = np.max(np.where(fluid, speed, 0.0))
    bad = ~np.isfinite(rho_s[0]) | ~np.isfinite(rho_s[1]) | ~np.isfinite(uF).all(axis=0)
    out[NONFINITE] = np.count_nonzero(bad & fluid)
    out[N_FLUID] = np.count_nonzero(fluid)

    if center is None:
        center = (nx / 2.0, ny / 2.0, nz / 2.0)
    z, y, x = np.meshgrid(np.arange(nz, dtype=float), np.arange(ny, dtype=float),
                          np.arange(nx, dtype=float), indexing="ij")
    dx = _min_image(x - center[0], nx)
    dy = _min_image(y - center[1], ny)
    dz = _min_image(z - center[2], nz)
    r2 = dx * dx + dy * dy + dz * dz
    G_ab = 0.5 * (p.G[0][1] + p.G[1][0])
    pr = pressure(rho_s[0], rho_s[1], G_ab)
    inner = fluid & (r2 < r_in * r_in)
    outer = fluid & (r2 > r_out * r_out)
    out[P_IN_SUM] = np.sum(np.where(inner, pr, 0.0))
    out[N_IN] = np.count_nonzero(inner)
    out[P_OUT_SUM] = np.sum(np.where(outer, pr, 0.0))
    out[N_OUT] = np.count_nonzero(outer)
    sel = fluid & (rho_s[0] > thr)
    out[N_THR] = np.count_nonzero(sel)
    out[SDX_THR] = np.sum(np.where(sel, dx, 0.0))
    out[SDY_THR] = np.sum(np.where(sel, dy, 0.0))
    out[SDZ_THR] = np.sum(np.where(sel, dz, 0.0))
    return out
