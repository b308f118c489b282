"""Helpers shared by the GPU parity tests: run the oracle and the HIP path on
the same seeded inputs and compare them field by field."""

import sys

import numpy as np

from oracle import diagnostics as odiag
from oracle import lbm as olbm


def say(msg):
    """Name the case before each GPU step, flushed, so a crash log shows it."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def oracle_run(rho0, p, steps, solid=None, storage=None, rho_shift=(0.0, 0.0)):
    f = olbm.init_state(rho0, solid)
    if storage is not None:
        fluid = olbm.fluid_mask(rho0.shape[1:], solid)
        f = np.where(fluid, olbm.round_storage(f, storage, rho_shift), 0.0)
        for _ in range(steps):
            f = olbm.step_stored(f, p, storage, rho_shift, solid)
        return f
    return olbm.run(f, p, steps, solid)


def oracle_fields(f, p, solid=None):
    rho_s, uF = olbm.observables(f, p, solid)
    return rho_s, uF


def rel_err(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.max(np.abs(ref))
    if scale == 0.0:
        return float(np.max(np.abs(gpu)))
    return float(np.max(np.abs(gpu - ref)) / scale)


def compare_fields(sim, f_ref, p, solid=None, tol=1e-5, tol_u=None, label=""):
    """Compare rho^A, rho^B, u_F and all populations of ``sim`` with the oracle."""
    rho, uf, diag = sim.moments()
    rho = rho.cpu().numpy()
    uf = uf.cpu().numpy()
    pops = sim.populations().cpu().numpy()
    rho_ref, uf_ref = oracle_fields(f_ref, p, solid)
    errs = {
        "rho_a": rel_err(rho[0], rho_ref[0]),
        "rho_b": rel_err(rho[1], rho_ref[1]),
        "u_f": rel_err(uf, uf_ref),
        "pops": rel_err(pops, f_ref),
    }
    tol_u = tol if tol_u is None else tol_u
    assert errs["rho_a"] <= tol, (label, errs)
    assert errs["rho_b"] <= tol, (label, errs)
    assert errs["pops"] <= tol, (label, errs)
    assert errs["u_f"] <= tol_u, (label, errs)
    return errs, diag


def oracle_diag(f, p, solid=None, **region):
    return odiag.diagnostics(f, p, solid, **region)
