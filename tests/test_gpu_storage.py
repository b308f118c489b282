"""Shifted FP16 / BF16 storage of the populations against the FP64 oracle.

The 16-bit forms store X_i - w_i rho_shift^a rounded to nearest even and
compute in FP32.  Two references: the oracle with the same rounding applied
to its post-collision populations (tight: the two differ only where an FP32
and an FP64 value round to neighbouring 16-bit numbers), and the exact FP64
oracle (the 1e-2 gate for FP16, relative to each field's maximum; BF16 is
reported).
"""

import os

import numpy as np
import pytest

from oracle import lbm as olbm
from paper_1601_01237_amd import inputs

from ._gpu_util import oracle_run, rel_err, say

pytestmark = pytest.mark.gpu

CS = 1.0 / np.sqrt(3.0)  # lattice sound speed sqrt(T0), the velocity scale of the u_F gate
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _fields(sim):
    rho, uf, diag = sim.moments()
    return rho.cpu().numpy(), uf.cpu().numpy(), diag


# One unit in the last place of the stored deviation, relative to the field's
# maximum: FP32 arithmetic against FP64 may round a value to the neighbouring
# 16-bit number, and the rest population inherits the others' roundings.
@pytest.mark.parametrize("storage,tol_emul", [("fp16", 2.0 ** -10), ("bf16", 2.0 ** -7)])
def test_16bit_storage_against_emulated_and_exact_oracle(lib, storage, tol_emul):
    from paper_1601_01237_amd.sim import Sim
    say(f"{storage} 32^3 x 20")
    shape = (32, 32, 32)
    rho0 = inputs.sphere_droplet(shape, radius=8.0, seed=0)
    p = olbm.Params(tau=(1.0, 1.0), G=((0.0, -1.0), (-1.0, 0.0)))
    sim = Sim(rho0, tau=p.tau, G=p.G, storage=storage)
    shift = sim.rho_shift
    sim.step(20)
    rho, uf, diag = _fields(sim)
    f_em = oracle_run(rho0, p, 20, storage=storage, rho_shift=shift)
    f_ex = oracle_run(rho0, p, 20)
    rho_em, _ = olbm.observables(f_em, p)
    rho_ex, _ = olbm.observables(f_ex, p)
    e_em = max(rel_err(rho[0], rho_em[0]), rel_err(rho[1], rho_em[1]))
    e_ex = max(rel_err(rho[0], rho_ex[0]), rel_err(rho[1], rho_ex[1]))
    say(f"{storage}: err vs emulated {e_em:.2e}, vs exact {e_ex:.2e}")
    assert e_em < tol_emul, e_em
    if storage == "fp16":
        assert e_ex < 1e-2, e_ex
    # mass of each species is carried by the shift and the stored deviations
    m = np.array([rho_ex[0].sum(), rho_ex[1].sum()])
    got = np.array([diag["mass_a"], diag["mass_b"]])
    assert np.all(np.abs(got - m) <= 2e-3 * m), (got, m)
    sim.close()


def _crop_input():
    rho_big, _, _ = inputs.random_droplets((512, 512, 512), count=64, rmin=8.0, rmax=24.0, seed=0)
    crop = np.ascontiguousarray(rho_big[:, :64, :64, :64])
    del rho_big
    return crop


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
def test_crop64_2000_steps_against_oracle(lib, storage):
    """64^3 crop of the 512^3 droplet field, tau = 0.6, G = -1, 2000 steps."""
    from paper_1601_01237_amd.sim import Sim
    ref = np.load(os.path.join(GOLDEN, "crop64_fp64.npz"))
    say(f"crop64 {storage} x 2000")
    rho0 = _crop_input()
    sim = Sim(rho0, tau=(0.6, 0.6), G=-1.0, storage=storage)
    idx = ref["idx"]
    report = {}
    t = 0
    for step in ref["steps"]:
        sim.step(int(step) - t)
        t = int(step)
        rho, uf, diag = _fields(sim)
        mx = ref[f"max_{t}"]
        r = rho.reshape(2, -1)[:, idx]
        u = uf.reshape(3, -1)[:, idx]
        want_r = ref[f"rho_{t}"]
        want_u = ref[f"uf_{t}"]
        e_a = float(np.max(np.abs(r[0] - want_r[0])) / mx[0])
        e_b = float(np.max(np.abs(r[1] - want_r[1])) / mx[1])
        e_u = float(np.max(np.abs(u - want_u)) / CS)
        e_umax = float(np.max(np.abs(u - want_u)) / mx[2])
        d_ref = ref[f"diag_{t}"]
        e_m = float(max(abs(diag["mass_a"] - d_ref[0]) / d_ref[0], abs(diag["mass_b"] - d_ref[1]) / d_ref[1]))
        report[t] = (e_a, e_b, e_u, e_m, e_umax)
        assert diag["nonfinite"] == 0
    say(f"crop64 {storage}: " + " ".join(
        f"t={k}: rhoA {v[0]:.1e} rhoB {v[1]:.1e} uF/cs {v[2]:.1e} mass {v[3]:.1e} uF/max {v[4]:.1e}"
        for k, v in report.items()))
    e_a, e_b, e_u, e_m, _ = report[2000]
    if storage == "fp32":
        assert max(e_a, e_b) < 1e-5 and e_m < 1e-6, report[2000]
        assert e_u < 1e-4, report[2000]
    elif storage == "fp16":
        assert max(e_a, e_b) < 1e-2 and e_m < 1e-2, report[2000]
    sim.close()
