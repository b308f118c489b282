"""lbm_moments_static (the diagnostics entry point that allocates nothing)
against lbm_moments, through the C ABI: fields and all 16 diagnostic entries
bitwise equal, on two calls in a row (the second on a smaller grid, so the
fixed partial-sum array still holds the first call's larger contents), and a
clear error beyond the array's limit."""

import ctypes as C

import numpy as np
import pytest
import torch

from paper_1601_01237_amd import _lib, inputs
from paper_1601_01237_amd.sim import Sim
from tests._gpu_util import say

pytestmark = pytest.mark.gpu


def _both(sim, region):
    """(fields, diag) of lbm_moments and of lbm_moments_static on the same state."""
    lib = sim.lib
    reg = _lib.DiagRegion()
    reg.center[0], reg.center[1], reg.center[2] = region["center"]
    reg.r_in, reg.r_out, reg.thr = region["r_in"], region["r_out"], region["thr"]
    out = []
    for name in ("lbm_moments", "lbm_moments_static"):
        rho = torch.full((2 * sim.n,), float("nan"), dtype=torch.float32, device=sim.device)
        uf = torch.full((3 * sim.n,), float("nan"), dtype=torch.float32, device=sim.device)
        diag = torch.full((_lib.DIAG_LEN,), float("nan"), dtype=torch.float64, device=sim.device)
        code = getattr(lib, name)(sim.ctx, C.c_void_p(rho.data_ptr()), C.c_void_p(uf.data_ptr()),
                                  C.c_void_p(diag.data_ptr()), C.byref(reg))
        _lib.check(name, code)
        torch.cuda.synchronize()
        out.append((rho.cpu().numpy(), uf.cpu().numpy(), diag.cpu().numpy()))
    return out


def _check(shape, steps, region, **kw):
    say(f"moments_static {shape} steps={steps} {kw}")
    rho0 = inputs.sphere_droplet(shape, radius=min(shape) / 4.0, seed=3)
    sim = Sim(rho0, tau=(0.9, 1.1), G=-1.6, **kw)
    sim.step(steps)
    (r0, u0, d0), (r1, u1, d1) = _both(sim, region)
    sim.close()
    assert np.isfinite(d0).all() and d0[7] == np.prod(shape)  # entry 7: fluid cells
    np.testing.assert_array_equal(r1, r0)
    np.testing.assert_array_equal(u1, u0)
    np.testing.assert_array_equal(d1, d0)
    return d0


def test_static_moments_equal_lbm_moments_on_two_calls_in_a_row():
    big = _check((40, 72, 136), 5, dict(center=(60.5, 30.25, 20.0), r_in=7.0, r_out=15.0, thr=0.4))
    small = _check((9, 10, 12), 3, dict(center=(5.5, 5.0, 4.0), r_in=2.0, r_out=4.0, thr=0.3))
    # the second (smaller) call reduced only its own workgroups' partials
    assert small[7] == 9 * 10 * 12 and big[7] == 40 * 72 * 136


def test_static_moments_with_walls_and_16bit_storage():
    shape = (24, 24, 48)
    rho0, solid = inputs.inclined_channel(shape, angle_deg=30.0, radius=4.0, seed=0)
    for storage in ("fp32", "fp16"):
        say(f"moments_static walls {shape} {storage}")
        sim = Sim(rho0, tau=(0.7, 0.7), G=-1.0, solid=solid, storage=storage, rho_wall=(0.1, 0.05))
        sim.step(4)
        (r0, u0, d0), (r1, u1, d1) = _both(sim, dict(center=(24.0, 12.0, 8.0), r_in=3.0, r_out=6.0, thr=0.4))
        sim.close()
        np.testing.assert_array_equal(r1, r0)
        np.testing.assert_array_equal(u1, u0)
        np.testing.assert_array_equal(d1, d0)


def test_static_moments_reject_grids_beyond_the_array():
    # 64 x 8 column tiles: 32 x 264 = 8448 tiles in one plane > LBM_STATIC_BLOCKS
    nx, ny, nz = 2048, 2112, 1
    say(f"moments_static limit {nx}x{ny}x{nz}")
    assert (nx // 64) * (ny // 8) > _lib.STATIC_BLOCKS
    rho0 = np.full((2, nz, ny, nx), 0.5)
    sim = Sim(rho0, tau=(1.0, 1.0), G=-1.0)
    diag = torch.empty(_lib.DIAG_LEN, dtype=torch.float64, device=sim.device)
    code = sim.lib.lbm_moments_static(sim.ctx, None, None, C.c_void_p(diag.data_ptr()), None)
    assert code == -5  # LBM_ENOTSUP
    assert sim.lib.lbm_moments_static(None, None, None, None, None) == -1
    # the allocating entry point still answers for this grid
    _, _, d = sim.moments(want_fields=False)
    sim.close()
    assert d["n_fluid"] == nx * ny * nz
