"""Sim.tune: the z-chunk search leaves the run bitwise unchanged.

Every tiling computes the same step, and tune() restores the state and time
level it started from, so a tuned run and an untuned run from the same input
hold identical states after the same number of steps."""

import pytest
import torch

from paper_1601_01237_amd import inputs

from ._gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_tune_keeps_the_run_bitwise(lib, storage):
    from paper_1601_01237_amd.sim import Sim
    say(f"tune {storage}")
    rho0, solid = inputs.inclined_channel((40, 48, 64), angle_deg=30.0, radius=10.0, seed=0)
    if storage == "fp16":
        solid = None
        rho0 = inputs.sphere_droplet((40, 48, 64), radius=10.0, seed=0)
    ref = Sim(rho0, tau=(0.8, 0.8), G=-1.0, storage=storage, solid=solid)
    ref.step(7)
    sim = Sim(rho0, tau=(0.8, 0.8), G=-1.0, storage=storage, solid=solid)
    sim.step(3)
    tiles = (-1, 0, 2, 8) if storage == "fp16" else (-1, 0, 1, 3)
    tile, z, times = sim.tune(zchunks=(0, 8, 16, 32, 64), tiles=tiles, steps=3)
    assert sim.t == 3
    # 64 > nz is skipped; on folded 16-bit rows every shape runs, with walls
    # every single-cell shape
    assert set(times) == {(t, zc) for t in tiles for zc in (0, 8, 16, 32)}
    assert (tile, z) in times and sim.tiling == (tile, z)
    sim.step(4)
    torch.cuda.synchronize()
    assert torch.equal(sim.state, ref.state)
    sim.close()
    ref.close()
