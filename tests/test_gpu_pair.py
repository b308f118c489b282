"""Paired march of folded 16-bit rows against the single-cell march.

With even nx the 16-bit forms store each row folded (32-bit word k holds
cells k and k + nx/2) and the step runs with two cells per lane.  Both
marches run the same cell arithmetic, so their stored states must agree
bitwise over several steps, tile shapes and z chunks; the single-cell march
and the paired one are each checked against the oracle elsewhere (odd and
even nx).  Shapes cover a ragged x-y plane, the shortest folded row (nx = 2,
where both fold crossings hit the same word), rows longer than one tile, and
one- and two-plane boxes (every z neighbour is the plane itself or the other).
"""

import numpy as np
import pytest
import torch

from oracle import lbm as olbm
from paper_1601_01237_amd import inputs

from ._gpu_util import oracle_run, rel_err, say

pytestmark = pytest.mark.gpu

SHAPES = [(20, 19, 70), (6, 5, 2), (9, 7, 130), (5, 33, 64), (1, 1, 2), (2, 1, 6), (1, 3, 4)]
PAIR_TILINGS = [(6, 0), (7, 0), (8, 0), (9, 0), (6, 1), (7, 3), (8, 2), (9, 5)]


def _state(rho0, storage, collision, tile, zchunk, steps=7):
    from paper_1601_01237_amd.sim import Sim
    sim = Sim(rho0, tau=(0.8, 1.1), G=-1.4, storage=storage, collision=collision, tile=tile, zchunk=zchunk)
    sim.step(steps)
    x = sim.state.clone().cpu()
    sim.close()
    return x


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("collision", ["bgk", "regularized"])
@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_paired_equals_single_cell_bitwise(lib, storage, collision, shape):
    say(f"paired vs single-cell {storage} {collision} {shape}")
    rho0 = inputs.sphere_droplet(shape, radius=max(1.0, min(shape) / 3.0), seed=11)
    ref = _state(rho0, storage, collision, 0, 0)
    for tile, zc in PAIR_TILINGS:
        got = _state(rho0, storage, collision, tile, zc)
        assert torch.equal(got, ref), (tile, zc)


def test_pair_shapes_rejected_where_rows_are_not_folded(lib):
    from paper_1601_01237_amd.sim import Sim
    say("pair shapes on unfolded rows")
    rho0 = inputs.sphere_droplet((6, 6, 7), radius=2.0, seed=1)
    for storage in ("fp32", "fp16"):
        sim = Sim(rho0, tau=(1.0, 1.0), G=-1.0, storage=storage)  # fp32, or odd nx
        with pytest.raises(RuntimeError):
            sim.set_tiling(6, 0)
        sim.close()
    solid = np.zeros((6, 6, 8), bool)
    solid[0] = True
    rho1 = inputs.sphere_droplet((6, 6, 8), radius=2.0, seed=1)
    rho1[:, solid] = 0.0
    sim = Sim(rho1, tau=(1.0, 1.0), G=-1.0, storage="fp16", solid=solid)
    with pytest.raises(RuntimeError):
        sim.set_tiling(7, 0)
    sim.close()


@pytest.mark.parametrize("shape,walls", [((12, 10, 15), False), ((10, 9, 22), False), ((10, 9, 22), True),
                                         ((10, 9, 22), "porous")])
def test_fp16_odd_and_even_rows_against_emulated_oracle(lib, shape, walls):
    """Unfolded (odd nx, or walls: single-cell march) and folded (even nx
    without walls: paired march) FP16 rows against the oracle with the same
    storage rounding.  The obstacle geometry reads one-byte wall classes,
    the random porous one (more distinct link words than classes) the
    4-byte link words."""
    from paper_1601_01237_amd.sim import Sim
    say(f"fp16 {shape} walls={walls} x 12 vs emulated oracle")
    rho0 = inputs.sphere_droplet(shape, radius=3.5, seed=4)
    solid = None
    if walls == "porous":
        solid = np.random.default_rng(8).uniform(size=shape) < 0.3
        solid[0] = True
        rho0[:, solid] = 0.0
    elif walls:
        solid = np.zeros(shape, bool)
        solid[0] = True
        solid[5, 2:5, 3:9] = True
        rho0[:, solid] = 0.0
    p = olbm.Params(tau=(0.9, 0.7), G=((0.0, -1.2), (-1.2, 0.0)), rho_wall=(0.2, 0.1))
    sim = Sim(rho0, tau=p.tau, G=p.G, storage="fp16", solid=solid, rho_wall=p.rho_wall)
    if walls:
        assert (sim.wall_classes() > 0) == (walls is True)
    assert (sim.row_half > 0) == (shape[2] % 2 == 0 and not walls)
    sim.step(12)
    rho = sim.moments()[0].cpu().numpy()
    pops = sim.populations().cpu().numpy()
    f_em = oracle_run(rho0, p, 12, solid=solid, storage="fp16", rho_shift=sim.rho_shift)
    rho_em, _ = olbm.observables(f_em, p, solid)
    e = max(rel_err(rho[0], rho_em[0]), rel_err(rho[1], rho_em[1]))
    e_pop = rel_err(pops, f_em)
    say(f"fp16 {shape} walls={walls}: rho {e:.2e} pops {e_pop:.2e}")
    assert e < 2.0 ** -10 and e_pop < 2.0 ** -10, (e, e_pop)
    sim.close()


def test_folded_state_layout_round_trip(lib):
    """to/from_state_layout and get/set_populations agree on the folded order."""
    from paper_1601_01237_amd.sim import Sim
    say("folded layout round trip")
    shape = (4, 5, 10)
    rho0 = inputs.sphere_droplet(shape, radius=2.0, seed=2)
    sim = Sim(rho0, tau=(1.0, 1.0), G=-1.0, storage="fp16")
    assert sim.row_half == 5
    # a stored state whose value encodes the cell's x coordinate
    nz, ny, nx = shape
    x = torch.arange(nx, dtype=torch.float32).expand(2, 19, nz, ny, nx) * 0.01
    flat = sim.to_state_layout(x.to(torch.float16).cuda())
    back = sim.from_state_layout(flat).float().cpu()
    assert torch.equal(back, x.to(torch.float16).float())
    raw = sim.plane_view(flat)[0, 0, 0, 0, 0].float().cpu()  # z 0, block 0, A, i = 0, row 0
    want = torch.tensor([0, 5, 1, 6, 2, 7, 3, 8, 4, 9], dtype=torch.float32) * 0.01
    assert torch.equal(raw, want.to(torch.float16).float())
    sim.close()
