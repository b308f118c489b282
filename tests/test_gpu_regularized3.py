"""The regularized collision that keeps the energy flux as well as the momentum
flux (Sec. 3, Eqs. 10-11, third-order reading) on the GPU against the FP64
oracle: every population and field, on ragged grids and tile shapes, with
walls, at full size and through the 16-bit storage (paired march); and its
reverse step."""

import numpy as np
import pytest
import torch

from oracle import lbm as olbm
from paper_1601_01237_amd import inputs

from ._gpu_util import compare_fields, oracle_run, rel_err, say

pytestmark = pytest.mark.gpu

TOL = 1e-5
REG3 = "regularized3"


def _params(tau, G=-1.0, rho_wall=(0.0, 0.0)):
    return olbm.Params(tau=tau, G=((0.0, G), (G, 0.0)), rho_wall=rho_wall, collision=REG3)


@pytest.mark.parametrize("steps", [1, 10])
def test_droplet_32cube(lib, steps):
    from paper_1601_01237_amd.sim import Sim
    say(f"regularized3 32^3 x {steps}")
    rho0 = inputs.sphere_droplet((32, 32, 32), radius=8.0, seed=0)
    p = _params((0.55, 0.7))
    sim = Sim(rho0, tau=p.tau, G=-1.0, collision=REG3)
    sim.step(steps)
    errs, _ = compare_fields(sim, oracle_run(rho0, p, steps), p, tol=TOL, label=f"reg3 {steps}")
    say(f"regularized3 32^3 x {steps}: {errs}")
    sim.close()


@pytest.mark.parametrize("shape,tile", [((13, 9, 70), -1), ((10, 17, 33), 2), ((9, 6, 131), 3), ((12, 14, 40), 5)])
def test_ragged_grids(lib, shape, tile):
    from paper_1601_01237_amd.sim import Sim
    say(f"regularized3 ragged {shape} tile {tile}")
    rho0 = inputs.sphere_droplet(shape, radius=3.0, seed=4)
    p = _params((0.6, 0.9), G=-1.3)
    sim = Sim(rho0, tau=p.tau, G=-1.3, collision=REG3, tile=tile)
    sim.step(4)
    compare_fields(sim, oracle_run(rho0, p, 4), p, tol=TOL, label=str(shape))
    sim.close()


def test_walls_inclined_channel(lib):
    from paper_1601_01237_amd.sim import Sim
    say("regularized3 walls 48x24x24")
    rho0, solid = inputs.inclined_channel((24, 24, 48), angle_deg=30.0, radius=6.0, seed=0)
    p = _params((0.7, 0.7), rho_wall=(0.1, 0.3))
    sim = Sim(rho0, tau=p.tau, G=-1.0, solid=solid, rho_wall=p.rho_wall, collision=REG3)
    sim.step(20)
    compare_fields(sim, oracle_run(rho0, p, 20, solid), p, solid=solid, tol=TOL, label="reg3 walls")
    sim.close()


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_16bit_storage_against_emulated(lib, storage):
    from paper_1601_01237_amd.sim import Sim
    say(f"regularized3 {storage} 24^3 x 20 (paired march)")
    rho0 = inputs.sphere_droplet((24, 24, 24), radius=6.0, seed=1)
    p = _params((0.8, 0.8))
    sim = Sim(rho0, tau=p.tau, G=-1.0, storage=storage, collision=REG3)
    assert sim.row_half == 12
    sim.step(20)
    rho, _, _ = sim.moments()
    f_em = oracle_run(rho0, p, 20, storage=storage, rho_shift=sim.rho_shift)
    rho_em, _ = olbm.observables(f_em, p)
    e = max(rel_err(rho[0].cpu().numpy(), rho_em[0]), rel_err(rho[1].cpu().numpy(), rho_em[1]))
    say(f"regularized3 {storage} vs emulated {e:.2e}")
    assert e < (2.0 ** -10 if storage == "fp16" else 2.0 ** -7)
    sim.close()


def test_tiling_invariance_bitwise(lib):
    from paper_1601_01237_amd.sim import Sim
    say("regularized3 tiling invariance")
    shape = (18, 19, 70)
    rho0 = inputs.sphere_droplet(shape, radius=5.0, seed=6)
    out = []
    for tile, zc in [(-1, 0), (0, 3), (2, 5), (3, 1), (5, 0)]:
        sim = Sim(rho0, tau=(0.6, 0.6), G=-1.5, collision=REG3, tile=tile, zchunk=zc)
        sim.step(6)
        out.append(sim.state.clone().cpu())
        sim.close()
    for o in out[1:]:
        assert torch.equal(o, out[0])


def test_headline_128cube_all_cells(lib):
    from paper_1601_01237_amd.sim import Sim
    say("regularized3 128^3 x 3")
    rho0 = inputs.sphere_droplet((128, 128, 128), radius=16.0, seed=0)
    p = _params((1.0, 0.6))
    sim = Sim(rho0, tau=p.tau, G=-1.0, collision=REG3)
    sim.step(3)
    compare_fields(sim, oracle_run(rho0, p, 3), p, tol=TOL, label="reg3 128")
    sim.close()


def test_reverse_step_of_the_third_order_reading(lib):
    """The third-order reading has a reverse step (its transpose is pinned in
    the oracle by complex-step derivatives; the one-step, fields, tiling and
    gradient parity tests of the adjoint run it too): one reverse step of the
    8^3 droplet matches the oracle's transpose."""
    from oracle import adjoint as oadj
    from paper_1601_01237_amd.autograd import Reverse, from_adjoint_layout, to_adjoint_layout
    from paper_1601_01237_amd.sim import Sim
    rho0 = inputs.sphere_droplet((8, 8, 8), radius=2.0, seed=1)
    sim = Sim(rho0, tau=(0.9, 0.9), G=-1.0, collision=REG3)
    sim.step(3)
    f = sim.populations().cpu().numpy().astype(np.float64)
    lam1 = np.random.default_rng(3).normal(size=f.shape).astype(np.float32)
    rev = Reverse(sim)
    lam, _ = rev.step(sim.state.clone(), to_adjoint_layout(torch.from_numpy(lam1).cuda(), sim))
    got = from_adjoint_layout(lam, sim).cpu().numpy()
    sim.close()
    p = olbm.Params(tau=(0.9, 0.9), G=((0.0, -1.0), (-1.0, 0.0)), collision=REG3)
    mu, _, _ = oadj.collide_adjoint(f, lam1.astype(np.float64), p)
    assert rel_err(got, oadj.stream_adjoint(mu)) < 1e-5
