"""GPU parity of the fused step against the FP64 oracle (through the C ABI).

Tolerance (FP32 storage and arithmetic): 1e-5 of the field's maximum for
rho^A, rho^B, u_F and all 38 populations.
"""

import numpy as np
import pytest
import torch

from oracle import lbm as olbm
from paper_1601_01237_amd import inputs

from ._gpu_util import compare_fields, oracle_diag, oracle_run, rel_err, say

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _sim(rho0, p, **kw):
    from paper_1601_01237_amd.sim import Sim
    return Sim(rho0, tau=p.tau, G=p.G, rho_wall=p.rho_wall, **kw)


def test_rest_state_after_init(lib):
    say("init 32^3")
    rho0 = inputs.sphere_droplet((32, 32, 32), radius=8.0, seed=0)
    p = olbm.Params(tau=(1.0, 1.0), G=((0.0, -1.0), (-1.0, 0.0)))
    sim = _sim(rho0, p)
    f = sim.populations().cpu().numpy()
    want = olbm.init_state(rho0)
    e_pop = rel_err(f, want)
    assert e_pop < 1e-7, e_pop           # one FP32 rounding of w_i rho0
    rho, uf, diag = sim.moments()
    e_rho = rel_err(rho.cpu().numpy(), rho0)
    assert e_rho < 1e-6, e_rho           # FP32 sum of 19 rounded populations
    # u = 0 at rest, but u_F = u + g/2 carries the Shan-Chen force of the
    # sharp initial interface (Eqs. 7-9)
    _, uf_ref = olbm.observables(want, p)
    e_u = rel_err(uf.cpu().numpy(), uf_ref)
    assert e_u < 1e-5, e_u
    sim.close()


@pytest.mark.parametrize("steps", [1, 10])
def test_c1_droplet_32cube(lib, steps):
    say(f"c1 32^3 steps={steps}")
    rho0 = inputs.sphere_droplet((32, 32, 32), radius=8.0, seed=0)
    p = olbm.Params(tau=(1.0, 1.0), G=((0.0, -1.0), (-1.0, 0.0)))
    sim = _sim(rho0, p)
    sim.step(steps)
    f_ref = oracle_run(rho0, p, steps)
    errs, diag = compare_fields(sim, f_ref, p, tol=TOL, label=f"c1 {steps}")
    d_ref = oracle_diag(f_ref, p)
    v = diag["vector"]
    # masses in FP64 on both sides: the GPU sums FP32 densities
    assert abs(v[0] - d_ref[0]) <= 1e-6 * d_ref[0]
    assert abs(v[1] - d_ref[1]) <= 1e-6 * d_ref[1]
    assert abs(v[5] - d_ref[5]) <= 1e-4 * d_ref[5]
    assert v[6] == 0 and v[7] == 32 ** 3
    sim.close()


@pytest.mark.parametrize("shape,tile", [((11, 13, 70), 0), ((3, 4, 5), 0), ((2, 1, 3), 0), ((9, 17, 130), 0),
                                        ((11, 29, 70), 1), ((11, 29, 70), 2), ((11, 29, 70), 3),
                                        ((11, 29, 70), 4), ((5, 3, 40), 2), ((11, 29, 300), 5),
                                        ((6, 7, 130), 3)])
def test_ragged_grids(lib, shape, tile):
    say(f"ragged {shape} tile {tile}")
    rng = np.random.default_rng(3)
    rho0 = 0.3 + rng.uniform(0.0, 0.7, size=(2,) + shape)
    p = olbm.Params(tau=(0.7, 1.3), G=((0.0, -1.6), (-0.9, 0.0)))
    sim = _sim(rho0, p, tile=tile)
    sim.step(4)
    f_ref = oracle_run(rho0, p, 4)
    compare_fields(sim, f_ref, p, tol=TOL, label=str(shape))
    sim.close()


def test_nonequilibrium_start_via_set_populations(lib):
    say("set_populations 12x10x14")
    shape = (12, 10, 14)
    rng = np.random.default_rng(4)
    rho = 0.4 + rng.uniform(0.0, 0.6, size=(2,) + shape)
    u = rng.uniform(-0.05, 0.05, size=(3,) + shape)
    f0 = np.stack([olbm.equilibrium(rho[a], u) for a in range(2)])
    f0 = f0 * (1.0 + 0.02 * rng.uniform(-1, 1, size=f0.shape))
    f0 = f0.astype(np.float32).astype(np.float64)
    p = olbm.Params(tau=(0.8, 0.6), G=((0.0, -2.0), (-2.0, 0.0)))
    sim = _sim(rho, p)
    sim.set_populations(torch.from_numpy(f0.astype(np.float32)))
    got = sim.populations().cpu().numpy()
    np.testing.assert_array_equal(got, f0.astype(np.float32))
    sim.step(3)
    f_ref = olbm.run(f0, p, 3)
    compare_fields(sim, f_ref, p, tol=TOL, label="noneq")
    sim.close()


def test_walls_inclined_channel(lib):
    say("walls 14x6x16")
    shape = (14, 6, 16)
    rho0, solid = inputs.inclined_channel(shape, angle_deg=30.0, radius=4.0, seed=3)
    p = olbm.Params(tau=(0.7, 0.7), G=((0.0, -1.0), (-1.0, 0.0)), rho_wall=(0.05, 0.2))
    sim = _sim(rho0, p, solid=solid)
    assert sim.wall_classes() > 2  # the marches read one-byte wall classes
    sim.step(6)
    f_ref = oracle_run(rho0, p, 6, solid)
    compare_fields(sim, f_ref, p, solid=solid, tol=TOL, label="walls")
    d = sim.moments()[2]["vector"]
    d_ref = oracle_diag(f_ref, p, solid)
    assert d[7] == d_ref[7]
    assert abs(d[0] - d_ref[0]) <= 1e-6 * d_ref[0]
    sim.close()


def test_walls_ragged_with_obstacle(lib):
    say("walls ragged 7x9x67")
    shape = (7, 9, 67)
    rng = np.random.default_rng(5)
    rho0 = 0.3 + rng.uniform(0.0, 0.7, size=(2,) + shape)
    solid = np.zeros(shape, bool)
    solid[0] = True
    solid[3, 2:5, 10:20] = True
    solid[:, 7, 66] = True
    rho0[:, solid] = 0.0
    p = olbm.Params(tau=(0.9, 1.2), G=((0.0, -1.3), (-1.1, 0.0)), rho_wall=(0.3, 0.1))
    sim = _sim(rho0, p, solid=solid)
    sim.step(5)
    f_ref = oracle_run(rho0, p, 5, solid)
    compare_fields(sim, f_ref, p, solid=solid, tol=TOL, label="walls ragged")
    sim.close()


def _wall_classes_expected(solid):
    """Classes the library should keep for a geometry: the fluid cells' link
    words (bit i: x - c_i is a wall cell), their distinct nonzero values plus
    the class of the fluid cells away from walls and that of the wall cells,
    or 0 beyond 256.  The count does not depend on the order of the bits."""
    words = np.zeros(solid.shape, np.int64)
    for i in range(1, olbm.Q):
        words |= olbm.at_offset(solid, -olbm.C[i]).astype(np.int64) << i
    fluid_words = np.unique(words[~solid])
    n = 2 + int(np.count_nonzero(fluid_words))
    return n if n <= 256 else 0


@pytest.mark.parametrize("collision", ["bgk", "regularized", "regularized3"])
@pytest.mark.parametrize("fill,expect_classes", [(0.01, True), (0.3, False)])
def test_walls_porous_classes_and_words(lib, fill, expect_classes, collision):
    """Random porous media: a sparse one keeps the one-byte wall classes
    (173 of them: class bytes above 127 too), a dense one has too many
    distinct link words and the marches read the words; both match the
    oracle, with each collision operator."""
    say(f"walls porous fill={fill} {collision}")
    shape = (18, 13, 70)
    rng = np.random.default_rng(21)
    solid = rng.uniform(size=shape) < fill
    solid[0] = True
    rho0 = 0.3 + rng.uniform(0.0, 0.7, size=(2,) + shape)
    rho0[:, solid] = 0.0
    p = olbm.Params(tau=(0.9, 1.1), G=((0.0, -1.2), (-1.2, 0.0)), rho_wall=(0.2, 0.3), collision=collision)
    sim = _sim(rho0, p, solid=solid, collision=collision)
    want = _wall_classes_expected(solid)
    assert sim.wall_classes() == want
    assert (want > 2) == expect_classes
    sim.step(4)
    f_ref = oracle_run(rho0, p, 4, solid)
    compare_fields(sim, f_ref, p, solid=solid, tol=TOL, label=f"porous {fill} {collision}")
    sim.close()


@pytest.mark.parametrize("case", ["all_solid", "one_cell", "slab"])
def test_walls_degenerate_geometries(lib, case):
    """A grid with no fluid cell, one fluid cell enclosed by walls (it keeps
    its populations by bounce-back and feels no net wall force), and a fluid
    layer one cell thick between walls."""
    say(f"walls degenerate {case}")
    shape = (6, 9, 70)
    rng = np.random.default_rng(31)
    solid = np.ones(shape, bool)
    if case == "one_cell":
        solid[3, 4, 40] = False
    elif case == "slab":
        solid[3] = False
    rho0 = np.where(solid, 0.0, 0.3 + rng.uniform(0.0, 0.7, size=(2,) + shape))
    p = olbm.Params(tau=(0.8, 1.1), G=((0.0, -1.5), (-1.5, 0.0)), rho_wall=(0.2, 0.3))
    sim = _sim(rho0, p, solid=solid)
    assert sim.wall_classes() == _wall_classes_expected(solid) == (2 if case == "all_solid" else 3)
    sim.step(5)
    f_ref = oracle_run(rho0, p, 5, solid)
    _, diag = compare_fields(sim, f_ref, p, solid=solid, tol=TOL, label=case)
    assert diag["vector"][7] == np.count_nonzero(~solid)
    if case == "one_cell":
        np.testing.assert_allclose(sim.moments()[0].cpu().numpy()[:, 3, 4, 40], rho0[:, 3, 4, 40], rtol=1e-6)
    sim.close()


def _state_after(rho0, p, steps, tile, zchunk, solid=None, place=(0, -1)):
    sim = _sim(rho0, p, solid=solid)
    sim.set_tiling(tile, zchunk)
    sim.set_placement(*place)
    sim.step(steps)
    x = sim.state.clone().cpu()
    sim.close()
    return x


@pytest.mark.parametrize("walls", [False, True])
def test_tiling_invariance_bitwise(lib, walls):
    say(f"tiling invariance walls={walls}")
    shape = (20, 19, 70)
    rho0 = inputs.sphere_droplet(shape, radius=5.0, seed=6)
    solid = None
    if walls:
        solid = np.zeros(shape, bool)
        solid[0] = True
        solid[10, 3:9, 20:40] = True
        rho0[:, solid] = 0.0
    p = olbm.Params(tau=(0.8, 0.8), G=((0.0, -1.5), (-1.5, 0.0)), rho_wall=(0.1, 0.2))
    ref = _state_after(rho0, p, 7, -1, 0, solid)
    for tile, zc in [(0, 0), (4, 0), (0, 1), (1, 3), (2, 20), (3, 7), (2, 2), (4, 5), (5, 0), (5, 3), (3, 1)]:
        got = _state_after(rho0, p, 7, tile, zc, solid)
        diff = float((got - ref).abs().max())
        assert torch.equal(got, ref), (tile, zc, diff)
    # every block order and x shifts of the tile grid (lbm_set_placement),
    # on ragged tiles and chunks
    for place, tile, zc in [((1, 0), 0, 3), ((2, 5), 1, 7), ((3, 16), 3, 0), ((4, 69), 2, 5), ((2, 1), 5, 1),
                            ((4, 33), 4, 20), ((0, 16), 0, 0), ((1, 63), 1, 2)]:
        got = _state_after(rho0, p, 7, tile, zc, solid, place=place)
        assert torch.equal(got, ref), (place, tile, zc)


def test_run_to_run_determinism(lib):
    say("determinism 48^3")
    rho0 = inputs.sphere_droplet((48, 48, 48), radius=12.0, seed=7)
    p = olbm.Params(tau=(1.0, 1.0), G=((0.0, -1.0), (-1.0, 0.0)))
    a = _state_after(rho0, p, 20, -1, 0)
    b = _state_after(rho0, p, 20, -1, 0)
    assert torch.equal(a, b)


def test_translation_equivariance_bitwise(lib):
    say("translation 24x20x66")
    shape = (24, 20, 66)
    rho0 = inputs.sphere_droplet(shape, radius=6.0, seed=8)
    p = olbm.Params(tau=(0.9, 0.9), G=((0.0, -1.2), (-1.2, 0.0)))
    from paper_1601_01237_amd.sim import Sim
    s1 = Sim(rho0, tau=p.tau, G=p.G)
    s1.step(9)
    f1 = s1.populations().cpu()
    s1.close()
    s2 = Sim(np.roll(rho0, shift=(1, 1, 1), axis=(1, 2, 3)), tau=p.tau, G=p.G)
    s2.step(9)
    f2 = s2.populations().cpu()
    s2.close()
    assert torch.equal(torch.roll(f1, shifts=(1, 1, 1), dims=(2, 3, 4)), f2)


def test_checkpoint_resume_bitwise(lib):
    say("checkpoint 32^3")
    rho0 = inputs.sphere_droplet((32, 32, 32), radius=8.0, seed=9)
    p = olbm.Params(tau=(1.0, 1.0), G=((0.0, -1.0), (-1.0, 0.0)))
    from paper_1601_01237_amd.sim import Sim
    s = Sim(rho0, tau=p.tau, G=p.G)
    s.step(10)
    ck = s.checkpoint()
    s.step(10)
    ref = s.state.clone()
    s.restore(ck)
    s.step(10)
    assert s.t == 20
    assert torch.equal(s.state, ref)
    s.close()


@pytest.mark.parametrize("storage,shape", [("fp32", (5, 9, 130)), ("fp16", (3, 7, 70)), ("fp32", (17, 4, 128)),
                                           ("fp32", (3, 2, 40))])
def test_march_copy_reference(lib, storage, shape):
    """lbm_march_copy (the bandwidth reference with the step's access
    pattern) copies every cell of every population plane (and, in the 16-bit
    forms, of the two residual rows) and nothing else."""
    import ctypes
    import torch
    from paper_1601_01237_amd.sim import Sim
    say(f"march copy {storage} {shape}")
    sim = Sim(inputs.sphere_droplet(shape, radius=2.0, seed=1), storage=storage)
    sim.step(2)
    src = sim.state
    dst = torch.full_like(src, 7.0)
    code = sim.lib.lbm_march_copy(sim.ctx, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()))
    assert code == 0
    torch.cuda.synchronize()
    live = sim.live_mask()
    assert int(live.sum()) == sim.layout[2] * sim.n
    assert sim.layout[2] == (38 if storage == "fp32" else 40)
    assert torch.equal(dst[live], src[live])
    assert bool((dst[~live] == 7.0).all())  # padding untouched
    assert sim.lib.lbm_march_copy(sim.ctx, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(src.data_ptr())) != 0
    sim.close()
