"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms,
conservation laws, special cases, textbook results or an independent brute-force
restatement (arXiv 1601.01237, Sec. 2 and Sec. 4).
"""

import itertools
import math

import numpy as np
import pytest

from oracle import lbm
from oracle.lbm import C, OPP, Q, T0, W, Params
from paper_1601_01237_amd import inputs

from . import _scalar_lbm


def _random_state(shape, seed, du=0.05):
    """Positive populations near equilibrium with random velocity (test input)."""
    rng = np.random.default_rng(seed)
    rho0 = 0.5 + rng.uniform(0.0, 0.5, size=(2,) + shape)
    u = rng.uniform(-du, du, size=(3,) + shape)
    f = np.stack([lbm.equilibrium(rho0[a], u) for a in range(2)])
    f = f * (1.0 + 0.02 * rng.uniform(-1.0, 1.0, size=f.shape))
    return f


# ---------------------------------------------------------------------------
# Lattice tables (Sec. 2: D3Q19 with isotropic weights, T0 = 1/3)
# ---------------------------------------------------------------------------

def test_velocity_set_is_d3q19():
    vecs = {tuple(v) for v in C}
    assert len(vecs) == 19
    expect = {v for v in itertools.product((-1, 0, 1), repeat=3) if sum(a * a for a in v) <= 2}
    assert vecs == expect
    for i in range(Q):
        assert (C[OPP[i]] == -C[i]).all()
        assert OPP[OPP[i]] == i
    # opposite directions sit next to each other after the rest particle
    for k in range(1, Q, 2):
        assert OPP[k] == k + 1


def test_weights_are_isotropic_to_fourth_order():
    assert math.isclose(W.sum(), 1.0, rel_tol=0, abs_tol=1e-15)
    for a in range(3):
        assert abs(np.sum(W * C[:, a])) < 1e-16
        for b in range(3):
            m2 = np.sum(W * C[:, a] * C[:, b])
            assert math.isclose(m2, T0 * (a == b), abs_tol=1e-15)
            for c in range(3):
                assert abs(np.sum(W * C[:, a] * C[:, b] * C[:, c])) < 1e-16
                for d in range(3):
                    m4 = np.sum(W * C[:, a] * C[:, b] * C[:, c] * C[:, d])
                    iso = T0 ** 2 * ((a == b) * (c == d) + (a == c) * (b == d) + (a == d) * (b == c))
                    assert math.isclose(m4, iso, abs_tol=1e-15)


# ---------------------------------------------------------------------------
# Eq. (3): moments of the equilibrium
# ---------------------------------------------------------------------------

def test_equilibrium_moments_closed_form():
    rng = np.random.default_rng(1)
    shape = (3, 4, 5)
    rho = rng.uniform(0.03, 1.2, size=shape)
    u = rng.uniform(-0.15, 0.15, size=(3,) + shape)
    E = lbm.equilibrium(rho, u)
    np.testing.assert_allclose(E.sum(0), rho, rtol=1e-14)
    for a in range(3):
        # the two third-order terms of Eq. (3) cancel in the first moment
        np.testing.assert_allclose(np.einsum("i,izyx->zyx", C[:, a], E), rho * u[a],
                                   rtol=1e-13, atol=1e-16)
        for b in range(3):
            m2 = np.einsum("i,i,izyx->zyx", C[:, a], C[:, b], E)
            np.testing.assert_allclose(m2, rho * (T0 * (a == b) + u[a] * u[b]),
                                       rtol=1e-13, atol=1e-16)


def test_equilibrium_at_rest_is_weight_times_density():
    rho = np.full((2, 2, 2), 0.7)
    E = lbm.equilibrium(rho, np.zeros((3, 2, 2, 2)))
    np.testing.assert_allclose(E, np.broadcast_to(W[:, None, None, None] * 0.7, E.shape), rtol=0, atol=1e-16)


# ---------------------------------------------------------------------------
# Eq. (7): Shan-Chen force, closed form on a sinusoid
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("axis", [0, 1, 2])
def test_shan_chen_force_on_sinusoid(axis):
    # rho^B = a + b sin(k s) along one axis s.  Then
    # sum_i w_i c_i rho^B(x + c_i) = T0 b sin(k) cos(k s) e_s  (sum over the
    # plane of w_i for c_is = 1 is T0/2), and F^{AB} = G rho^A times that.
    shape = [6, 7, 8]                 # nz, ny, nx
    n = shape[2 - axis]
    k = 2 * math.pi * 2 / n
    a0, b0, G = 0.4, 0.05, -1.7
    coord = np.arange(n, dtype=float)
    prof = a0 + b0 * np.sin(k * coord)
    rho_b = np.broadcast_to(
        prof.reshape([n if ax == 2 - axis else 1 for ax in range(3)]), shape).copy()
    rng = np.random.default_rng(2)
    rho_a = rng.uniform(0.1, 1.0, size=shape)
    rho_s = np.stack([rho_a, rho_b])
    fluid = np.ones(shape, bool)
    F = lbm.shan_chen_force(rho_s, ((0.0, G), (G, 0.0)), fluid, (0.0, 0.0))
    expect_prof = T0 * b0 * math.sin(k) * np.cos(k * coord)
    expect = np.broadcast_to(
        expect_prof.reshape([n if ax == 2 - axis else 1 for ax in range(3)]), shape)
    for a in range(3):
        want = G * rho_a * expect if a == axis else np.zeros(shape)
        np.testing.assert_allclose(F[0, 1, a], want, rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(F[0, 0], 0.0)
    np.testing.assert_allclose(F[1, 1], 0.0)


def test_wall_potential_force_next_to_flat_wall():
    # Fluid at z = 1 above a wall at z = 0, uniform rho^B = b everywhere else:
    # the z component of the Eq. (7) sum is (1/18 + 4/36) (b - rho_s) = (b - rho_s)/6
    shape = (6, 4, 5)
    solid = np.zeros(shape, bool)
    solid[0] = True
    b, rs, G, ra = 0.8, 0.3, -1.2, 0.25
    rho_s = np.stack([np.full(shape, ra), np.full(shape, b)])
    fluid = ~solid
    F = lbm.shan_chen_force(rho_s, ((0.0, G), (G, 0.0)), fluid, (0.1, rs))
    np.testing.assert_allclose(F[0, 1, 2][1], G * ra * (b - rs) / 6.0, rtol=1e-13)
    np.testing.assert_allclose(F[0, 1, 2][5], -G * ra * (b - rs) / 6.0, rtol=1e-13)  # below wall at z=0 (periodic)
    np.testing.assert_allclose(F[0, 1, 2][2:5], 0.0, atol=1e-16)
    np.testing.assert_allclose(F[0, 1, 0][1:], 0.0, atol=1e-16)


# ---------------------------------------------------------------------------
# Conservation laws of Eqs. (1)-(2) with the forcing term
# ---------------------------------------------------------------------------

def test_mass_is_conserved_per_species():
    rho0 = inputs.sphere_droplet((12, 10, 14), radius=3.5, seed=0)
    f = lbm.init_state(rho0)
    p = Params(tau=(0.8, 1.3), G=((0.0, -1.0), (-1.0, 0.0)))
    m0 = lbm.species_density(f).sum(axis=(1, 2, 3))
    f = lbm.run(f, p, 30)
    m1 = lbm.species_density(f).sum(axis=(1, 2, 3))
    np.testing.assert_allclose(m1, m0, rtol=1e-13)


def test_mass_is_conserved_with_walls():
    rho0, solid = inputs.inclined_channel((14, 6, 16), angle_deg=30.0, radius=4.0, seed=3)
    f = lbm.init_state(rho0, solid)
    p = Params(tau=(0.7, 0.7), G=((0.0, -1.0), (-1.0, 0.0)), rho_wall=(0.05, 0.2))
    m0 = lbm.species_density(f).sum(axis=(1, 2, 3))
    f = lbm.run(f, p, 25, solid)
    m1 = lbm.species_density(f).sum(axis=(1, 2, 3))
    np.testing.assert_allclose(m1, m0, rtol=1e-13)
    assert np.all(f[:, :, solid] == 0.0)


def _momentum(f):
    return np.array([np.sum(C[:, a][None, :, None, None, None] * f) for a in range(3)])


def test_local_momentum_gain_equals_summed_force():
    # Equal tau: collision keeps rho u per cell; the forcing term adds F^A + F^B.
    f = _random_state((5, 6, 7), seed=4)
    p = Params(tau=(0.9, 0.9), G=((0.0, -1.3), (-0.7, 0.0)))
    m = lbm.macroscopic(f, p)
    fstar = lbm.collide(f, p)
    for a in range(3):
        before = np.einsum("i,sizyx->zyx", C[:, a], f)
        after = np.einsum("i,sizyx->zyx", C[:, a], fstar)
        force = m["F"][0, 1, a] + m["F"][1, 0, a]
        np.testing.assert_allclose(after - before, force, rtol=1e-12, atol=1e-15)
    # mass of each species unchanged by collision + forcing in every cell
    np.testing.assert_allclose(lbm.species_density(fstar), lbm.species_density(f), rtol=1e-14)


def test_species_momentum_with_unequal_tau():
    # Per species: j*^a = (1 - w_a) j^a + w_a rho^a u + F^a  (omega_a = 1/tau_a).
    f = _random_state((4, 5, 6), seed=5)
    p = Params(tau=(0.6, 1.7), G=((0.0, -1.0), (-1.0, 0.0)))
    m = lbm.macroscopic(f, p)
    fstar = lbm.collide(f, p)
    for s in range(2):
        om = 1.0 / p.tau[s]
        for a in range(3):
            j = np.einsum("i,izyx->zyx", C[:, a], f[s])
            js = np.einsum("i,izyx->zyx", C[:, a], fstar[s])
            want = (1 - om) * j + om * m["rho_s"][s] * m["u"][a] + m["F"][s, 1 - s, a]
            np.testing.assert_allclose(js, want, rtol=1e-12, atol=1e-15)


def test_total_momentum_conserved_for_symmetric_G_periodic():
    rho0 = inputs.sphere_droplet((10, 12, 11), radius=3.0, seed=6)
    f = lbm.init_state(rho0)
    f = f + 0.0  # rest start: total momentum zero
    p = Params(tau=(1.2, 1.2), G=((0.0, -2.5), (-2.5, 0.0)))
    for _ in range(20):
        f = lbm.step(f, p)
    mom = _momentum(f)
    assert np.all(np.abs(mom) < 1e-13 * rho0.sum())


def test_total_momentum_of_moving_state_is_kept():
    f = _random_state((6, 5, 7), seed=7, du=0.04)
    p = Params(tau=(0.75, 0.75), G=((0.0, -1.5), (-1.5, 0.0)))
    m0 = _momentum(f)
    f = lbm.run(f, p, 10)
    np.testing.assert_allclose(_momentum(f), m0, rtol=1e-12, atol=1e-13)


def test_uniform_state_is_a_fixed_point():
    shape = (5, 6, 7)
    rho0 = np.stack([np.full(shape, 0.37), np.full(shape, 0.81)])
    f0 = lbm.init_state(rho0)
    p = Params(tau=(0.55, 1.9), G=((0.0, -3.0), (-3.0, 0.0)))
    f = lbm.run(f0, p, 5)
    np.testing.assert_allclose(f, f0, rtol=1e-14, atol=0)  # a few ulp per step


def test_tau_one_gives_equilibrium_of_shifted_velocity():
    # tau = 1 removes f from Eq. (2): the post-collision second moment is the
    # closed form rho^a (T0 I + v v) with v = u + g^a.
    f = _random_state((4, 4, 5), seed=8)
    p = Params(tau=(1.0, 1.0), G=((0.0, -1.1), (-1.1, 0.0)))
    m = lbm.macroscopic(f, p)
    fstar = lbm.collide(f, p)
    for s in range(2):
        v = m["u"] + m["g"][s]
        for a in range(3):
            for b in range(3):
                m2 = np.einsum("i,i,izyx->zyx", C[:, a], C[:, b], fstar[s])
                want = m["rho_s"][s] * (T0 * (a == b) + v[a] * v[b])
                np.testing.assert_allclose(m2, want, rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------------------
# Brute force: independent scalar restatement on tiny non-cubic grids
# ---------------------------------------------------------------------------

def _to_scalar(f, shape):
    vel, _, _ = _scalar_lbm.lattice()
    idx = [int(np.nonzero((C == np.array(v)).all(1))[0][0]) for v in vel]
    nz, ny, nx = shape
    out = [[dict() for _ in range(19)] for _ in range(2)]
    for s in range(2):
        for q, i in enumerate(idx):
            for z in range(nz):
                for y in range(ny):
                    for x in range(nx):
                        out[s][q][(z, y, x)] = float(f[s, i, z, y, x])
    return out, idx


def _from_scalar(fs, shape, idx):
    nz, ny, nx = shape
    out = np.zeros((2, 19) + shape)
    for s in range(2):
        for q, i in enumerate(idx):
            for (z, y, x), v in fs[s][q].items():
                out[s, i, z, y, x] = v
    return out


@pytest.mark.parametrize("walls", [False, True])
def test_brute_force_two_steps(walls):
    shape = (3, 4, 5)
    f = _random_state(shape, seed=9)
    solid = None
    solid_set = set()
    if walls:
        solid = np.zeros(shape, bool)
        solid[0, :, :] = True
        solid[1, 2, 3] = True
        f[:, :, solid] = 0.0
        solid_set = {tuple(c) for c in np.argwhere(solid)}
    p = Params(tau=(0.7, 1.4), G=((0.0, -1.3), (-0.9, 0.0)), rho_wall=(0.2, 0.45))
    fs, idx = _to_scalar(f, shape)
    for _ in range(2):
        fs = _scalar_lbm.step(fs, shape, p.tau, p.G, solid_set, p.rho_wall)
        f = lbm.step(f, p, solid)
    np.testing.assert_allclose(f, _from_scalar(fs, shape, idx), rtol=1e-13, atol=1e-16)


# ---------------------------------------------------------------------------
# Textbook: BGK shear viscosity nu = T0 (tau - 1/2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("tau", [0.6, 1.0, 1.5])
def test_shear_wave_decay_rate(tau):
    L = 64
    shape = (1, L, 2)
    U = 1e-4
    y = np.arange(L)
    k = 2 * math.pi / L
    u = np.zeros((3,) + shape)
    u[0] = U * np.sin(k * y)[None, :, None]
    rho = np.ones(shape)
    f = np.stack([lbm.equilibrium(0.5 * rho, u), lbm.equilibrium(0.5 * rho, u)])
    p = Params(tau=(tau, tau), G=((0.0, 0.0), (0.0, 0.0)))
    steps = 200

    def amp(f):
        m = lbm.macroscopic(f, p)
        return 2.0 / L * np.sum(m["u"][0][0, :, 0] * np.sin(k * y))

    # skip the transient of the equilibrium start (no initial shear stress)
    f = lbm.run(f, p, 50)
    a0 = amp(f)
    f = lbm.run(f, p, steps)
    rate = -math.log(amp(f) / a0) / steps
    nu = T0 * (tau - 0.5)
    # BGK gives nu = T0 (tau - 1/2) up to O(k^2) lattice corrections (< 0.3 % at L = 64)
    assert abs(rate / (nu * k * k) - 1.0) < 0.005


def test_channel_mode_decay_with_halfway_bounce_back():
    # Walls at z = 0 and z = H+1; fluid layers z = 1..H; halfway walls sit at
    # z = 1/2 and z = H + 1/2, so u_x = U sin(pi (z - 1/2) / H) decays at nu (pi/H)^2.
    H = 24
    shape = (H + 2, 1, 2)
    solid = np.zeros(shape, bool)
    solid[0] = True
    solid[-1] = True
    tau = 0.8
    z = np.arange(H + 2)
    prof = np.where((z >= 1) & (z <= H), np.sin(math.pi * (z - 0.5) / H), 0.0)
    u = np.zeros((3,) + shape)
    u[0] = 1e-4 * prof[:, None, None]
    rho = np.ones(shape)
    f = np.stack([lbm.equilibrium(0.5 * rho, u), lbm.equilibrium(0.5 * rho, u)])
    f[:, :, solid] = 0.0
    p = Params(tau=(tau, tau), G=((0.0, 0.0), (0.0, 0.0)))

    def amp(f):
        m = lbm.macroscopic(f, p, solid)
        return np.sum(m["u"][0][:, 0, 0] * prof)

    a0 = amp(f)
    steps = 300
    f = lbm.run(f, p, steps, solid)
    rate = -math.log(amp(f) / a0) / steps
    nu = T0 * (tau - 0.5)
    assert abs(rate / (nu * (math.pi / H) ** 2) - 1.0) < 0.02


def test_closed_channel_at_rest_is_a_fixed_point():
    shape = (8, 3, 4)
    solid = np.zeros(shape, bool)
    solid[0] = True
    solid[-1] = True
    rho0 = np.stack([np.full(shape, 0.6), np.full(shape, 0.4)])
    rho0[:, solid] = 0.0
    f0 = lbm.init_state(rho0, solid)
    p = Params(tau=(0.9, 0.9), G=((0.0, 0.0), (0.0, 0.0)))
    f = lbm.run(f0, p, 4, solid)
    np.testing.assert_allclose(f, f0, rtol=1e-15, atol=1e-17)


# ---------------------------------------------------------------------------
# Symmetries
# ---------------------------------------------------------------------------

def test_translation_equivariance():
    rho0 = inputs.sphere_droplet((8, 9, 10), radius=2.5, seed=10)
    p = Params(tau=(0.8, 0.8), G=((0.0, -1.5), (-1.5, 0.0)))
    f = lbm.run(lbm.init_state(rho0), p, 6)
    shifted = np.roll(rho0, shift=(1, -2, 3), axis=(1, 2, 3))
    g = lbm.run(lbm.init_state(shifted), p, 6)
    np.testing.assert_allclose(g, np.roll(f, shift=(1, -2, 3), axis=(2, 3, 4)), rtol=1e-13, atol=1e-17)


def test_axis_permutation_equivariance():
    f = _random_state((5, 6, 7), seed=11)
    p = Params(tau=(0.7, 1.1), G=((0.0, -1.2), (-0.8, 0.0)))
    g = lbm.run(f, p, 3)
    # swap x <-> z: spatial axes (z, y, x) -> (x, y, z), velocity (cx, cy, cz) -> (cz, cy, cx)
    perm = [int(np.nonzero((C == C[i][[2, 1, 0]]).all(1))[0][0]) for i in range(Q)]
    fp = np.transpose(f, (0, 1, 4, 3, 2))[:, perm]
    gp = lbm.run(fp, p, 3)
    np.testing.assert_allclose(gp, np.transpose(g, (0, 1, 4, 3, 2))[:, perm], rtol=1e-12, atol=1e-16)


def test_species_swap_equivariance():
    f = _random_state((4, 5, 6), seed=12)
    p = Params(tau=(0.7, 1.1), G=((0.0, -1.2), (-0.8, 0.0)), rho_wall=(0.1, 0.3))
    q = Params(tau=(1.1, 0.7), G=((0.0, -0.8), (-1.2, 0.0)), rho_wall=(0.3, 0.1))
    g = lbm.run(f, p, 3)
    h = lbm.run(f[::-1].copy(), q, 3)
    np.testing.assert_allclose(h, g[::-1], rtol=1e-13, atol=1e-17)


# ---------------------------------------------------------------------------
# Eqs. (8)-(9): force velocity
# ---------------------------------------------------------------------------

def test_force_velocity_is_mean_of_pre_and_post_collision_velocity():
    f = _random_state((4, 5, 6), seed=13)
    p = Params(tau=(0.85, 0.85), G=((0.0, -1.4), (-1.4, 0.0)))
    m = lbm.macroscopic(f, p)
    fstar = lbm.collide(f, p)
    rho = m["rho"]
    post = np.stack([np.einsum("i,sizyx->zyx", C[:, a], fstar) for a in range(3)]) / rho
    uF = lbm.force_velocity(f, p)
    np.testing.assert_allclose(uF, 0.5 * (m["u"] + post), rtol=1e-12, atol=1e-16)


# ---------------------------------------------------------------------------
# Storage emulation against library conversions
# ---------------------------------------------------------------------------

def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(14)
    x = rng.normal(size=4096) * 10.0 ** rng.integers(-6, 2, size=4096)
    want = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(lbm._round_bf16(x), want)


def test_fp16_storage_round_trip_bound():
    rng = np.random.default_rng(15)
    fstar = rng.uniform(0.0, 0.4, size=(2, 19, 2, 3, 4))
    shift = (0.3, 0.6)
    r = lbm.round_storage(fstar, "fp16", shift)
    dev = np.abs(fstar - W[None, :, None, None, None] * np.array(shift)[:, None, None, None, None])
    # moving populations, round to nearest: at most half an fp16 ulp of the
    # stored deviation
    assert np.all(np.abs(r - fstar)[:, 1:] <= dev[:, 1:] * 2.0 ** -11 + 2.0 ** -25)
    # rest population absorbs the others' rounding, kept as a stored value
    # plus a stored residual: the decoded populations sum to the density up
    # to the rounding of that residual, itself at most half an ulp of half an
    # ulp of the rest deviation (2^-11 * 2^-11)
    rest_dev = np.abs(r[:, 0] - W[0] * np.array(shift)[:, None, None, None])
    rho = fstar.sum(axis=1)
    err = np.abs(r.sum(axis=1) - rho)
    assert np.all(err <= rest_dev * 2.0 ** -21 + 1e-15)
    # far below a single rounding of the rest value
    assert err.max() < 1e-3 * (rest_dev * 2.0 ** -11).max()
    # the same for BF16 (unit roundoff 2^-8 each)
    rb = lbm.round_storage(fstar, "bf16", shift)
    rest_b = np.abs(rb[:, 0] - W[0] * np.array(shift)[:, None, None, None])
    assert np.all(np.abs(rb.sum(axis=1) - rho) <= rest_b * 2.0 ** -15 + 1e-15)
