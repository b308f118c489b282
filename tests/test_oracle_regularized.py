"""Pins of the oracle's regularized collision (Sec. 3, Eqs. 10-11).

The paper names the operator (a Hermite filter that keeps the non-equilibrium
momentum flux and drops higher non-equilibrium moments) and delegates its
formula to citations; the oracle reads Phi as the second-order Hermite
projection.  What that reading fixes, checked here against the mathematics
rather than against the oracle's own formula:

* the projected f^neq has no mass or momentum and reproduces the
  non-equilibrium momentum flux exactly (fourth-order isotropy of D3Q19);
* it is a projection: applied to a state whose non-equilibrium part is already
  second-order Hermite, it returns that part unchanged;
* the collision does not see non-equilibrium content outside the first three
  moments (it "removes other higher order nonequilibrium moments");
* at tau = 1 it coincides with BGK; mass and momentum are conserved; the
  shear viscosity is still T0 (tau - 1/2);
* an independent pure-Python pull-form loop agrees.
"""

import math

import numpy as np
import pytest

from oracle import lbm
from oracle.lbm import C, Q, T0, W, Params
from paper_1601_01237_amd import inputs

from . import _scalar_lbm
from .test_oracle_pins import _from_scalar, _random_state, _to_scalar

REG = dict(collision="regularized")


def _moment(f, *axes):
    w = np.ones(Q)
    for a in axes:
        w = w * C[:, a]
    return np.einsum("i,i...->...", w, f)


def test_projection_keeps_exactly_the_momentum_flux():
    rng = np.random.default_rng(21)
    shape = (3, 4, 5)
    f = _random_state(shape, seed=22)
    for a in range(2):
        rho = f[a].sum(0)
        u = rng.uniform(-0.1, 0.1, size=(3,) + shape)
        neq = lbm.regularized_neq(f[a], rho, u)
        d = f[a] - lbm.equilibrium(rho, u)
        np.testing.assert_allclose(_moment(neq), 0.0, atol=1e-15)
        for x in range(3):
            np.testing.assert_allclose(_moment(neq, x), 0.0, atol=1e-15)
            for y in range(3):
                # second moment of the projection = second moment of f - f^eq
                np.testing.assert_allclose(_moment(neq, x, y), _moment(d, x, y), rtol=1e-12, atol=1e-15)
                for z in range(3):
                    np.testing.assert_allclose(_moment(neq, x, y, z), 0.0, atol=1e-15)


def test_projection_is_idempotent():
    rng = np.random.default_rng(23)
    shape = (2, 3, 4)
    rho = rng.uniform(0.2, 1.0, size=shape)
    u = rng.uniform(-0.1, 0.1, size=(3,) + shape)
    A = rng.normal(size=(3, 3) + shape) * 1e-3
    A = 0.5 * (A + A.transpose(1, 0, 2, 3, 4))
    # a non-equilibrium part that already lies in the second-order Hermite space
    herm = np.empty((Q,) + shape)
    for i in range(Q):
        herm[i] = W[i] * (sum(C[i, a] * C[i, b] * A[a, b] for a in range(3) for b in range(3))
                          - T0 * (A[0, 0] + A[1, 1] + A[2, 2])) / (2 * T0 * T0)
    f = lbm.equilibrium(rho, u) + herm
    np.testing.assert_allclose(lbm.regularized_neq(f, rho, u), herm, rtol=1e-12, atol=1e-17)


def _ghost(shape, seed):
    """Random populations with zero density, momentum and momentum flux per cell."""
    rng = np.random.default_rng(seed)
    rows = [np.ones(Q)] + [C[:, a].astype(float) for a in range(3)]
    rows += [(C[:, a] * C[:, b]).astype(float) for a in range(3) for b in range(a, 3)]
    M = np.array(rows)                       # 10 x 19
    _, _, vt = np.linalg.svd(M)
    null = vt[10:]                           # 9 x 19 basis of the null space
    coef = rng.normal(size=(2, 9) + shape) * 1e-3
    return np.einsum("kq,skzyx->sqzyx", null, coef)


def test_collision_ignores_higher_order_nonequilibrium():
    shape = (4, 3, 5)
    f = _random_state(shape, seed=24)
    ghost = _ghost(shape, seed=25)
    assert np.abs(ghost).max() > 1e-4
    p = Params(tau=(0.7, 1.3), G=((0.0, -1.2), (-0.8, 0.0)), **REG)
    np.testing.assert_allclose(lbm.collide(f + ghost, p), lbm.collide(f, p), rtol=1e-12, atol=1e-15)
    # BGK keeps the ghost content, relaxed by (1 - 1/tau)
    pb = Params(tau=(0.7, 1.3), G=((0.0, -1.2), (-0.8, 0.0)))
    diff = lbm.collide(f + ghost, pb) - lbm.collide(f, pb)
    for a in range(2):
        np.testing.assert_allclose(diff[a], (1 - 1 / pb.tau[a]) * ghost[a], rtol=1e-10, atol=1e-15)


def test_tau_one_equals_bgk():
    f = _random_state((3, 5, 4), seed=26)
    kw = dict(tau=(1.0, 1.0), G=((0.0, -1.7), (-1.7, 0.0)))
    np.testing.assert_allclose(lbm.collide(f, Params(**kw, **REG)), lbm.collide(f, Params(**kw)),
                               rtol=1e-13, atol=1e-16)


def test_mass_and_momentum_are_conserved():
    rho0 = inputs.sphere_droplet((10, 12, 9), radius=3.0, seed=3)
    p = Params(tau=(0.55, 0.55), G=((0.0, -1.4), (-1.4, 0.0)), **REG)
    f = lbm.init_state(rho0)
    m0 = lbm.species_density(f).sum(axis=(1, 2, 3))
    j0 = np.array([np.sum(C[:, a][None, :, None, None, None] * f) for a in range(3)])
    f = lbm.run(f, p, 25)
    m1 = lbm.species_density(f).sum(axis=(1, 2, 3))
    j1 = np.array([np.sum(C[:, a][None, :, None, None, None] * f) for a in range(3)])
    np.testing.assert_allclose(m1, m0, rtol=1e-13)
    np.testing.assert_allclose(j1, j0, atol=1e-12)


def test_mass_is_conserved_with_walls():
    rho0, solid = inputs.inclined_channel((12, 6, 14), angle_deg=30.0, radius=3.5, seed=5)
    p = Params(tau=(0.6, 1.2), G=((0.0, -1.0), (-1.0, 0.0)), rho_wall=(0.05, 0.2), **REG)
    f = lbm.init_state(rho0, solid)
    m0 = lbm.species_density(f).sum(axis=(1, 2, 3))
    f = lbm.run(f, p, 20, solid)
    np.testing.assert_allclose(lbm.species_density(f).sum(axis=(1, 2, 3)), m0, rtol=1e-13)


@pytest.mark.parametrize("walls", [False, True])
def test_brute_force_two_steps(walls):
    shape = (3, 4, 5)
    f = _random_state(shape, seed=27)
    solid = None
    solid_set = set()
    if walls:
        solid = np.zeros(shape, bool)
        solid[0, :, :] = True
        solid[2, 1, 3] = True
        f[:, :, solid] = 0.0
        solid_set = {tuple(c) for c in np.argwhere(solid)}
    p = Params(tau=(0.6, 1.7), G=((0.0, -1.1), (-0.7, 0.0)), rho_wall=(0.3, 0.1), **REG)
    fs, idx = _to_scalar(f, shape)
    for _ in range(2):
        fs = _scalar_lbm.step(fs, shape, p.tau, p.G, solid_set, p.rho_wall, collision="regularized")
        f = lbm.step(f, p, solid)
    np.testing.assert_allclose(f, _from_scalar(fs, shape, idx), rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("tau", [0.55, 1.0])
def test_shear_wave_viscosity(tau):
    L = 64
    shape = (1, L, 2)
    y = np.arange(L)
    k = 2 * math.pi / L
    u = np.zeros((3,) + shape)
    u[0] = 1e-4 * np.sin(k * y)[None, :, None]
    f = np.stack([lbm.equilibrium(0.5 * np.ones(shape), u)] * 2)
    p = Params(tau=(tau, tau), G=((0.0, 0.0), (0.0, 0.0)), **REG)

    def amp(f):
        return 2.0 / L * np.sum(lbm.macroscopic(f, p)["u"][0][0, :, 0] * np.sin(k * y))

    f = lbm.run(f, p, 50)
    a0 = amp(f)
    f = lbm.run(f, p, 200)
    rate = -math.log(amp(f) / a0) / 200
    assert abs(rate / (T0 * (tau - 0.5) * k * k) - 1.0) < 0.005


def test_unequal_tau_momentum():
    """The projected non-equilibrium part carries no momentum, so with
    tau_A != tau_B the regularized collision still changes the total momentum
    of a cell by exactly F^A + F^B; BGK relaxes each species' momentum at its
    own rate and does not."""
    f = _random_state((4, 5, 3), seed=28)
    kw = dict(tau=(0.6, 2.5), G=((0.0, -1.1), (-1.1, 0.0)))
    for collision, conserves in (("regularized", True), ("bgk", False)):
        p = Params(collision=collision, **kw)
        m = lbm.macroscopic(f, p)
        fstar = lbm.collide(f, p)
        for a in range(3):
            before = np.einsum("i,sizyx->zyx", C[:, a], f)
            after = np.einsum("i,sizyx->zyx", C[:, a], fstar)
            err = np.abs(after - before - (m["F"][0, 1, a] + m["F"][1, 0, a])).max()
            if conserves:
                assert err < 1e-15, err
            else:
                assert err > 1e-6, err
