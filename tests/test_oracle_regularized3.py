"""Pins of the oracle's third-order reading of the regularized filter (Sec. 3,
Eqs. 10-11): the non-equilibrium part is projected onto the momentum flux
(second order) and the energy flux (the contracted third-order moment), and
every other non-equilibrium moment is removed.

What the reading fixes, checked against the mathematics of the D3Q19 lattice
rather than against the oracle's formula:

* the energy-flux polynomials H^E_a = sum_{b != a} (c_a c_b^2 - T0 c_a) are
  orthogonal (w-weighted) to 1, c and c c, and their lattice norm is
  2 T0^3 = 2/27 -- half the continuum value, because the lattice has no
  velocity with three non-zero components;
* the projection has no mass or momentum, reproduces the momentum flux and
  the contracted third moment sum_b c_a c_b c_b of f - f^eq exactly (up to
  the first moment it removes), and has no non-contracted third moment;
* it is idempotent on content in its range;
* the collision keeps energy-flux content (relaxed by 1 - 1/tau, where the
  second-order reading drops it) and ignores the six-dimensional rest;
* tau = 1 gives BGK, mass and momentum are conserved (also for unequal tau),
  the shear viscosity is still T0 (tau - 1/2);
* an independent pure-Python loop agrees.
"""

import math

import numpy as np
import pytest

from oracle import lbm
from oracle.lbm import C, Q, T0, W, Params
from paper_1601_01237_amd import inputs

from . import _scalar_lbm
from .test_oracle_pins import _from_scalar, _random_state, _to_scalar

REG3 = dict(collision="regularized3")


def _moment(f, *axes):
    w = np.ones(Q)
    for a in axes:
        w = w * C[:, a]
    return np.einsum("i,i...->...", w, f)


def _energy_basis():
    """The three contracted third-order polynomials, written out per axis."""
    out = np.zeros((Q, 3))
    for a in range(3):
        for b in range(3):
            if b != a:
                out[:, a] += C[:, a] * C[:, b] ** 2 - T0 * C[:, a]
    return out


def test_energy_flux_polynomials_on_d3q19():
    he = lbm.energy_flux_hermite()
    np.testing.assert_allclose(he, _energy_basis(), rtol=0, atol=1e-15)
    # the diagonal cubic c_a^3 - 3 T0 c_a vanishes on the lattice (T0 = 1/3)
    for a in range(3):
        np.testing.assert_allclose(C[:, a] ** 3 - 3 * T0 * C[:, a], 0.0, atol=1e-15)
    # orthogonal to 1, c_b, c_b c_c and to each other
    for a in range(3):
        assert abs(np.sum(W * he[:, a])) < 1e-15
        for b in range(3):
            assert abs(np.sum(W * he[:, a] * C[:, b])) < 1e-15
            for c in range(3):
                assert abs(np.sum(W * he[:, a] * C[:, b] * C[:, c])) < 1e-15
            if b != a:
                assert abs(np.sum(W * he[:, a] * he[:, b])) < 1e-15
        # norm 2 T0^3: 8 edges with c_a != 0, (1/36) (1/3)^2 each, and 2 faces, (1/18) (2/3)^2 each
        assert abs(np.sum(W * he[:, a] ** 2) - 2.0 * T0 ** 3) < 1e-15


def test_projection_keeps_momentum_and_energy_flux():
    rng = np.random.default_rng(31)
    shape = (3, 4, 5)
    f = _random_state(shape, seed=32)
    for a in range(2):
        rho = f[a].sum(0)
        u = rng.uniform(-0.1, 0.1, size=(3,) + shape)
        neq = lbm.regularized_neq(f[a], rho, u, order=3)
        d = f[a] - lbm.equilibrium(rho, u)
        np.testing.assert_allclose(_moment(neq), 0.0, atol=1e-15)
        for x in range(3):
            np.testing.assert_allclose(_moment(neq, x), 0.0, atol=1e-15)
            for y in range(3):
                np.testing.assert_allclose(_moment(neq, x, y), _moment(d, x, y), rtol=1e-12, atol=1e-15)
            # contracted third moment sum_b c_x c_b c_b: on the lattice it is
            # the energy-flux polynomial plus (1 + 2 T0) c_x, whose first
            # moment the projection removes
            q_neq = sum(_moment(neq, x, b, b) for b in range(3))
            q_d = sum(_moment(d, x, b, b) for b in range(3)) - (1 + 2 * T0) * _moment(d, x)
            np.testing.assert_allclose(q_neq, q_d, rtol=1e-12, atol=1e-15)
        # non-contracted third moments are removed
        for x, y, z in ((0, 1, 2),):
            np.testing.assert_allclose(_moment(neq, x, y, z), 0.0, atol=1e-15)
        for x, y, z in ((0, 1, 2), (1, 0, 2), (2, 0, 1)):
            np.testing.assert_allclose(_moment(neq, x, y, y) - _moment(neq, x, z, z), 0.0, atol=1e-15)
        # the second-order reading drops the energy flux, this one keeps it
        neq2 = lbm.regularized_neq(f[a], rho, u, order=2)
        assert np.abs(sum(_moment(neq - neq2, 0, b, b) for b in range(3))).max() > 1e-6


def test_projection_is_idempotent():
    rng = np.random.default_rng(33)
    shape = (2, 3, 4)
    rho = rng.uniform(0.2, 1.0, size=shape)
    u = rng.uniform(-0.1, 0.1, size=(3,) + shape)
    A = rng.normal(size=(3, 3) + shape) * 1e-3
    A = 0.5 * (A + A.transpose(1, 0, 2, 3, 4))
    qv = rng.normal(size=(3,) + shape) * 1e-3
    he = _energy_basis()
    norm = 2.0 * T0 ** 3
    content = np.empty((Q,) + shape)
    for i in range(Q):
        content[i] = W[i] * ((sum(C[i, a] * C[i, b] * A[a, b] for a in range(3) for b in range(3))
                              - T0 * (A[0, 0] + A[1, 1] + A[2, 2])) / (2 * T0 * T0)
                             + sum(he[i, a] * qv[a] for a in range(3)) / norm)
    f = lbm.equilibrium(rho, u) + content
    np.testing.assert_allclose(lbm.regularized_neq(f, rho, u, order=3), content, rtol=1e-12, atol=1e-17)


def _null_space(rows, shape, seed, count):
    rng = np.random.default_rng(seed)
    M = np.array(rows)
    _, _, vt = np.linalg.svd(M)
    null = vt[len(rows):]
    coef = rng.normal(size=(2, count) + shape) * 1e-3
    return np.einsum("kq,skzyx->sqzyx", null, coef)


def test_collision_keeps_energy_flux_and_ignores_the_rest():
    shape = (4, 3, 5)
    f = _random_state(shape, seed=34)
    he = _energy_basis()
    rows = [np.ones(Q)] + [C[:, a].astype(float) for a in range(3)]
    rows += [(C[:, a] * C[:, b]).astype(float) for a in range(3) for b in range(a, 3)]
    rest = _null_space(rows + [he[:, a] for a in range(3)], shape, seed=35, count=6)
    assert np.abs(rest).max() > 1e-4
    kw = dict(tau=(0.7, 1.3), G=((0.0, -1.2), (-0.8, 0.0)))
    p3 = Params(**kw, **REG3)
    np.testing.assert_allclose(lbm.collide(f + rest, p3), lbm.collide(f, p3), rtol=1e-12, atol=1e-15)
    # pure energy-flux content (zero density, momentum, momentum flux): kept
    # and relaxed by (1 - 1/tau); the second-order reading removes it
    rng = np.random.default_rng(36)
    qv = rng.normal(size=(2, 3) + shape) * 1e-3
    flux = np.einsum("ia,sazyx->sizyx", W[:, None] * he / (2 * T0 ** 3), qv)
    diff3 = lbm.collide(f + flux, p3) - lbm.collide(f, p3)
    for a in range(2):
        np.testing.assert_allclose(diff3[a], (1 - 1 / kw["tau"][a]) * flux[a], rtol=1e-10, atol=1e-15)
    p2 = Params(**kw, collision="regularized")
    np.testing.assert_allclose(lbm.collide(f + flux, p2), lbm.collide(f, p2), rtol=1e-12, atol=1e-15)


def test_tau_one_equals_bgk():
    f = _random_state((3, 5, 4), seed=37)
    kw = dict(tau=(1.0, 1.0), G=((0.0, -1.7), (-1.7, 0.0)))
    np.testing.assert_allclose(lbm.collide(f, Params(**kw, **REG3)), lbm.collide(f, Params(**kw)),
                               rtol=1e-13, atol=1e-16)


def test_mass_and_momentum_are_conserved_with_unequal_tau():
    rho0 = inputs.sphere_droplet((10, 12, 9), radius=3.0, seed=3)
    p = Params(tau=(0.55, 1.9), G=((0.0, -1.4), (-1.4, 0.0)), **REG3)
    f = lbm.init_state(rho0)
    m0 = lbm.species_density(f).sum(axis=(1, 2, 3))
    j0 = np.array([np.sum(C[:, a][None, :, None, None, None] * f) for a in range(3)])
    f = lbm.run(f, p, 25)
    np.testing.assert_allclose(lbm.species_density(f).sum(axis=(1, 2, 3)), m0, rtol=1e-13)
    j1 = np.array([np.sum(C[:, a][None, :, None, None, None] * f) for a in range(3)])
    np.testing.assert_allclose(j1, j0, atol=1e-12)


@pytest.mark.parametrize("walls", [False, True])
def test_brute_force_two_steps(walls):
    shape = (3, 4, 5)
    f = _random_state(shape, seed=38)
    solid = None
    solid_set = set()
    if walls:
        solid = np.zeros(shape, bool)
        solid[0, :, :] = True
        solid[2, 1, 3] = True
        f[:, :, solid] = 0.0
        solid_set = {tuple(c) for c in np.argwhere(solid)}
    p = Params(tau=(0.6, 1.7), G=((0.0, -1.1), (-0.7, 0.0)), rho_wall=(0.3, 0.1), **REG3)
    fs, idx = _to_scalar(f, shape)
    for _ in range(2):
        fs = _scalar_lbm.step(fs, shape, p.tau, p.G, solid_set, p.rho_wall, collision="regularized3")
        f = lbm.step(f, p, solid)
    np.testing.assert_allclose(f, _from_scalar(fs, shape, idx), rtol=1e-13, atol=1e-16)


def test_shear_wave_viscosity():
    L, tau = 64, 0.55
    shape = (1, L, 2)
    y = np.arange(L)
    k = 2 * math.pi / L
    u = np.zeros((3,) + shape)
    u[0] = 1e-4 * np.sin(k * y)[None, :, None]
    f = np.stack([lbm.equilibrium(0.5 * np.ones(shape), u)] * 2)
    p = Params(tau=(tau, tau), G=((0.0, 0.0), (0.0, 0.0)), **REG3)

    def amp(f):
        return 2.0 / L * np.sum(lbm.macroscopic(f, p)["u"][0][0, :, 0] * np.sin(k * y))

    f = lbm.run(f, p, 50)
    a0 = amp(f)
    f = lbm.run(f, p, 200)
    rate = -math.log(amp(f) / a0) / 200
    assert abs(rate / (T0 * (tau - 0.5) * k * k) - 1.0) < 0.005
