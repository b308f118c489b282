"""Pins of the oracle's hand-written adjoint against the forward oracle.

The forward map is complex-analytic, so complex-step derivatives
(Im L(p + i h) / h, h = 1e-30) give its exact tangent to rounding; the adjoint
must reproduce them (dot-product test) and agree with central differences.
"""

import numpy as np
import pytest

from oracle import adjoint, lbm
from oracle.lbm import Params
from paper_1601_01237_amd import inputs

H_CS = 1e-30


def _state(shape, seed, solid=None):
    rng = np.random.default_rng(seed)
    rho0 = 0.4 + rng.uniform(0.0, 0.6, size=(2,) + shape)
    u = rng.uniform(-0.05, 0.05, size=(3,) + shape)
    f = np.stack([lbm.equilibrium(rho0[a], u) for a in range(2)])
    f = f * (1.0 + 0.02 * rng.uniform(-1.0, 1.0, size=f.shape))
    if solid is not None:
        f[:, :, solid] = 0.0
    return f


def _walls(shape):
    solid = np.zeros(shape, bool)
    solid[0] = True
    solid[2, 1, 2] = True
    return solid


@pytest.mark.parametrize("collision", ["bgk", "regularized", "regularized3"])
@pytest.mark.parametrize("walls", [False, True])
def test_one_step_dot_product(walls, collision):
    shape = (5, 4, 6)
    solid = _walls(shape) if walls else None
    f = _state(shape, 1, solid)
    p = Params(tau=(0.7, 1.3), G=((0.0, -1.4), (-0.6, 0.0)), rho_wall=(0.15, 0.35), collision=collision)
    rng = np.random.default_rng(2)
    v = rng.normal(size=f.shape)
    w = rng.normal(size=f.shape)
    if solid is not None:
        v[:, :, solid] = 0.0
        w[:, :, solid] = 0.0
    jv = lbm.step(f + 1j * H_CS * v, p, solid).imag / H_CS
    jtw, _, _ = adjoint.step_adjoint(f, w, p, solid)
    lhs = np.sum(jv * w)
    rhs = np.sum(v * jtw)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("collision", ["bgk", "regularized", "regularized3"])
@pytest.mark.parametrize("walls", [False, True])
def test_one_step_parameter_derivatives(walls, collision):
    shape = (4, 5, 6)
    solid = _walls(shape) if walls else None
    f = _state(shape, 3, solid)
    tau, G = (0.8, 1.2), ((0.0, -1.3), (-0.9, 0.0))
    p = Params(tau=tau, G=G, rho_wall=(0.1, 0.2), collision=collision)
    w = np.random.default_rng(4).normal(size=f.shape)
    _, dG, dtau = adjoint.step_adjoint(f, w, p, solid)

    def L(pp):
        return np.sum(lbm.step(f.astype(complex), pp, solid) * w)

    for (a, b) in ((0, 1), (1, 0)):
        Gc = [list(r) for r in G]
        Gc[a][b] = G[a][b] + 1j * H_CS
        cs = L(Params(tau=tau, G=Gc, rho_wall=p.rho_wall, collision=collision)).imag / H_CS
        assert abs(dG[a, b] - cs) <= 1e-12 * abs(cs)
    for a in range(2):
        tc = list(tau)
        tc[a] = tau[a] + 1j * H_CS
        cs = L(Params(tau=tuple(tc), G=G, rho_wall=p.rho_wall, collision=collision)).imag / H_CS
        assert abs(dtau[a] - cs) <= 1e-12 * abs(cs)


def _calibration_case(n=6, steps=12):
    rho0 = inputs.sphere_droplet((n, n, n), radius=n / 4.0, seed=5)
    target = inputs.target_ellipsoid((n, n, n), radius=n / 4.0, seed=6)
    return rho0, target, steps


def test_full_sweep_against_complex_step():
    rho0, target, steps = _calibration_case()
    G, tau = -1.0, 1.0
    p = Params(tau=(tau, tau), G=((0.0, G), (G, 0.0)))
    L, dG, dtau, drho0 = adjoint.loss_and_gradient(rho0, p, steps, target)
    assert L > 0
    Gc = G + 1j * H_CS
    cs_G = adjoint.loss(rho0, Params(tau=(tau, tau), G=((0.0, Gc), (Gc, 0.0))), steps, target).imag / H_CS
    tc = tau + 1j * H_CS
    cs_t = adjoint.loss(rho0, Params(tau=(tc, tc), G=p.G), steps, target).imag / H_CS
    v = inputs.uniform_noise(rho0.shape, seed=7)
    cs_r = adjoint.loss(rho0 + 1j * H_CS * v, p, steps, target).imag / H_CS
    assert abs(dG - cs_G) <= 1e-11 * abs(cs_G)
    assert abs(dtau - cs_t) <= 1e-11 * abs(cs_t)
    assert abs(np.sum(drho0 * v) - cs_r) <= 1e-11 * abs(cs_r)


def test_full_sweep_with_walls_against_complex_step():
    shape = (8, 4, 10)
    rho0, solid = inputs.inclined_channel(shape, angle_deg=30.0, radius=3.0, seed=8)
    target = inputs.target_ellipsoid(shape, radius=2.5, seed=9)
    p = Params(tau=(0.9, 0.9), G=((0.0, -1.0), (-1.0, 0.0)), rho_wall=(0.0, 0.1))
    L, dG, dtau, drho0 = adjoint.loss_and_gradient(rho0, p, 8, target, solid)
    v = inputs.uniform_noise(rho0.shape, seed=10)
    v[:, solid] = 0.0
    cs_r = adjoint.loss(rho0 + 1j * H_CS * v, p, 8, target, solid).imag / H_CS
    assert abs(np.sum(drho0 * v) - cs_r) <= 1e-11 * abs(cs_r)
    Gc = -1.0 + 1j * H_CS
    cs_G = adjoint.loss(rho0, Params(tau=p.tau, G=((0.0, Gc), (Gc, 0.0)), rho_wall=p.rho_wall),
                        8, target, solid).imag / H_CS
    assert abs(dG - cs_G) <= 1e-11 * abs(cs_G)


def test_full_sweep_against_central_differences():
    rho0, target, steps = _calibration_case(n=6, steps=10)
    G, tau, h = -1.0, 1.0, 1e-4
    p = Params(tau=(tau, tau), G=((0.0, G), (G, 0.0)))
    _, dG, dtau, _ = adjoint.loss_and_gradient(rho0, p, steps, target)

    def LG(g):
        return adjoint.loss(rho0, Params(tau=(tau, tau), G=((0.0, g), (g, 0.0))), steps, target)

    def Lt(t):
        return adjoint.loss(rho0, Params(tau=(t, t), G=p.G), steps, target)

    fd_G = (LG(G + h) - LG(G - h)) / (2 * h)
    fd_t = (Lt(tau + h) - Lt(tau - h)) / (2 * h)
    assert abs(dG - fd_G) <= 1e-6 * abs(fd_G)
    assert abs(dtau - fd_t) <= 1e-6 * abs(fd_t)


@pytest.mark.parametrize("walls", [False, True])
def test_regularized_full_sweep_against_complex_step(walls):
    """The regularized operator (Sec. 3) over a whole run, unequal tau."""
    shape = (6, 5, 7)
    rho0 = inputs.sphere_droplet(shape, radius=1.8, seed=11)
    solid = None
    if walls:
        solid = np.zeros(shape, bool)
        solid[0] = True
        rho0[:, solid] = 0.0
    target = inputs.target_ellipsoid(shape, radius=1.8, seed=12)
    p = Params(tau=(0.7, 1.1), G=((0.0, -1.2), (-1.2, 0.0)), rho_wall=(0.0, 0.1), collision="regularized")
    steps = 8
    L, dG, dtau, drho0 = adjoint.loss_and_gradient(rho0, p, steps, target, solid)
    assert L > 0
    Gc = -1.2 + 1j * H_CS
    cs_G = adjoint.loss(rho0, Params(tau=p.tau, G=((0.0, Gc), (Gc, 0.0)), rho_wall=p.rho_wall,
                                     collision="regularized"), steps, target, solid).imag / H_CS
    assert abs(dG - cs_G) <= 1e-11 * abs(cs_G)
    v = inputs.uniform_noise(rho0.shape, seed=13)
    if solid is not None:
        v[:, solid] = 0.0
    cs_r = adjoint.loss(rho0 + 1j * H_CS * v, p, steps, target, solid).imag / H_CS
    assert abs(np.sum(drho0 * v) - cs_r) <= 1e-11 * abs(cs_r)

