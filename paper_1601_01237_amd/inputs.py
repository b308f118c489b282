"""Seeded synthetic inputs for the two-component D3Q19 lattice Boltzmann step.

This module only builds initial density fields, solid masks and target shapes
from a seed.  It contains none of the lattice Boltzmann arithmetic, so both the
FP64 CPU oracle and the HIP path can be fed the same arrays.

Array conventions (shared by every producer and consumer of these arrays):

* grid shape is ``(nz, ny, nx)``; ``x`` is the fastest index (C order);
* a density field ``rho0`` has shape ``(2, nz, ny, nx)``, float64, species
  A = index 0 (the droplet phase) and species B = index 1;
* a solid mask has shape ``(nz, ny, nx)``, ``bool``; ``True`` marks a wall cell.

The paper runs its droplet tests with a density of 0.22 per component in 2-D
(Sec. 3); the 3-D workloads here use 1.0 inside / 0.03 outside for the droplet
species, mirrored for the other species, plus uniform noise of +-1e-3 per
species and cell.  Random numbers come from ``numpy.random.default_rng(seed)``
(PCG64) and are drawn in a fixed order: droplet parameters first, then the
noise of species A, then the noise of species B, each in C order (z, y, x).
"""

from __future__ import annotations

import math

import numpy as np

RHO_IN = 1.0
RHO_OUT = 0.03
NOISE = 1.0e-3


def _grid(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64),
                          np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def _min_image(d, n):
    """Minimum-image displacement on a periodic axis of length n."""
    return d - n * np.round(d / n)


def _periodic_dist2(shape, center):
    nz, ny, nx = shape
    x, y, z = _grid(shape)
    dx = _min_image(x - center[0], nx)
    dy = _min_image(y - center[1], ny)
    dz = _min_image(z - center[2], nz)
    return dx * dx + dy * dy + dz * dz


def _two_species(inside, rng, noise=NOISE):
    rho_a = np.where(inside, RHO_IN, RHO_OUT)
    rho_b = np.where(inside, RHO_OUT, RHO_IN)
    shape = inside.shape
    if noise:
        rho_a = rho_a + rng.uniform(-noise, noise, size=shape)
        rho_b = rho_b + rng.uniform(-noise, noise, size=shape)
    return np.stack([rho_a, rho_b]).astype(np.float64)


def sphere_droplet(shape, radius, seed=0, center=None, noise=NOISE, width=0.0):
    """One spherical droplet of species A in a periodic box.

    A cell (integer centre) is inside iff its minimum-image squared distance to
    ``center`` is below ``radius**2``.  ``center`` defaults to
    ``(nx/2, ny/2, nz/2)`` given as (x, y, z).  With ``width`` > 0 the
    interface is the profile 1/2 (1 - tanh((r - R) / width)) between the two
    phase densities instead of a step.  Returns ``rho0`` ``(2, nz, ny, nx)``
    float64.
    """
    nz, ny, nx = shape
    if center is None:
        center = (nx / 2.0, ny / 2.0, nz / 2.0)
    rng = np.random.default_rng(seed)
    d2 = _periodic_dist2(shape, center)
    if width <= 0.0:
        return _two_species(d2 < radius * radius, rng, noise)
    frac = 0.5 * (1.0 - np.tanh((np.sqrt(d2) - radius) / width))
    rho_a = RHO_OUT + (RHO_IN - RHO_OUT) * frac
    rho_b = RHO_IN - (RHO_IN - RHO_OUT) * frac
    if noise:
        rho_a = rho_a + rng.uniform(-noise, noise, size=shape)
        rho_b = rho_b + rng.uniform(-noise, noise, size=shape)
    return np.stack([rho_a, rho_b]).astype(np.float64)


def random_droplets(shape, count=64, rmin=8.0, rmax=24.0, seed=0, noise=NOISE):
    """Union of ``count`` spheres with centres U[0, n) per axis and radii U[rmin, rmax].

    Centres are drawn first (count x 3, columns x, y, z), then radii, then the
    noise of species A and B.  Periodic minimum-image distances.
    """
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    centers = rng.uniform(0.0, 1.0, size=(count, 3)) * np.array([nx, ny, nz], dtype=np.float64)
    radii = rng.uniform(rmin, rmax, size=count)
    inside = np.zeros(shape, dtype=bool)
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    z = np.arange(nz, dtype=np.float64)
    for (cx, cy, cz), r in zip(centers, radii):
        # Work on the bounding box only (wrapped), so 512^3 stays cheap.
        dz = _min_image(z - cz, nz)
        dy = _min_image(y - cy, ny)
        dx = _min_image(x - cx, nx)
        kz = np.nonzero(np.abs(dz) < r)[0]
        ky = np.nonzero(np.abs(dy) < r)[0]
        kx = np.nonzero(np.abs(dx) < r)[0]
        if kz.size == 0 or ky.size == 0 or kx.size == 0:
            continue
        d2 = (dz[kz][:, None, None] ** 2 + dy[ky][None, :, None] ** 2
              + dx[kx][None, None, :] ** 2)
        sub = inside[np.ix_(kz, ky, kx)]
        inside[np.ix_(kz, ky, kx)] = sub | (d2 < r * r)
    return _two_species(inside, rng, noise), centers, radii


def inclined_channel(shape, angle_deg=30.0, radius=32.0, seed=0, noise=NOISE):
    """Channel with walls on z = 0 and z = nz-1 plus a plane inclined in x-z.

    The plane passes through (x, z) = (nx/2, nz/3) with unit normal
    (-sin a, 0, cos a); cells strictly below it are solid.  x and y are
    periodic.  A sphere of species A with radius ``radius`` centred on the plane
    at (nx/2, ny/2, nz/3) sits on the wall (a hemispherical cap in the fluid).
    Returns ``(rho0, solid)``; ``rho0`` is zero on solid cells.
    """
    nz, ny, nx = shape
    a = math.radians(angle_deg)
    x, y, z = _grid(shape)
    xc, zc = nx / 2.0, nz / 3.0
    below = (-(x - xc) * math.sin(a) + (z - zc) * math.cos(a)) < 0.0
    solid = below.copy()
    solid[0] = True
    solid[nz - 1] = True
    rng = np.random.default_rng(seed)
    d2 = (x - xc) ** 2 + (y - ny / 2.0) ** 2 + (z - zc) ** 2
    inside = d2 < radius * radius
    rho0 = _two_species(inside, rng, noise)
    rho0[:, solid] = 0.0
    return rho0, solid


def flat_channel(shape, seed=0, noise=NOISE, radius=None):
    """Walls on z = 0 and z = nz-1 only, optional hemispherical droplet on z = 1."""
    nz, ny, nx = shape
    solid = np.zeros(shape, dtype=bool)
    solid[0] = True
    solid[nz - 1] = True
    rng = np.random.default_rng(seed)
    if radius is None:
        inside = np.zeros(shape, dtype=bool)
    else:
        x, y, z = _grid(shape)
        inside = (x - nx / 2.0) ** 2 + (y - ny / 2.0) ** 2 + (z - 0.5) ** 2 < radius * radius
    rho0 = _two_species(inside, rng, noise)
    rho0[:, solid] = 0.0
    return rho0, solid


def slug_channel(shape, x0, x1, seed=0, noise=NOISE):
    """Walls on z = 0 and z = nz-1; species A fills the slab x0 <= x < x1 of
    the fluid between them (a slug across the channel), species B the rest.
    Returns ``(rho0, solid)``; ``rho0`` is zero on solid cells."""
    nz, ny, nx = shape
    solid = np.zeros(shape, dtype=bool)
    solid[0] = True
    solid[nz - 1] = True
    rng = np.random.default_rng(seed)
    x, _, _ = _grid(shape)
    inside = (x >= x0) & (x < x1)
    rho0 = _two_species(inside, rng, noise)
    rho0[:, solid] = 0.0
    return rho0, solid


def target_ellipsoid(shape, radius, seed=0):
    """Target density of species A for the calibration objective.

    Axis-aligned ellipsoid, semi-axes ``radius * (1 + 0.2 U(-1, 1))`` (x, y, z
    drawn in that order) and centre ``(n/2) + U(-2, 2)`` per axis; 1.0 inside,
    0.03 outside.  Returns ``(nz, ny, nx)`` float64.
    """
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    semi = radius * (1.0 + 0.2 * rng.uniform(-1.0, 1.0, size=3))
    off = rng.uniform(-2.0, 2.0, size=3)
    x, y, z = _grid(shape)
    dx = _min_image(x - (nx / 2.0 + off[0]), nx) / semi[0]
    dy = _min_image(y - (ny / 2.0 + off[1]), ny) / semi[1]
    dz = _min_image(z - (nz / 2.0 + off[2]), nz) / semi[2]
    inside = dx * dx + dy * dy + dz * dz < 1.0
    return np.where(inside, RHO_IN, RHO_OUT).astype(np.float64)


def uniform_noise(shape, seed=0, scale=1.0):
    """Plain U(-scale, scale) array of the given shape (for perturbation directions)."""
    return np.random.default_rng(seed).uniform(-scale, scale, size=shape)


def droplet_radius_for_box(n):
    """Radius used for a box of side ``n`` when a workload is scaled down (R/N = 1/4)."""
    return n / 4.0
