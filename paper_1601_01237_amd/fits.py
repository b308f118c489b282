"""Host-side fits of reduced droplet diagnostics (post-processing, FP64 NumPy).

These turn the fields and FP64 sums that liblbm.so returns into the
measurements of arXiv 1601.01237:

* Young-Laplace law (Eq. 12): the paper's 2-D form is dP = sigma / R; for
  spheres the same law reads dP = 2 sigma / R, so sigma is half the slope of
  dP against 1/R (:func:`laplace_fit`);
* droplet radius from a hyperbolic-tangent fit of the density profile
  (Sec. 3, :func:`tanh_radius`) or from the volume of the droplet phase
  (:func:`equivalent_radius`);
* static contact angle from a circle (here: sphere) fitted to the interface
  (Sec. 4.2.2, :func:`sphere_fit`, :func:`contact_angle`);
* droplet drift velocity from the change of the droplet's centre of mass
  between two times (Sec. 4.2.3, :func:`drift_velocity`).

Bulk pressure of the two-component mixture (leading-order continuum form of
Eq. 7, a reading: the paper prints no pressure formula):
p = T0 (rho^A + rho^B) - G T0 rho^A rho^B with T0 = 1/3.
"""

from __future__ import annotations

import math

import numpy as np

T0 = 1.0 / 3.0


def pressure(rho_a, rho_b, G):
    return T0 * (rho_a + rho_b) - G * T0 * rho_a * rho_b


def laplace_fit(radius, dp):
    """Least-squares line dP = a (1/R) + b.  Returns (sigma, a, b, r2) with sigma = a / 2."""
    x = 1.0 / np.asarray(radius, dtype=np.float64)
    y = np.asarray(dp, dtype=np.float64)
    A = np.stack([x, np.ones_like(x)], axis=1)
    (a, b), *_ = np.linalg.lstsq(A, y, rcond=None)
    pred = a * x + b
    ss_res = float(np.sum((y - pred) ** 2))
    ss_tot = float(np.sum((y - y.mean()) ** 2))
    r2 = 1.0 - ss_res / ss_tot if ss_tot > 0 else 1.0
    return 0.5 * a, a, b, r2


def equivalent_radius(mass_a, n_cells, rho_in, rho_out):
    """Radius of the sphere holding the droplet phase of species A.

    V = (M_A - rho_out N) / (rho_in - rho_out), R = (3 V / 4 pi)^(1/3).
    """
    vol = (mass_a - rho_out * n_cells) / (rho_in - rho_out)
    return (3.0 * vol / (4.0 * math.pi)) ** (1.0 / 3.0)


def min_image(d, n):
    return d - n * np.round(d / n)


def radial_coordinate(shape, center):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=float), np.arange(ny, dtype=float),
                          np.arange(nx, dtype=float), indexing="ij")
    dx = min_image(x - center[0], nx)
    dy = min_image(y - center[1], ny)
    dz = min_image(z - center[2], nz)
    return np.sqrt(dx * dx + dy * dy + dz * dz)


def tanh_radius(rho_a, center, r_max=None):
    """R from a least-squares fit of rho(r) = a - b tanh((r - R) / w) to all cells."""
    from scipy.optimize import curve_fit
    r = radial_coordinate(rho_a.shape, center).ravel()
    v = np.asarray(rho_a, dtype=np.float64).ravel()
    if r_max is not None:
        keep = r < r_max
        r, v = r[keep], v[keep]
    hi, lo = float(v.max()), float(v.min())
    r0 = float(np.sqrt(np.mean(r[v > 0.5 * (hi + lo)] ** 2) * 5.0 / 3.0)) if np.any(v > 0.5 * (hi + lo)) else 1.0

    def model(rr, a, b, R, w):
        return a - b * np.tanh((rr - R) / w)

    p0 = (0.5 * (hi + lo), 0.5 * (hi - lo), r0, 1.5)
    popt, _ = curve_fit(model, r, v, p0=p0, maxfev=20000)
    return float(popt[2]), popt


def sphere_fit(points):
    """Algebraic least-squares sphere through points (N, 3): returns (centre, radius)."""
    P = np.asarray(points, dtype=np.float64)
    A = np.concatenate([2.0 * P, np.ones((P.shape[0], 1))], axis=1)
    b = np.sum(P * P, axis=1)
    sol, *_ = np.linalg.lstsq(A, b, rcond=None)
    c = sol[:3]
    radius = math.sqrt(sol[3] + float(c @ c))
    return c, radius


def interface_points(rho_a, fluid, level, band):
    """Coordinates (x, y, z) of fluid cells with |rho_A - level| < band."""
    sel = fluid & (np.abs(rho_a - level) < band)
    z, y, x = np.nonzero(sel)
    return np.stack([x, y, z], axis=1).astype(np.float64)


def contact_angle(center, radius, wall_height):
    """Angle inside the droplet between the wall (plane z = wall_height) and the
    fitted sphere: cos(theta) = (wall_height - z_c) / R, in degrees."""
    c = np.clip((wall_height - center[2]) / radius, -1.0, 1.0)
    return math.degrees(math.acos(c))


def drift_velocity(com_a, com_b, steps, lengths=None):
    """|d(com)| / steps between two centres of mass (periodic minimum image if lengths given)."""
    d = np.asarray(com_b, dtype=np.float64) - np.asarray(com_a, dtype=np.float64)
    if lengths is not None:
        d = min_image(d, np.asarray(lengths, dtype=np.float64))
    return float(np.linalg.norm(d)) / steps, d / steps
