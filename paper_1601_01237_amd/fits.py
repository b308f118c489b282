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
  (Sec. 4.2.2, :func:`sphere_fit`, :func:`contact_angle`); for a slug between
  plates, a circle fitted to the meniscus in the x-z plane
  (:func:`meniscus_points`, :func:`circle_fit`, :func:`meniscus_angle`);
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


def plane_contact_angle(center, radius, point, normal):
    """Angle inside a droplet between a wall plane (through ``point``, unit
    ``normal`` pointing into the fluid) and the fitted sphere:
    cos(theta) = -d / R with d the signed distance of the centre from the
    plane, in degrees (the flat-wall form of :func:`contact_angle`)."""
    n = np.asarray(normal, dtype=np.float64)
    d = float(np.dot(np.asarray(center, dtype=np.float64) - np.asarray(point, dtype=np.float64), n))
    return math.degrees(math.acos(max(-1.0, min(1.0, -d / radius))))


def drift_velocity(com_a, com_b, steps, lengths=None):
    """|d(com)| / steps between two centres of mass (periodic minimum image if lengths given)."""
    d = np.asarray(com_b, dtype=np.float64) - np.asarray(com_a, dtype=np.float64)
    if lengths is not None:
        d = min_image(d, np.asarray(lengths, dtype=np.float64))
    return float(np.linalg.norm(d)) / steps, d / steps


def circle_fit(points):
    """Algebraic least-squares circle through points (N, 2): returns (centre, radius)."""
    P = np.asarray(points, dtype=np.float64)
    A = np.concatenate([2.0 * P, np.ones((P.shape[0], 1))], axis=1)
    b = np.sum(P * P, axis=1)
    sol, *_ = np.linalg.lstsq(A, b, rcond=None)
    c = sol[:2]
    return c, math.sqrt(sol[2] + float(c @ c))


def meniscus_points(profile, level, x_lo, x_hi, rows):
    """Interface of a slug seen in an x-z section.  ``profile`` is rho_A[z, x];
    for each z in ``rows`` the position x in [x_lo, x_hi) where rho_A crosses
    ``level`` (linear interpolation between the two cells that bracket it).
    Returns an (N, 2) array of (x, z)."""
    pts = []
    for z in rows:
        v = np.asarray(profile[z], dtype=np.float64)
        for x in range(x_lo, x_hi - 1):
            a, b = v[x] - level, v[x + 1] - level
            if a == 0.0:
                pts.append((float(x), float(z)))
                break
            if a * b < 0.0:
                pts.append((x + a / (a - b), float(z)))
                break
    return np.array(pts, dtype=np.float64)


def meniscus_angle(center, radius, z_wall, phase_a_side, x_ref):
    """Contact angle, measured through phase A, between the wall z = z_wall and
    a circular meniscus (centre (x_c, z_c), radius R) that crosses it.
    ``phase_a_side`` is -1 when phase A lies at smaller x than the meniscus,
    +1 when it lies at larger x; ``x_ref`` is a point of the meniscus (e.g.
    the mean x of the fitted points), which picks the crossing on its side of
    the centre.  With t the tangent of the circle at the contact point,
    oriented away from the wall, cos(theta) = t . (phase_a_side, 0)."""
    xc, zc = float(center[0]), float(center[1])
    dz = z_wall - zc
    if abs(dz) >= radius:
        return float("nan")
    side = 1.0 if x_ref >= xc else -1.0
    rx, rz = side * math.sqrt(radius * radius - dz * dz), dz
    away = 1.0 if dz < 0.0 else -1.0  # into the fluid, away from the wall
    tx, tz = -rz, rx
    if tz * away < 0.0:
        tx, tz = -tx, -tz
    c = (tx * phase_a_side) / radius
    return math.degrees(math.acos(max(-1.0, min(1.0, c))))
