"""Host-side fits against closed forms (no GPU)."""

import math

import numpy as np

from paper_1601_01237_amd import fits


def test_laplace_fit_recovers_exact_line():
    R = np.array([8.0, 12.0, 16.0, 24.0])
    sigma = 0.037
    dp = 2 * sigma / R + 1e-4
    s, a, b, r2 = fits.laplace_fit(R, dp)
    assert abs(s - sigma) < 1e-12 and abs(b - 1e-4) < 1e-12 and r2 > 1 - 1e-12


def test_equivalent_radius_of_exact_sphere_volume():
    R = 10.0
    N = 64 ** 3
    vol = 4.0 / 3.0 * math.pi * R ** 3
    mass = 1.2 * vol + 0.05 * (N - vol)
    assert abs(fits.equivalent_radius(mass, N, 1.2, 0.05) - R) < 1e-12


def test_tanh_radius_of_synthetic_profile():
    shape = (40, 40, 40)
    center = (20.3, 19.7, 20.1)
    r = fits.radial_coordinate(shape, center)
    rho = 0.5 - 0.45 * np.tanh((r - 9.3) / 1.7)
    R, _ = fits.tanh_radius(rho, center)
    assert abs(R - 9.3) < 1e-6


def test_sphere_fit_and_contact_angle():
    rng = np.random.default_rng(0)
    c = np.array([30.0, 31.0, 5.5])
    rad = 12.0
    v = rng.normal(size=(500, 3))
    pts = c + rad * v / np.linalg.norm(v, axis=1, keepdims=True)
    cc, rr = fits.sphere_fit(pts)
    assert np.allclose(cc, c, atol=1e-9) and abs(rr - rad) < 1e-9
    # wall at the centre height: hemisphere, 90 degrees
    assert abs(fits.contact_angle(cc, rr, 5.5) - 90.0) < 1e-6
    # wall below the centre: more than a hemisphere sits above it
    theta = fits.contact_angle(cc, rr, 5.5 - 6.0)
    assert abs(theta - math.degrees(math.acos(-0.5))) < 1e-6


def test_drift_velocity_wraps_periodically():
    v, d = fits.drift_velocity([1.0, 5.0, 2.0], [99.0, 5.0, 2.0], 10, lengths=(100.0, 100.0, 50.0))
    assert abs(v - 0.2) < 1e-12 and abs(d[0] + 0.2) < 1e-12


def test_wall_potential_parameterisation():
    from paper_1601_01237_amd.experiments import wall_potential
    assert wall_potential(0.0, 0.22) == (0.0, 0.0)
    a, b = wall_potential(0.4, 0.22)
    assert abs(a - 0.088) < 1e-15 and b == 0.0          # the paper's 40-degree slug value
    a, b = wall_potential(-0.5, 1.0)
    assert a == 0.0 and b == 0.5


def test_meniscus_angle_of_synthetic_arcs():
    """Circular menisci spanning a channel of height 32 (walls at z = 0.5 and
    32.5) drawn for a given contact angle through phase A, on either side of
    the slug, are measured back at that angle."""
    import math
    from paper_1601_01237_amd import fits
    zc, half = 16.5, 16.0
    zs = np.arange(2.0, 31.0)
    for theta in (25.0, 40.0, 75.0, 110.0, 140.0):
        t = math.radians(theta)
        R = half / abs(math.cos(t))
        sgn = 1.0 if theta > 90.0 else -1.0  # A at smaller x: bulges into B when non-wetting
        xc = 64.0 - sgn * R * math.sin(t)
        xs = xc + sgn * np.sqrt(R * R - (zs - zc) ** 2)
        for side, x in ((-1, xs), (+1, 128.0 - xs)):  # the mirror meniscus has A on its right
            # sub-cell crossings of a smooth profile recover the points
            prof = np.array([[0.5 + side * 0.5 * math.tanh(xx - xz) for xx in range(128)] for xz in x])
            pts = fits.meniscus_points(np.concatenate([np.zeros((2, 128)), prof]), 0.5, 0, 128,
                                       range(2, 2 + len(zs)))
            pts[:, 1] = zs
            c, r = fits.circle_fit(pts)
            for zw in (0.5, 32.5):
                got = fits.meniscus_angle(c, r, zw, side, float(pts[:, 0].mean()))
                assert abs(got - theta) < 0.5, (theta, side, zw, got)
