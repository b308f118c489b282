"""Pins of the oracle's global diagnostics on states with known answers."""

import numpy as np

from oracle import diagnostics as D
from oracle import lbm
from paper_1601_01237_amd import inputs


def test_rest_droplet_diagnostics():
    n = 16
    rho0 = inputs.sphere_droplet((n, n, n), radius=4.0, seed=0, noise=0.0)
    f = lbm.init_state(rho0)
    p = lbm.Params(tau=(1.0, 1.0), G=((0.0, -2.0), (-2.0, 0.0)))
    d = D.diagnostics(f, p, center=(8.0, 8.0, 8.0), r_in=2.0, r_out=6.0, thr=0.515)
    inside = rho0[0] > 0.5
    assert abs(d[D.MASS_A] - np.sum(rho0[0])) < 1e-12 * np.sum(rho0[0])
    assert abs(d[D.MASS_B] - np.sum(rho0[1])) < 1e-12 * np.sum(rho0[1])
    assert d[D.N_FLUID] == n ** 3
    assert d[D.NONFINITE] == 0
    assert d[D.N_THR] == np.count_nonzero(inside)
    # symmetric sphere about its centre: the offsets of the selected cells cancel
    assert abs(d[D.SDX_THR]) < 1e-12 and abs(d[D.SDY_THR]) < 1e-12 and abs(d[D.SDZ_THR]) < 1e-12
    # pure phases: p = T0 (1 + 0.03) - G T0 * 0.03 both inside and outside
    pin = d[D.P_IN_SUM] / d[D.N_IN]
    pout = d[D.P_OUT_SUM] / d[D.N_OUT]
    want = lbm.T0 * 1.03 + 2.0 * lbm.T0 * 0.03
    assert abs(pin - want) < 1e-14 and abs(pout - want) < 1e-14
    # cells with |x - c|^2 < 4: squared norms 0, 1, 2, 3 -> 1 + 6 + 12 + 8 lattice points
    assert d[D.N_IN] == 27


def test_centre_of_mass_follows_a_shift_across_the_periodic_boundary():
    n = 12
    rho0 = inputs.sphere_droplet((n, n, n), radius=3.0, seed=0, noise=0.0,
                                 center=(11.0, 6.0, 6.0))
    f = lbm.init_state(rho0)
    p = lbm.Params()
    d = D.diagnostics(f, p, center=(10.0, 6.0, 6.0))
    # droplet centred at x = 11 seen from x = 10 across the wrap: mean offset +1
    assert abs(d[D.SDX_THR] / d[D.N_THR] - 1.0) < 1e-12


def test_divergent_run_is_flagged():
    """tau just above 1/2 with a strongly supercritical coupling diverges; the
    non-finite count of the diagnostics (what the GPU wrapper checks) flags
    it within a few tens of steps, and a stable run never does."""
    import warnings
    shape = (12, 12, 12)
    rho0 = inputs.sphere_droplet(shape, radius=4.0, seed=0)
    for tau, G, diverges in ((0.51, -3.0, True), (1.0, -1.0, False)):
        p = lbm.Params(tau=(tau, tau), G=((0.0, G), (G, 0.0)))
        f = lbm.init_state(rho0)
        flagged = None
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", RuntimeWarning)
            for t in range(1, 41):
                f = lbm.step(f, p)
                if D.diagnostics(f, p)[D.NONFINITE] > 0:
                    flagged = t
                    break
        assert (flagged is not None) == diverges, (tau, G, flagged)
