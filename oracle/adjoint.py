"""FP64 CPU oracle: adjoint of the two-component D3Q19 step (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may use this module.  It is the transpose, written out by hand, of the
forward map in :mod:`oracle.lbm` (Sec. 2, Eqs. 1-9 of arXiv 1601.01237 with the
exact-difference forcing reading), checked in the tests against complex-step
derivatives of that forward map.

With omega_a = 1 / tau_a, v^a = u + g^a and E_i(rho, v) = w_i rho P_i(v) the
collision of Eqs. (1)-(2) is

    f*_i^a = (1 - omega_a) f_i^a + (omega_a - 1) E_i(rho^a, u) + E_i(rho^a, v^a)

where rho^a = sum_i f_i^a, u = j / rho and g^a = sum_b G^{ab} S^b with
S^b(x) = sum_i w_i c_i rho~^b(x + c_i) (Eq. 7 divided by rho^a).  Given
lam*_i^a = dL / df*_i^a the local pullback is

    rho_bar^a = sum_i lam*_i^a w_i [(omega_a - 1) P_i(u) + P_i(v^a)]
    u_bar     = sum_a rho^a sum_i lam*_i^a w_i [(omega_a - 1) dP_i(u) + dP_i(v^a)]
    g_bar^a   = rho^a sum_i lam*_i^a w_i dP_i(v^a)
    lam_k^a   = (1 - omega_a) lam*_k^a + rho_bar^a + u_bar . (c_k - u) / rho

and the Eq. (7) gather becomes a gather of S_bar^b = sum_a G^{ab} g_bar^a from
the neighbours x - c_i:  lam_k^b(x) += sum_i w_i c_i . S_bar^b(x - c_i) on
fluid x (a solid neighbour holds the constant rho_s and passes nothing back).
Parameters: dL/dG^{ab} = sum_x g_bar^a . S^b and
dL/dtau_a = sum_x sum_i lam*_i^a (f_i^a - E_i(rho^a, u)) / tau_a^2.

With the regularized operator (Sec. 3, Eqs. 10-11, read as the
second-order Hermite projection) the collision is

    f*_i^a = E_i(rho^a, v^a) + (1 - omega_a) N_i^a,
    N_i^a  = w_i (c_i c_i - T0 I) : Pi^a / (2 T0^2),
    Pi^a   = sum_j c_j c_j (f_j^a - E_j(rho^a, u)).

With Pi_bar^a = (1 - omega_a) sum_i lam*_i^a w_i (c_i c_i - T0 I) / (2 T0^2)
the pullback through Pi^a is dL = Pi_bar^a : dPi^a, so the terms above keep
their form with two substitutions: the population that multiplies
E_j(rho^a, u) is mu_j^a = -c_j c_j : Pi_bar^a instead of
(omega_a - 1) lam*_j^a, and the direct term of lam_k^a is c_k c_k : Pi_bar^a
instead of (1 - omega_a) lam*_k^a.  dL/dtau_a = sum_x sum_i lam*_i^a N_i^a /
tau_a^2.  The third-order reading adds w_i H_i . q^a / N to N_i^a (energy-flux
polynomials H, their norm N, q^a = sum_j H_j (f_j^a - E_j(rho^a, u))), which
is linear in f - E(rho, u) as Pi^a is: with q_bar^a = (1 - omega_a) sum_i
lam*_i^a w_i H_i / N, mu_j^a gains -H_j . q_bar^a and the direct term
H_k . q_bar^a.  All three operators are written below with mu:

    rho_bar^a = sum_i w_i [mu_i^a P_i(u) + lam*_i^a P_i(v^a)]
    u_bar     = sum_a rho^a sum_i w_i [mu_i^a dP_i(u) + lam*_i^a dP_i(v^a)]
    lam_k^a   = -mu_k^a + rho_bar^a + u_bar . (c_k - u) / rho

Streaming (push with bounce-back) is a permutation; its transpose reads
lam*_i(x) = lam_i(x + c_i) when x + c_i is fluid and lam_{opp(i)}(x) otherwise.
"""

from __future__ import annotations

import numpy as np

from . import lbm
from .lbm import C, OPP, Q, T0, W, Params


def _bracket(cu, uu):
    """The bracket of Eq. (3): P(v) at c.v = cu, v.v = uu."""
    return (1.0 + cu / T0 + cu ** 2 / (2.0 * T0 ** 2) - uu / (2.0 * T0)
            + cu ** 3 / (6.0 * T0 ** 3) - cu * uu / (2.0 * T0 ** 2))


def _bracket_grad(c, v):
    """dP/dv of the bracket of Eq. (3), as a (3, ...) array."""
    cu = c[0] * v[0] + c[1] * v[1] + c[2] * v[2]
    uu = v[0] * v[0] + v[1] * v[1] + v[2] * v[2]
    out = np.empty((3,) + np.shape(cu), dtype=np.result_type(v))
    for a in range(3):
        out[a] = (c[a] / T0 + cu * c[a] / T0 ** 2 - v[a] / T0
                  + cu ** 2 * c[a] / (2.0 * T0 ** 3)
                  - (c[a] * uu + 2.0 * cu * v[a]) / (2.0 * T0 ** 2))
    return out


def stream_adjoint(lam, solid=None):
    """Transpose of :func:`oracle.lbm.stream`."""
    fluid = lbm.fluid_mask(lam.shape[2:], solid)
    out = np.zeros_like(lam)
    for i in range(Q):
        target_fluid = lbm.at_offset(fluid, C[i])
        go = fluid & target_fluid
        back = fluid & ~target_fluid
        out[:, i] = (np.where(go, lbm.at_offset(lam[:, i], C[i]), 0.0)
                     + np.where(back, lam[:, OPP[i]], 0.0))
    return out


def _projection_weights(lam_a, omega, order=2):
    """mu_j = -c_j c_j : Pi_bar of the regularized operator, with
    Pi_bar = (1 - omega) sum_i lam_i w_i (c_i c_i - T0 I) / (2 T0^2); with
    the third-order reading also -H_j . q_bar, where H are the energy-flux
    polynomials of :func:`oracle.lbm.energy_flux_hermite`, N their norm and
    q_bar = (1 - omega) sum_i lam_i w_i H_i / N (the pullback through the
    coefficients q = sum_j H_j (f_j - E_j))."""
    shape = lam_a.shape[1:]
    pbar = np.zeros((3, 3) + shape, dtype=lam_a.dtype)
    for i in range(Q):
        for a in range(3):
            for b in range(3):
                h = C[i, a] * C[i, b] - (T0 if a == b else 0.0)
                if h != 0.0:
                    pbar[a, b] = pbar[a, b] + lam_a[i] * W[i] * h
    pbar = pbar * ((1.0 - omega) / (2.0 * T0 * T0))
    mu = np.empty_like(lam_a)
    for j in range(Q):
        mu[j] = -sum(C[j, a] * C[j, b] * pbar[a, b] for a in range(3) for b in range(3))
    if order == 3:
        he = lbm.energy_flux_hermite()
        norm = float(np.sum(W * he[:, 0] ** 2))
        qbar = [(1.0 - omega) / norm * sum(lam_a[i] * W[i] * he[i, a] for i in range(Q) if he[i, a] != 0.0)
                for a in range(3)]
        for j in range(Q):
            mu[j] = mu[j] - sum(he[j, a] * qbar[a] for a in range(3) if he[j, a] != 0.0)
    elif order != 2:
        raise ValueError(order)
    return mu


def collide_adjoint(f, lam_star, p: Params, solid=None):
    """Transpose of :func:`oracle.lbm.collide` at state ``f`` (BGK or the
    regularized collision, second- or third-order reading).

    Returns ``(lam, dG, dtau)``: lam = dL/df (same shape as f), dG a (2, 2)
    array of dL/dG^{ab} and dtau a length-2 array of dL/dtau_a.
    """
    if p.collision not in ("bgk", "regularized", "regularized3"):
        raise ValueError(p.collision)
    order = 3 if p.collision == "regularized3" else 2
    m = lbm.macroscopic(f, p, solid)
    fluid, rho_s, rho, u = m["fluid"], m["rho_s"], m["rho"], m["u"]
    shape = f.shape[2:]
    sums = [lbm.neighbour_sum(rho_s[b], fluid, p.rho_wall[b]) for b in range(2)]
    g = m["g"]
    dtype = np.result_type(f, lam_star, np.asarray(p.tau).dtype)

    rho_bar = np.zeros((2,) + shape, dtype=dtype)
    u_bar = np.zeros((3,) + shape, dtype=dtype)
    g_bar = np.zeros((2, 3) + shape, dtype=dtype)
    mu = np.zeros((2, Q) + shape, dtype=dtype)
    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    dtau = np.zeros(2, dtype=dtype)
    for a in range(2):
        omega = 1.0 / p.tau[a]
        v = u + g[a]
        vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2]
        if p.collision == "bgk":
            mu[a] = (omega - 1.0) * lam_star[a]
            part = f[a] - lbm.equilibrium(rho_s[a], u)        # df*/dtau = (f - E) / tau^2
        else:
            mu[a] = _projection_weights(lam_star[a], omega, order)
            part = lbm.regularized_neq(f[a], rho_s[a], u, order)  # df*/dtau = N / tau^2
        for i in range(Q):
            ci = C[i]
            cu = ci[0] * u[0] + ci[1] * u[1] + ci[2] * u[2]
            cv = ci[0] * v[0] + ci[1] * v[1] + ci[2] * v[2]
            lw = lam_star[a, i] * W[i]
            mw = mu[a, i] * W[i]
            rho_bar[a] += mw * _bracket(cu, uu) + lw * _bracket(cv, vv)
            dpu = _bracket_grad(ci, u)
            dpv = _bracket_grad(ci, v)
            u_bar += rho_s[a] * (mw * dpu + lw * dpv)
            g_bar[a] += rho_s[a] * lw * dpv
        dtau[a] = np.sum(np.where(fluid, lam_star[a] * part, 0.0)) / p.tau[a] ** 2

    rho_bar = np.where(fluid, rho_bar, 0.0)
    u_bar = np.where(fluid, u_bar, 0.0)
    g_bar = np.where(fluid, g_bar, 0.0)
    rho_safe = np.where(fluid, rho, 1.0)

    lam = np.zeros(f.shape, dtype=dtype)
    for a in range(2):
        for k in range(Q):
            ck = C[k]
            proj = (u_bar[0] * (ck[0] - u[0]) + u_bar[1] * (ck[1] - u[1])
                    + u_bar[2] * (ck[2] - u[2])) / rho_safe
            lam[a, k] = -mu[a, k] + rho_bar[a] + proj

    # Transpose of the Eq. (7) neighbour gather.
    dG = np.zeros((2, 2), dtype=dtype)
    for b in range(2):
        s_bar = np.zeros((3,) + shape, dtype=dtype)
        for a in range(2):
            if p.G[a][b] != 0:
                s_bar = s_bar + p.G[a][b] * g_bar[a]
                dG[a, b] = np.sum(g_bar[a] * sums[b])
        r = np.zeros(shape, dtype=dtype)
        for i in range(1, Q):
            ci = C[i]
            back = lbm.at_offset(s_bar, -ci)          # S_bar^b(x - c_i)
            r = r + W[i] * (ci[0] * back[0] + ci[1] * back[1] + ci[2] * back[2])
        lam[b] = lam[b] + np.where(fluid, r, 0.0)[None]

    lam = np.where(fluid[None, None], lam, 0.0)
    return lam, dG, dtau


def step_adjoint(f_t, lam_next, p: Params, solid=None):
    """dL/df_t from dL/df_{t+1} for one step f_{t+1} = stream(collide(f_t))."""
    return collide_adjoint(f_t, stream_adjoint(lam_next, solid), p, solid)


def shape_loss(rho_a, rho_target, fluid):
    """L = 1/2 sum_x (rho^A(x, T) - rho_target(x))^2 over fluid cells."""
    d = np.where(fluid, rho_a - rho_target, 0.0)
    return 0.5 * np.sum(d * d)


def loss_and_gradient(rho0, p: Params, steps, rho_target, solid=None):
    """Calibration objective and its gradient, by a full reverse sweep.

    Forward: f_0 = init_state(rho0), f_{t+1} = step(f_t), L = shape_loss.
    Returns ``(L, dL_dG_tied, dL_dtau_tied, dL_drho0)`` where the tied
    derivatives assume G^{AB} = G^{BA} and tau_A = tau_B.
    """
    f = lbm.init_state(rho0, solid)
    fluid = lbm.fluid_mask(rho0.shape[1:], solid)
    states = [f]
    for _ in range(steps):
        f = lbm.step(f, p, solid)
        states.append(f)
    rho_a = lbm.species_density(f)[0]
    L = shape_loss(rho_a, rho_target, fluid)

    lam = np.zeros(f.shape, dtype=np.result_type(f, rho_target))
    lam[0] = np.where(fluid, rho_a - rho_target, 0.0)[None]
    dG = np.zeros((2, 2))
    dtau = np.zeros(2)
    for t in range(steps - 1, -1, -1):
        lam, dG_t, dtau_t = step_adjoint(states[t], lam, p, solid)
        dG = dG + dG_t
        dtau = dtau + dtau_t
    drho0 = np.einsum("i,aizyx->azyx", W, lam)
    return L, dG[0, 1] + dG[1, 0], dtau[0] + dtau[1], drho0


def loss(rho0, p: Params, steps, rho_target, solid=None):
    """Forward-only objective (works in complex128 for complex-step checks)."""
    f = lbm.run(lbm.init_state(rho0, solid), p, steps, solid)
    fluid = lbm.fluid_mask(rho0.shape[1:], solid)
    return shape_loss(lbm.species_density(f)[0], rho_target, fluid)
